// prep.hip -- row preparation: L2 normalisation fused with the narrow-format
// rounding and K padding of the operand copies.
//
// The tensor join computes cosine similarity as the dot product of
// L2-normalised rows (Section IV.C).  This pass reads each input row once,
// finds its norm, and writes the normalised row in the contraction format
// (float32, bfloat16 or OCP e4m3 with a per-row power-of-two scale), zero
// padded to the contraction depth Kp and to a whole number of row tiles, so
// that the matrix-core kernel runs without bounds checks or per-element
// scaling.  It also records per-row data used by the error bounds.
#include "common.hpp"
#include "batch.hpp"
#include "launch.hpp"

namespace ej {

// Prepare input row `src` into output row `row` (one wave; src >= rows is
// tile padding, written as zeros).  Returns the row's quantisation error
// norm (0 for FP32).
template <int PREC>
__device__ __forceinline__ float prep_one_row(const float* __restrict__ X, int64_t rows, int dim,
                                              int64_t ld, void* __restrict__ Xq, int Kp,
                                              RowInfo* __restrict__ info,
                                              unsigned long long* __restrict__ hdr, int64_t row,
                                              int64_t src, int lane, int real_ = -1) {
    float inv = 0.0f, qscale = 1.0f, enorm = 0.0f;
    uint32_t flags = 0;
    const float* x = X + src * ld;
    const bool real = real_ < 0 ? src < rows : real_ != 0;

    if (real) {
        // pass 1: finiteness and max |x|
        float amax = 0.0f;
        bool bad = false;
        for (int k = lane; k < dim; k += 64) {
            float v = x[k];
            bad |= !isfinite(v);
            amax = fmaxf(amax, fabsf(v));
        }
        bad = __any(bad);
        amax = wave_max(amax);
        if (bad) {
            flags = F_NONFINITE;
        } else if (amax > 0.0f) {
            // pass 2: sum of squares of the row scaled by a power of two so
            // that max |x| lands in [1, 2): no overflow or underflow
            int e = ilogbf(amax);
            float sc = ldexpf(1.0f, -e);
            float ss = 0.0f;
            for (int k = lane; k < dim; k += 64) {
                float v = x[k] * sc;
                ss = fmaf(v, v, ss);
            }
            ss = wave_sum(ss);
            // ||x|| = sqrt(ss) * 2^e with sqrt(ss) in [1, 2 sqrt(dim))
            if (e < -100 || e > 99) {
                flags = F_RANGE;
            } else {
                inv = ldexpf(1.0f / sqrtf(ss), -e);
            }
        }
    }
    if (flags != 0 && lane == 0) atomicOr(hdr + H_FLAGS, (unsigned long long)flags);

    // FP8: choose the largest power of two p with max|x_hat| * 2^p <= 448
    if (PREC == P_FP8 && inv != 0.0f) {
        float amax = 0.0f;
        for (int k = lane; k < dim; k += 64) amax = fmaxf(amax, fabsf(x[k] * inv));
        amax = wave_max(amax);
        int p = ilogbf(448.0f / amax);
        while (ldexpf(amax, p + 1) <= 448.0f) ++p;
        while (ldexpf(amax, p) > 448.0f) --p;
        qscale = ldexpf(1.0f, p);
    }

    // pass 3: write the normalised, rounded, zero-padded row
    float esq = 0.0f;
    if (PREC == P_FP32) {
        float* out = (float*)Xq + row * (int64_t)Kp;
        for (int k = lane; k < Kp; k += 64) {
            float v = (k < dim && inv != 0.0f) ? x[k] * inv : 0.0f;
            out[k] = v;
        }
    } else if (PREC == P_BF16) {
        uint16_t* out = (uint16_t*)Xq + row * (int64_t)Kp;
        for (int k = lane; k < Kp; k += 64) {
            uint16_t b = 0;
            if (k < dim && inv != 0.0f) {
                float v = x[k] * inv;
                b = f32_to_bf16_rne(v);
                float e = bf16_to_f32(b) - v;
                esq = fmaf(e, e, esq);
            }
            out[k] = b;
        }
    } else {
        uint8_t* out = (uint8_t*)Xq + row * (int64_t)Kp;
        const float rq = 1.0f / qscale;  // exact: power of two
        for (int k = lane; k < Kp; k += 64) {
            uint8_t b = 0;
            if (k < dim && inv != 0.0f) {
                float v = x[k] * inv;
                float q = e4m3_round(v * qscale);
                b = e4m3_bits(q);
                float e = q * rq - v;
                esq = fmaf(e, e, esq);
            }
            out[k] = b;
        }
    }
    if (PREC != P_FP32) {
        esq = wave_sum(esq);
        enorm = sqrtf(esq);
    }
    if (lane == 0) {
        RowInfo ri;
        ri.inv = inv;
        ri.qscale = qscale;
        ri.enorm = enorm;
        ri.flags = flags;
        info[row] = ri;
    }
    return enorm;
}

// Register-resident form of prep_one_row for rows of at most 1024 elements:
// the row is read from memory once (lane l holds elements l + 64 j) and every
// pass works on the registers.  Same arithmetic in the same order as
// prep_one_row, so both give identical bits.  The load is separate so that a
// wave can fetch its next row while it finishes the current one.
constexpr int kRegMax = 1024;
constexpr int kRegNV = kRegMax / 64;

// NV registers per lane hold rows of up to 64 NV elements; every loop below
// runs over the same k = lane + 64 j in the same order whatever NV is, so a
// smaller NV gives the same bits.
template <int NV>
__device__ __forceinline__ void load_row_reg(const float* __restrict__ X, bool real, int dim,
                                             int64_t ld, int64_t src, int lane,
                                             float (&xv)[NV]) {
    const float* x = X + src * ld;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int k = lane + 64 * j;
        xv[j] = (real && k < dim) ? x[k] : 0.0f;
    }
}

template <int PREC, int NV>
__device__ __forceinline__ float prep_row_regs(const float (&xv)[NV], bool real, int dim,
                                               void* __restrict__ Xq, int Kp,
                                               RowInfo* __restrict__ info,
                                               unsigned long long* __restrict__ hdr, int64_t row,
                                               int lane) {
    float inv = 0.0f, qscale = 1.0f, enorm = 0.0f;
    uint32_t flags = 0;
    float amax = 0.0f;
    bool bad = false;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        bad |= !isfinite(xv[j]);
        amax = fmaxf(amax, fabsf(xv[j]));
    }
    if (real) {
        bad = __any(bad);
        amax = wave_max(amax);
        if (bad) {
            flags = F_NONFINITE;
        } else if (amax > 0.0f) {
            int e = ilogbf(amax);
            float sc = ldexpf(1.0f, -e);
            float ss = 0.0f;
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                if (lane + 64 * j < dim) {
                    float v = xv[j] * sc;
                    ss = fmaf(v, v, ss);
                }
            }
            ss = wave_sum(ss);
            if (e < -100 || e > 99) flags = F_RANGE;
            else inv = ldexpf(1.0f / sqrtf(ss), -e);
        }
    }
    if (flags != 0 && lane == 0) atomicOr(hdr + H_FLAGS, (unsigned long long)flags);

    if (PREC == P_FP8 && inv != 0.0f) {
        float am = 0.0f;
#pragma unroll
        for (int j = 0; j < NV; ++j)
            if (lane + 64 * j < dim) am = fmaxf(am, fabsf(xv[j] * inv));
        am = wave_max(am);
        int p = ilogbf(448.0f / am);
        while (ldexpf(am, p + 1) <= 448.0f) ++p;
        while (ldexpf(am, p) > 448.0f) --p;
        qscale = ldexpf(1.0f, p);
    }

    float esq = 0.0f;
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const int k = lane + 64 * j;
        if (k >= Kp) break;
        const bool live = k < dim && inv != 0.0f;
        if (PREC == P_FP32) {
            ((float*)Xq)[row * (int64_t)Kp + k] = live ? xv[j] * inv : 0.0f;
        } else if (PREC == P_BF16) {
            uint16_t b = 0;
            if (live) {
                float v = xv[j] * inv;
                b = f32_to_bf16_rne(v);
                float e = bf16_to_f32(b) - v;
                esq = fmaf(e, e, esq);
            }
            ((uint16_t*)Xq)[row * (int64_t)Kp + k] = b;
        } else {
            uint8_t b = 0;
            if (live) {
                float v = xv[j] * inv;
                float q = e4m3_round(v * qscale);
                b = e4m3_bits(q);
                float e = q * (1.0f / qscale) - v;
                esq = fmaf(e, e, esq);
            }
            ((uint8_t*)Xq)[row * (int64_t)Kp + k] = b;
        }
    }
    if (PREC != P_FP32) {
        esq = wave_sum(esq);
        enorm = sqrtf(esq);
    }
    if (lane == 0) {
        RowInfo ri;
        ri.inv = inv;
        ri.qscale = qscale;
        ri.enorm = enorm;
        ri.flags = flags;
        info[row] = ri;
    }
    return enorm;
}

template <int PREC>
__device__ __forceinline__ float prep_row_reg(const float* __restrict__ X, int64_t rows, int dim,
                                              int64_t ld, void* __restrict__ Xq, int Kp,
                                              RowInfo* __restrict__ info,
                                              unsigned long long* __restrict__ hdr, int64_t row,
                                              int64_t src, int lane) {
    float xv[kRegNV];
    load_row_reg<kRegNV>(X, src < rows, dim, ld, src, lane, xv);
    return prep_row_regs<PREC, kRegNV>(xv, src < rows, dim, Xq, Kp, info, hdr, row, lane);
}

template <int PREC>
__device__ __forceinline__ float prep_row(const float* __restrict__ X, int64_t rows, int dim,
                                          int64_t ld, void* __restrict__ Xq, int Kp,
                                          RowInfo* __restrict__ info,
                                          unsigned long long* __restrict__ hdr, int64_t row,
                                          int64_t src, int lane) {
    if (Kp <= kRegMax)
        return prep_row_reg<PREC>(X, rows, dim, ld, Xq, Kp, info, hdr, row, src, lane);
    return prep_one_row<PREC>(X, rows, dim, ld, Xq, Kp, info, hdr, row, src, lane);
}

// One wave per row, grid-stride.
// With a selection (sel != nullptr) output row i < rows is input row sel[i]
// of a relation of n_src rows; the ids must be strictly ascending and in
// range, else the row is prepared as a zero row and F_BADSEL is raised.
__device__ __forceinline__ int64_t sel_source(const int32_t* __restrict__ sel, int64_t n_src,
                                              int64_t row, int64_t rows,
                                              unsigned long long* __restrict__ hdr, int lane,
                                              bool& real) {
    real = row < rows;
    if (!sel || !real) return row;
    const int64_t id = sel[row];
    const bool ok = id >= 0 && id < n_src && (row == 0 || (int64_t)sel[row - 1] < id);
    if (!ok) {
        if (lane == 0) atomicOr(hdr + H_FLAGS, (unsigned long long)F_BADSEL);
        real = false;
        return 0;
    }
    return id;
}

template <int PREC>
__global__ __launch_bounds__(256) void prep_rows(const float* __restrict__ X, int64_t rows,
                                                 int dim, int64_t ld, void* __restrict__ Xq,
                                                 int Kp, int64_t rows_pad,
                                                 RowInfo* __restrict__ info,
                                                 unsigned long long* __restrict__ hdr,
                                                 int enorm_slot, const int32_t* __restrict__ sel,
                                                 int64_t n_src) {
    const int lane = threadIdx.x & 63;
    float wave_emax = 0.0f;  // largest error norm seen by this wave
    const int64_t first = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t stride = (int64_t)gridDim.x * 4;
    if (Kp <= kRegMax) {
        // rows in registers; the wave's next row is loaded before the
        // current one is reduced and written
        float xa[kRegNV], xb[kRegNV];
        bool ra = false, rb = false;
        if (first < rows_pad) {
            const int64_t s0 = sel_source(sel, n_src, first, rows, hdr, lane, ra);
            load_row_reg<kRegNV>(X, ra, dim, ld, s0, lane, xa);
        }
        for (int64_t row = first; row < rows_pad; row += stride) {
            const int64_t next = row + stride;
            if (next < rows_pad) {
                const int64_t s1 = sel_source(sel, n_src, next, rows, hdr, lane, rb);
                load_row_reg<kRegNV>(X, rb, dim, ld, s1, lane, xb);
            }
            wave_emax = fmaxf(wave_emax, prep_row_regs<PREC, kRegNV>(xa, ra, dim, Xq, Kp, info,
                                                                     hdr, row, lane));
#pragma unroll
            for (int j = 0; j < kRegNV; ++j) xa[j] = xb[j];
            ra = rb;
        }
    } else {
        for (int64_t row = first; row < rows_pad; row += stride) {
            bool real;
            const int64_t src = sel_source(sel, n_src, row, rows, hdr, lane, real);
            wave_emax = fmaxf(wave_emax, prep_one_row<PREC>(X, rows, dim, ld, Xq, Kp, info, hdr,
                                                            row, src, lane, real ? 1 : 0));
        }
    }
    // one atomic per workgroup for the maximum error norm
    __shared__ float s_emax[4];
    if (lane == 0) s_emax[threadIdx.x >> 6] = wave_emax;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float m = fmaxf(fmaxf(s_emax[0], s_emax[1]), fmaxf(s_emax[2], s_emax[3]));
        if (m > 0.0f) atomicMax((unsigned int*)(hdr + enorm_slot), __float_as_uint(m));
    }
}

// Batched prep: the rows of every relation of a batch form one flat range;
// a wave finds its first row's relation by binary search over the segment
// starts and then walks forward.  Each wave takes a contiguous range of rows
// and keeps the next two rows' loads in flight while it prepares one (rows
// of relations whose depth exceeds the NV registers go through the
// unregistered form).  The grid is the number of workgroups the GPU holds at
// once, so every wave runs from the start.  The largest error norm of each
// side of a job goes to the job's counters for its measured band.
template <int PREC, int NV>
__global__ __launch_bounds__(256) void batch_prep(const BatchHead* __restrict__ head,
                                                  const PrepSeg* __restrict__ segs,
                                                  bool ordered) {
    const int lane = threadIdx.x & 63;
    const int64_t n = head->n_rows;
    const int nseg = head->n_segs;
    int lo = 0, hi = nseg - 1;
    // with an ordering, output row r holds input row perm[r]
    auto src_of = [&](const PrepSeg& g, int64_t r) {
        return (ordered && g.perm) ? (int64_t)g.perm[r] : r;
    };
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    const int64_t per = (n + n_waves - 1) / n_waves;
    const int64_t first = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * per;
    const int64_t last = min(n, first + per);
    if (first >= last) return;
    // segment of the first row (the last one starting at or before it)
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].row_base <= first) lo = mid;
        else hi = mid - 1;
    }
    auto advance = [&](int sg, int64_t row) {
        while (sg + 1 < nseg && segs[sg + 1].row_base <= row) ++sg;
        return sg;
    };
    auto fetch = [&](int sg, int64_t row, float (&x)[NV]) {
        const PrepSeg& h = segs[sg];
        if (h.Kp <= 64 * NV) {
            const int64_t sr = src_of(h, row - h.row_base);
            load_row_reg<NV>(h.X, sr < h.rows, h.dim, h.ld, sr, lane, x);
        }
    };
    float x0[NV], x1[NV], x2[NV];
    int g0 = lo, g1 = lo, g2 = lo;
    fetch(g0, first, x0);
    if (first + 1 < last) {
        g1 = advance(g0, first + 1);
        fetch(g1, first + 1, x1);
    }
    float emax = 0.0f;  // largest error norm of segment eseg among this wave's rows
    int eseg = g0;
    auto flush = [&]() {
        if (PREC != P_FP32 && lane == 0 && emax > 0.0f)
            atomicMax((unsigned int*)(segs[eseg].hdr + segs[eseg].enorm_slot),
                      __float_as_uint(emax));
    };
    for (int64_t row = first; row < last; ++row) {
        if (row + 2 < last) {
            g2 = advance(g1, row + 2);
            fetch(g2, row + 2, x2);
        }
        const PrepSeg& g = segs[g0];
        const int64_t r = row - g.row_base;
        const int64_t src = src_of(g, r);
        const float en =
            g.Kp <= 64 * NV
                ? prep_row_regs<PREC, NV>(x0, src < g.rows, g.dim, g.Xq, g.Kp, g.info, g.hdr, r,
                                          lane)
                : prep_one_row<PREC>(g.X, g.rows, g.dim, g.ld, g.Xq, g.Kp, g.info, g.hdr, r, src,
                                     lane);
        if (g0 != eseg) {
            flush();
            emax = 0.0f;
            eseg = g0;
        }
        emax = fmaxf(emax, en);
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            x0[j] = x1[j];
            x1[j] = x2[j];
        }
        g0 = g1;
        g1 = g2;
    }
    flush();
}

// registers per lane of the batched prep for the deepest relation of a batch
// (rows deeper than 1024 elements take the unregistered form)
inline int batch_prep_nv(int kp_max) {
    const int nv = (kp_max + 63) / 64;
    return nv <= 4 ? 4 : nv <= 8 ? 8 : nv <= 12 ? 12 : 16;
}

template <int PREC, int NV>
int batch_prep_grid() {
    static int grid = 0;  // resident workgroups of the device in use first
    if (grid == 0) {
        int dev = 0, cus = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, batch_prep<PREC, NV>, 256, 0) !=
                hipSuccess ||
            cus < 1 || occ < 1)
            return 1024;
        grid = cus * occ;
    }
    return grid;
}

template <int PREC, int NV>
hipError_t launch_batch_prep_nv(const BatchHead* head, const PrepSeg* segs, bool ordered,
                                hipStream_t st) {
    hipLaunchKernelGGL((batch_prep<PREC, NV>), dim3((unsigned)batch_prep_grid<PREC, NV>()),
                       dim3(256), 0, st, head, segs, ordered);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_batch_prep_p(int kp_max, const BatchHead* head, const PrepSeg* segs,
                               bool ordered, hipStream_t st) {
    switch (batch_prep_nv(kp_max)) {
        case 4: return launch_batch_prep_nv<PREC, 4>(head, segs, ordered, st);
        case 8: return launch_batch_prep_nv<PREC, 8>(head, segs, ordered, st);
        case 12: return launch_batch_prep_nv<PREC, 12>(head, segs, ordered, st);
        default: return launch_batch_prep_nv<PREC, 16>(head, segs, ordered, st);
    }
}

template <int PREC>
int batch_prep_grid_p(int kp_max) {
    switch (batch_prep_nv(kp_max)) {
        case 4: return batch_prep_grid<PREC, 4>();
        case 8: return batch_prep_grid<PREC, 8>();
        case 12: return batch_prep_grid<PREC, 12>();
        default: return batch_prep_grid<PREC, 16>();
    }
}

int batch_prep_query(int prec, int kp_max) {
    return prec == P_FP32   ? batch_prep_grid_p<P_FP32>(kp_max)
           : prec == P_BF16 ? batch_prep_grid_p<P_BF16>(kp_max)
                            : batch_prep_grid_p<P_FP8>(kp_max);
}

hipError_t launch_batch_prep(int prec, int kp_max, const BatchHead* head, const PrepSeg* segs,
                             bool ordered, hipStream_t st) {
    switch (prec) {
        case P_FP32: return launch_batch_prep_p<P_FP32>(kp_max, head, segs, ordered, st);
        case P_BF16: return launch_batch_prep_p<P_BF16>(kp_max, head, segs, ordered, st);
        default: return launch_batch_prep_p<P_FP8>(kp_max, head, segs, ordered, st);
    }
}

// Prefilter training rows: slot i < B is the R row of drawn pair i, slot
// B + i its S row, prepared exactly as the join prepares BF16 operands (one
// wave per slot).
__global__ __launch_bounds__(256) void train_rows(const TrainJob* __restrict__ jobs,
                                                  const int4* __restrict__ samples, int B, int Dp,
                                                  uint16_t* __restrict__ pool,
                                                  RowInfo* __restrict__ info,
                                                  unsigned long long* __restrict__ hdr) {
    const int lane = threadIdx.x & 63;
    const int slot = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (slot >= 2 * B) return;
    const int4 smp = samples[slot < B ? slot : slot - B];
    const TrainJob& J = jobs[smp.x];
    int64_t r = smp.z, c = smp.w;
    if (smp.y == 1) {
        const Pair p = J.out[smp.z];
        r = p.r;
        c = p.s;
    }
    if (slot < B)
        prep_row<P_BF16>(J.R, J.nR, J.dim, J.ldR, pool, Dp, info, hdr, slot, r, lane);
    else
        prep_row<P_BF16>(J.S, J.nS, J.dim, J.ldS, pool, Dp, info, hdr, slot, c, lane);
}

hipError_t launch_train_rows(const TrainJob* jobs, const int4* samples, int B, int Dp,
                             uint16_t* pool, RowInfo* info, unsigned long long* hdr,
                             hipStream_t st) {
    hipLaunchKernelGGL(train_rows, dim3((unsigned)((2 * B + 3) / 4)), dim3(256), 0, st, jobs,
                       samples, B, Dp, pool, info, hdr);
    return hipGetLastError();
}

// Zero the workspace header (a kernel rather than a memset so that the call
// sequence stays safe to capture in a graph).
__global__ void zero_header(unsigned long long* hdr) {
    if (threadIdx.x < H_COUNT) hdr[threadIdx.x] = 0ull;
}

hipError_t launch_zero_header(unsigned long long* hdr, hipStream_t st) {
    hipLaunchKernelGGL(zero_header, dim3(1), dim3(64), 0, st, hdr);
    return hipGetLastError();
}

hipError_t launch_prep(int prec, const float* X, int64_t rows, int dim, int64_t ld, void* Xq,
                       int Kp, int64_t rows_pad, RowInfo* info, unsigned long long* hdr,
                       int enorm_slot, hipStream_t st, const int32_t* sel, int64_t n_src) {
    if (rows_pad <= 0) return hipSuccess;
    int64_t nb = (rows_pad + 3) / 4;
    if (nb > 4096) nb = 4096;  // 16 workgroups per CU, a few rows per wave
    dim3 grid((unsigned)nb), block(256);
    switch (prec) {
        case P_FP32:
            hipLaunchKernelGGL(prep_rows<P_FP32>, grid, block, 0, st, X, rows, dim, ld, Xq, Kp,
                               rows_pad, info, hdr, enorm_slot, sel, n_src);
            break;
        case P_BF16:
            hipLaunchKernelGGL(prep_rows<P_BF16>, grid, block, 0, st, X, rows, dim, ld, Xq, Kp,
                               rows_pad, info, hdr, enorm_slot, sel, n_src);
            break;
        default:
            hipLaunchKernelGGL(prep_rows<P_FP8>, grid, block, 0, st, X, rows, dim, ld, Xq, Kp,
                               rows_pad, info, hdr, enorm_slot, sel, n_src);
            break;
    }
    return hipGetLastError();
}

}  // namespace ej
