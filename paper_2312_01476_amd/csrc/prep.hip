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

// Every memory access of the prep kernels goes through global (not generic)
// pointers: a generic access may be served by LDS as well, and while one is
// in flight the compiler waits for every outstanding load before it uses any
// loaded register, which would drain the rows kept in flight.
typedef __attribute__((address_space(1))) const float* gsrc_ptr;

__device__ __forceinline__ void global_or(unsigned long long* p, unsigned long long v) {
    __hip_atomic_fetch_or((__attribute__((address_space(1))) unsigned long long*)p, v,
                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void global_max_u32(unsigned long long* slot, float v) {
    __hip_atomic_fetch_max((__attribute__((address_space(1))) unsigned int*)slot,
                           __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
// one 16-byte global store of a row's RowInfo
__device__ __forceinline__ void store_info(RowInfo* info, int64_t row, float inv, float qscale,
                                           float enorm, uint32_t flags) {
    typedef unsigned int v4u __attribute__((ext_vector_type(4)));
    v4u w;
    w[0] = __float_as_uint(inv);
    w[1] = __float_as_uint(qscale);
    w[2] = __float_as_uint(enorm);
    w[3] = flags;
    *(__attribute__((address_space(1))) v4u*)(info + row) = w;
}

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
    const gsrc_ptr x = (gsrc_ptr)(X + src * ld);
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
    if (flags != 0 && lane == 0) global_or(hdr + H_FLAGS, (unsigned long long)flags);

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
        const auto out = gptr((float*)Xq + row * (int64_t)Kp);
        for (int k = lane; k < Kp; k += 64) {
            float v = (k < dim && inv != 0.0f) ? x[k] * inv : 0.0f;
            out[k] = v;
        }
    } else if (PREC == P_BF16) {
        const auto out = gptr((uint16_t*)Xq + row * (int64_t)Kp);
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
        const auto out = gptr((uint8_t*)Xq + row * (int64_t)Kp);
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
    if (lane == 0) store_info(info, row, inv, qscale, enorm, flags);
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
// Every lane issues all NV loads, whatever the row and its length (a row that
// is not real reads row 0, a lane past dim the row's last element), so that
// the number of loads in flight never depends on a branch and the compiler
// can wait for one row while the next ones load.  The values are raw: the
// elements that are not the row's are zeroed by prep_row_regs, where they
// are first used.  X must hold a row 0.
template <int NV>
__device__ __forceinline__ void load_row_reg(const float* __restrict__ X, bool real, int dim,
                                             int64_t ld, int64_t src, int lane,
                                             float (&xv)[NV]) {
    const gsrc_ptr x = (gsrc_ptr)(X + (real ? src : 0) * ld);
#pragma unroll
    for (int j = 0; j < NV; ++j) xv[j] = x[min(lane + 64 * j, dim - 1)];
}

template <int PREC, int NV>
__device__ __forceinline__ float prep_row_regs(const float (&xraw)[NV], bool real, int dim,
                                               void* __restrict__ Xq, int Kp,
                                               RowInfo* __restrict__ info,
                                               unsigned long long* __restrict__ hdr, int64_t row,
                                               int lane) {
    float xv[NV];  // the row's elements, zero past dim and for a row that is not real
#pragma unroll
    for (int j = 0; j < NV; ++j) xv[j] = (real && lane + 64 * j < dim) ? xraw[j] : 0.0f;
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
    if (flags != 0 && lane == 0) global_or(hdr + H_FLAGS, (unsigned long long)flags);

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
            ((__attribute__((address_space(1))) float*)Xq)[row * (int64_t)Kp + k] =
                live ? xv[j] * inv : 0.0f;
        } else if (PREC == P_BF16) {
            uint16_t b = 0;
            if (live) {
                float v = xv[j] * inv;
                b = f32_to_bf16_rne(v);
                float e = bf16_to_f32(b) - v;
                esq = fmaf(e, e, esq);
            }
            ((__attribute__((address_space(1))) uint16_t*)Xq)[row * (int64_t)Kp + k] = b;
        } else {
            uint8_t b = 0;
            if (live) {
                float v = xv[j] * inv;
                float q = e4m3_round(v * qscale);
                b = e4m3_bits(q);
                float e = q * (1.0f / qscale) - v;
                esq = fmaf(e, e, esq);
            }
            ((__attribute__((address_space(1))) uint8_t*)Xq)[row * (int64_t)Kp + k] = b;
        }
    }
    if (PREC != P_FP32) {
        esq = wave_sum(esq);
        enorm = sqrtf(esq);
    }
    if (lane == 0) store_info(info, row, inv, qscale, enorm, flags);
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
    typedef const __attribute__((address_space(4))) int32_t* csel_ptr;  // scalar loads
    const int64_t id = ((csel_ptr)sel)[row];
    const bool ok =
        id >= 0 && id < n_src && (row == 0 || (int64_t)((csel_ptr)sel)[row - 1] < id);
    if (!ok) {
        if (lane == 0) global_or(hdr + H_FLAGS, (unsigned long long)F_BADSEL);
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
    // the wave index made visibly uniform: row numbers, selection ids and
    // table fields then come through scalar loads, whose waits leave the
    // vector loads of the rows in flight
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t first = (int64_t)blockIdx.x * 4 + wv;
    const int64_t stride = (int64_t)gridDim.x * 4;
    // rows in registers when some input row exists to stand in for padding
    const bool x_rows = sel ? n_src > 0 : rows > 0;
    if (Kp <= kRegMax && x_rows && first < rows_pad) {
        // three row buffers in a fixed rotation: the wave's next two rows are
        // loaded before the current one is reduced and written (the loop is
        // unrolled by three rather than copying buffers: a copy of a register
        // whose load is in flight would wait for it); prefetches past the end
        // load the last row again
        float x0[kRegNV], x1[kRegNV], x2[kRegNV];
        bool r0, r1, r2;
        auto fetch = [&](int64_t row, float (&x)[kRegNV], bool& rl) {
            const int64_t rc = min(row, rows_pad - 1);
            const int64_t src = sel_source(sel, n_src, rc, rows, hdr, lane, rl);
            load_row_reg<kRegNV>(X, rl, dim, ld, src, lane, x);
        };
        auto body = [&](int64_t row, const float (&x)[kRegNV], bool rl) {
            wave_emax = fmaxf(wave_emax,
                              prep_row_regs<PREC, kRegNV>(x, rl, dim, Xq, Kp, info, hdr, row, lane));
        };
        fetch(first, x0, r0);
        fetch(first + stride, x1, r1);
        for (int64_t row = first;;) {
            fetch(row + 2 * stride, x2, r2);
            body(row, x0, r0);
            if ((row += stride) >= rows_pad) break;
            fetch(row + 2 * stride, x0, r0);
            body(row, x1, r1);
            if ((row += stride) >= rows_pad) break;
            fetch(row + 2 * stride, x1, r1);
            body(row, x2, r2);
            if ((row += stride) >= rows_pad) break;
        }
    } else if (Kp > kRegMax || !x_rows) {
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
        if (m > 0.0f) global_max_u32(hdr + enorm_slot, m);
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
    // (the permutation is read through the constant address space: one
    // scalar load of a uniform address, waited for apart from the rows)
    auto src_of = [&](const PrepSeg& g, int64_t r) {
        const int ri = __builtin_amdgcn_readfirstlane((int)r);  // r < 2^31, uniform
        return (ordered && g.perm)
                   ? (int64_t)((const __attribute__((address_space(4))) int32_t*)g.perm)[ri]
                   : r;
    };
    const int64_t n_waves = (int64_t)gridDim.x * 4;
    const int64_t per = (n + n_waves - 1) / n_waves;
    // the wave index made visibly uniform: segment fields, permutation
    // entries and row numbers then come through scalar loads, whose waits
    // leave the vector loads of the next rows in flight
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t first = ((int64_t)blockIdx.x * 4 + wv) * per;
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
    // every fetch loads (see load_row_reg), also for a relation deeper than
    // the registers (its first 1024 elements, unused) and past the wave's
    // last row (the last row again); every relation with rows in the flat
    // range has a row 0
    auto fetch = [&](int sg, int64_t row, float (&x)[NV]) {
        const PrepSeg& h = segs[sg];
        const int64_t sr = src_of(h, row - h.row_base);
        load_row_reg<NV>(h.X, sr < h.rows, h.dim, h.ld, sr, lane, x);
    };
    // three row buffers in a fixed rotation (the loop is unrolled by three
    // rather than copying buffers: a copy of a register whose load is in
    // flight would wait for that load)
    float x0[NV], x1[NV], x2[NV];
    int ga = lo, gb = lo, gc = lo;  // segments of the rows in x0, x1, x2
    fetch(ga, first, x0);
    gb = advance(ga, min(first + 1, last - 1));
    fetch(gb, min(first + 1, last - 1), x1);
    float emax = 0.0f;  // largest error norm of segment eseg among this wave's rows
    int eseg = ga;
    auto flush = [&]() {
        if (PREC != P_FP32 && lane == 0 && emax > 0.0f)
            global_max_u32(segs[eseg].hdr + segs[eseg].enorm_slot, emax);
    };
    auto body = [&](int64_t row, const float (&x)[NV], int sg) {
        const PrepSeg& g = segs[sg];
        const int64_t r = row - g.row_base;
        const int64_t src = src_of(g, r);
        // (only the 16-register form meets relations deeper than its registers)
        const float en =
            (NV == kRegNV && g.Kp > 64 * NV)
                ? prep_one_row<PREC>(g.X, g.rows, g.dim, g.ld, g.Xq, g.Kp, g.info, g.hdr, r, src,
                                     lane)
                : prep_row_regs<PREC, NV>(x, src < g.rows, g.dim, g.Xq, g.Kp, g.info, g.hdr, r,
                                          lane);
        if (sg != eseg) {
            flush();
            emax = 0.0f;
            eseg = sg;
        }
        emax = fmaxf(emax, en);
    };
    for (int64_t row = first;;) {
        // x0: row, x1: row + 1; row + 2 goes to x2
        const int64_t p2 = min(row + 2, last - 1);
        gc = advance(gb, p2);
        fetch(gc, p2, x2);
        body(row, x0, ga);
        if (++row >= last) break;
        // x1: row, x2: row + 1; row + 2 goes to x0
        const int64_t p0 = min(row + 2, last - 1);
        ga = advance(gc, p0);
        fetch(ga, p0, x0);
        body(row, x1, gb);
        if (++row >= last) break;
        // x2: row, x0: row + 1; row + 2 goes to x1
        const int64_t p1 = min(row + 2, last - 1);
        gb = advance(ga, p1);
        fetch(gb, p1, x1);
        body(row, x2, gc);
        if (++row >= last) break;
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
