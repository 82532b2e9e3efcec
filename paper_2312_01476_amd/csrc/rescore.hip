// rescore.hip -- FP64 rescoring of the pairs whose approximate score falls in
// the uncertainty band around theta.
//
// The similarity is the cosine of Section III.A.  The band pairs are decided
// with the canonical FP64 rule, evaluated from the caller's original float32
// rows:
//     dot(a,b) = (((0 + a0 b0) + a1 b1) + ...)  sequential, one rounding per
//                product and per sum.  The product of two float32 values is
//                exact in float64 (at most 48 significant bits, exponents far
//                inside the range), so its rounding changes nothing and each
//                step is computed as one fused multiply-add, whose single
//                rounding is the sum's; no other contraction appears (the
//                file is compiled without it);
//     sim64    = dot(r,s) / sqrt(dot(r,r) dot(s,s)),  0 for a zero row;
//     accept   iff sim64 >= theta.
// The same rule defines the exact result set, so a pair accepted here is a
// pair of that set and the score written is sim64 rounded to float.
#include <algorithm>

#include "common.hpp"
#include "batch.hpp"
#include "launch.hpp"

namespace ej {

// Each lane of a wave holds one pair (rp, sp, dim; valid = false for none)
// and gets sim64 of it: the rule is sequential in k, so one lane sums one
// pair.  The rows come in through LDS in chunks of 16 elements so that every
// global load reads whole row segments: four lanes take the 64-byte segment
// of one row (R or S of one pair) at the address they find in the wave's
// pair table in LDS, 16 segments per load, 16 bytes per lane (as four 4-byte
// loads when some row of the wave does not start on 16 bytes); the LDS
// stores and every lane's reads of its own pair also move 16 bytes.  The
// next two chunks' loads are in flight in registers while a chunk is summed.
// Elements past a pair's dim are zero and are summed like the others:
// x + 0 * 0 = x exactly, so the sums are those of the sequential definition
// over k < dim.  A lane without a pair borrows lane 0's (every calling wave
// has one there) and its result is not used.
constexpr int kChunk = 16;
// floats per pair: R chunk, S chunk, pad to an odd number of 16-byte groups,
// so that 16 lanes reading 16 bytes of 16 pairs hit 16 different bank groups
constexpr int kPairStride = 2 * kChunk + 4;

typedef __attribute__((address_space(1))) const float* grow_ptr;

struct alignas(16) PairLds {
    uint64_t ptr[64][2];  // the wave's pairs: R row, S row (global addresses)
    float buf[64 * kPairStride];  // 10 KB a wave with the table: four workgroups per CU
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const v4f* gv4f_ptr;

// The sequential sums of the wave's pairs (table in L, pair lengths kmax,
// smallest and largest dmin, dmax).  Load j of a chunk: row segment
// 16 j + lane / 4 (pair (16 j + lane / 4) / 2, R or S by its parity),
// elements 4 (lane % 4) .. + 4 of the chunk.  The chunks inside every pair
// run with two chunks' loads in flight (every load issued whatever the
// chunk, so that the compiler waits for one chunk while the next loads); the
// chunks past some pair's end follow one at a time.
template <bool VEC>
__device__ __forceinline__ void sim64_sums(PairLds& L, int dmin, int dmax, int kmax, double& dot,
                                           double& nr, double& ns) {
    const int lane = threadIdx.x & 63;
    const int piece = lane & 3, rcl = lane >> 2;
    const float* mine = L.buf + lane * kPairStride;
    auto load_full = [&](int c, v4f (&v)[8]) {
        const int k = kChunk * c + 4 * piece;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int rc = 16 * j + rcl;
            const grow_ptr x = (grow_ptr)L.ptr[rc >> 1][rc & 1] + k;
            if (VEC) {
                v[j] = *(gv4f_ptr)x;
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) v[j][t] = x[t];
            }
        }
    };
    auto load_tail = [&](int c, v4f (&v)[8]) {
        const int k = kChunk * c + 4 * piece;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int rc = 16 * j + rcl;
            const grow_ptr x = (grow_ptr)L.ptr[rc >> 1][rc & 1];
            const int km = __shfl(kmax, rc >> 1, 64);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const bool ok = k + t < km;
                const float xv = x[ok ? k + t : 0];
                v[j][t] = ok ? xv : 0.0f;
            }
        }
    };
    auto store = [&](const v4f (&v)[8]) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int rc = 16 * j + rcl;
            *(v4f*)(L.buf + (rc >> 1) * kPairStride + (rc & 1) * kChunk + 4 * piece) = v[j];
        }
    };
    auto sum = [&]() {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const v4f ra = *(const v4f*)(mine + 4 * t);
            const v4f sa = *(const v4f*)(mine + kChunk + 4 * t);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double x = (double)ra[c];
                const double y = (double)sa[c];
                dot = __builtin_fma(x, y, dot);  // x * y exact: the sum's rounding only
                nr = __builtin_fma(x, x, nr);
                ns = __builtin_fma(y, y, ns);
            }
        }
    };
    const int nfull = dmin / kChunk;  // chunks inside every pair (wave-uniform)
    if (nfull > 0) {
        // two buffers in a fixed rotation; past the last full chunk the
        // loads repeat it (unused)
        v4f va[8], vb[8];
        load_full(0, va);
        load_full(min(1, nfull - 1), vb);
        int c = 0;
        for (; c + 1 < nfull; c += 2) {
            store(va);
            wave_lds_sync();
            load_full(min(c + 2, nfull - 1), va);
            sum();
            wave_lds_sync();
            store(vb);
            wave_lds_sync();
            load_full(min(c + 3, nfull - 1), vb);
            sum();
            wave_lds_sync();
        }
        if (c < nfull) {
            store(va);
            wave_lds_sync();
            sum();
            wave_lds_sync();
        }
    }
    for (int c = nfull; kChunk * c < dmax; ++c) {
        v4f vt[8];
        load_tail(c, vt);
        store(vt);
        wave_lds_sync();
        sum();
        wave_lds_sync();
    }
}

__device__ __forceinline__ double wave_sim64(const float* rp, const float* sp, int dim, bool valid,
                                             PairLds& L) {
    const int lane = threadIdx.x & 63;
    // lane 0's pair stands in for lanes without one
    const uint64_t r0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                             (int)(uint32_t)((uint64_t)rp >> 32), 0) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)rp, 0);
    const uint64_t s0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(
                             (int)(uint32_t)((uint64_t)sp >> 32), 0) << 32) |
                        (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)sp, 0);
    const int d0 = __builtin_amdgcn_readlane(dim, 0);
    const int kmax = valid ? dim : d0;
    L.ptr[lane][0] = valid ? (uint64_t)rp : r0;
    L.ptr[lane][1] = valid ? (uint64_t)sp : s0;
    int dmax = kmax, dmin = kmax;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        dmax = max(dmax, __shfl_xor(dmax, o, 64));
        dmin = min(dmin, __shfl_xor(dmin, o, 64));
    }
    // every row of the wave on 16 bytes (lanes without a pair stand in lane
    // 0's): 16-byte loads, else four 4-byte loads of the same elements
    const bool vec = __all(!valid || ((((uint64_t)rp | (uint64_t)sp) & 15) == 0)) &&
                     (((r0 | s0) & 15) == 0);
    wave_lds_sync();
    double dot = 0.0, nr = 0.0, ns = 0.0;
    if (vec) sim64_sums<true>(L, dmin, dmax, kmax, dot, nr, ns);
    else sim64_sums<false>(L, dmin, dmax, kmax, dot, nr, ns);
    if (nr == 0.0 || ns == 0.0) return 0.0;
    return dot / __builtin_sqrt(nr * ns);
}

// One lane per band pair; accepted pairs are appended to the output with one
// atomicAdd per wave.
__global__ __launch_bounds__(256) void rescore_band(const float* __restrict__ R, int64_t ldR,
                                                    const float* __restrict__ S, int64_t ldS,
                                                    int dim, const int2* __restrict__ band,
                                                    int64_t band_cap, double theta,
                                                    Pair* __restrict__ out, int64_t capacity,
                                                    unsigned long long* __restrict__ hdr,
                                                    const int32_t* __restrict__ sel_r,
                                                    const int32_t* __restrict__ sel_s) {
    if (hdr[H_FLAGS] != 0) return;
    __shared__ PairLds s_pairs[4];
    PairLds& lds = s_pairs[threadIdx.x >> 6];
    const int64_t n = min((int64_t)hdr[H_BAND], band_cap);
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n;
         base += stride) {
        const int64_t p = base + lane;
        bool acc = false;
        double sim = 0.0;
        int2 e = make_int2(0, 0);
        if (p < n) e = band[p];
        const int64_t ri = (p < n && sel_r) ? (int64_t)sel_r[e.x] : (int64_t)e.x;
        const int64_t si = (p < n && sel_s) ? (int64_t)sel_s[e.y] : (int64_t)e.y;
        sim = wave_sim64(R + ri * ldR, S + si * ldS, dim, p < n, lds);
        acc = p < n && sim >= theta;
        const uint64_t m = __ballot(acc);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            unsigned long long b = 0;
            if (lane == leader) {
                b = atomicAdd(hdr + H_OUT, (unsigned long long)__popcll(m));
                atomicAdd(hdr + H_BAND_ACC, (unsigned long long)__popcll(m));
            }
            const uint32_t blo = __shfl((uint32_t)b, leader, 64);
            const uint32_t bhi = __shfl((uint32_t)(b >> 32), leader, 64);
            const unsigned long long bb = ((unsigned long long)bhi << 32) | blo;
            if (acc) {
                const unsigned long long q = bb + lanes_below(m);
                if ((int64_t)q < capacity) {
                    Pair pr;
                    pr.r = e.x;
                    pr.s = e.y;
                    pr.score = (float)sim;
                    out[q] = pr;
                }
            }
        }
    }
}

hipError_t launch_rescore_band(const float* R, int64_t ldR, const float* S, int64_t ldS, int dim,
                               const int2* band, int64_t band_cap, double theta, Pair* out,
                               int64_t capacity, unsigned long long* hdr, hipStream_t st,
                               const int32_t* sel_r, const int32_t* sel_s) {
    if (band_cap <= 0) return hipSuccess;
    int64_t blocks = (band_cap + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(rescore_band, dim3((unsigned)blocks), dim3(256), 0, st, R, ldR, S, ldS, dim,
                       band, band_cap, theta, out, capacity, hdr, sel_r, sel_s);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// selections pushed below the join: offsets back to the caller's row ids
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void map_pairs(Pair* __restrict__ out, int64_t capacity,
                                                 const unsigned long long* __restrict__ hdr,
                                                 const int32_t* __restrict__ sel_r,
                                                 const int32_t* __restrict__ sel_s) {
    if (hdr[H_FLAGS] != 0) return;
    const int64_t n = min((int64_t)hdr[H_OUT], capacity);
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        Pair p = out[q];
        if (sel_r) p.r = sel_r[p.r];
        if (sel_s) p.s = sel_s[p.s];
        out[q] = p;
    }
}

hipError_t launch_map_pairs(Pair* out, int64_t capacity, const unsigned long long* hdr,
                            const int32_t* sel_r, const int32_t* sel_s, hipStream_t st) {
    if (capacity <= 0 || (!sel_r && !sel_s)) return hipSuccess;
    int64_t blocks = (capacity + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(map_pairs, dim3((unsigned)blocks), dim3(256), 0, st, out, capacity, hdr,
                       sel_r, sel_s);
    return hipGetLastError();
}

// one wave per selected row: check the id, copy the row
__global__ __launch_bounds__(256) void gather_rows(const float* __restrict__ X, int64_t ld, int dim,
                                                   const int32_t* __restrict__ sel, int64_t n,
                                                   int64_t n_src, float* __restrict__ dst,
                                                   unsigned long long* __restrict__ hdr) {
    const int lane = threadIdx.x & 63;
    for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n;
         i += (int64_t)gridDim.x * 4) {
        const int64_t id = sel[i];
        const bool ok = id >= 0 && id < n_src && (i == 0 || (int64_t)sel[i - 1] < id);
        float* d = dst + i * (int64_t)dim;
        if (!ok) {
            if (lane == 0) atomicOr(hdr + H_FLAGS, (unsigned long long)F_BADSEL);
            for (int k = lane; k < dim; k += 64) d[k] = 0.0f;
            continue;
        }
        const float* x = X + id * ld;
        for (int k = lane; k < dim; k += 64) d[k] = x[k];
    }
}

hipError_t launch_gather_rows(const float* X, int64_t ld, int dim, const int32_t* sel, int64_t n,
                              int64_t n_src, float* dst, unsigned long long* hdr, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 3) / 4;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(gather_rows, dim3((unsigned)blocks), dim3(256), 0, st, X, ld, dim, sel, n,
                       n_src, dst, hdr);
    return hipGetLastError();
}

// After a failed input check the outputs were never written: nothing runs.
__global__ __launch_bounds__(256) void map_topk(int32_t* __restrict__ idx, int64_t n,
                                                const int32_t* __restrict__ sel_s, int64_t n_sel,
                                                const unsigned long long* __restrict__ hdr) {
    if (hdr[H_FLAGS] != 0) return;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = idx[q];
        if (j >= 0 && j < n_sel) idx[q] = sel_s[j];
    }
}

hipError_t launch_map_topk(int32_t* idx, int64_t n, const int32_t* sel_s, int64_t n_sel,
                           const unsigned long long* hdr, hipStream_t st) {
    if (n <= 0 || !sel_s) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(map_topk, dim3((unsigned)blocks), dim3(256), 0, st, idx, n, sel_s, n_sel,
                       hdr);
    return hipGetLastError();
}

// Batched rescore: one lane per entry of the band list shared by the jobs
// of a batch ({r, s, job}); each entry is decided with its own job's rows and
// theta.  Accepted pairs are appended to their job's output with one
// atomicAdd per (wave, job): lanes are grouped by job with ballots (entries
// of one tile are contiguous, so a wave nearly always holds one job).
__global__ __launch_bounds__(256) void batch_rescore(const BatchHead* __restrict__ head,
                                                     const BatchJob* __restrict__ jobs,
                                                     const unsigned long long* __restrict__ bctr) {
    const int64_t n = min((int64_t)bctr[B_BAND], head->band_cap);
    const int4* __restrict__ band = head->band;
    __shared__ PairLds s_pairs[4];
    PairLds& lds = s_pairs[threadIdx.x >> 6];
    const int lane = threadIdx.x & 63;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < n;
         base += stride) {
        const int64_t p = base + lane;
        bool acc = false;
        double sim = 0.0;
        int4 e = make_int4(0, 0, -1, 0);
        const float* rp = nullptr;
        const float* sp = nullptr;
        int dim = 0;
        double theta = 0.0;
        if (p < n) {
            e = band[p];
            const BatchJob& J = jobs[e.z];
            rp = J.R + (int64_t)e.x * J.ldR;
            sp = J.S + (int64_t)e.y * J.ldS;
            dim = J.dim;
            theta = J.theta;
        }
        sim = wave_sim64(rp, sp, dim, p < n, lds);
        acc = p < n && sim >= theta;
        uint64_t todo = __ballot(acc);
        while (todo) {
            const int leader = __ffsll((unsigned long long)todo) - 1;
            const int job = __shfl(e.z, leader, 64);
            const uint64_t m = __ballot(acc && e.z == job);
            todo &= ~m;
            unsigned long long* hdr = jobs[job].hdr;
            unsigned long long b = 0;
            if (lane == leader) {
                b = atomicAdd(hdr + H_OUT, (unsigned long long)__popcll(m));
                atomicAdd(hdr + H_BAND_ACC, (unsigned long long)__popcll(m));
            }
            const uint32_t blo = __shfl((uint32_t)b, leader, 64);
            const uint32_t bhi = __shfl((uint32_t)(b >> 32), leader, 64);
            const unsigned long long bb = ((unsigned long long)bhi << 32) | blo;
            if ((m >> lane) & 1ull) {
                const unsigned long long q = bb + lanes_below(m);
                if ((int64_t)q < jobs[job].capacity) {
                    Pair pr;
                    pr.r = e.x;
                    pr.s = e.y;
                    pr.score = (float)sim;
                    jobs[job].out[q] = pr;
                }
            }
        }
    }
}

hipError_t launch_batch_rescore(const BatchHead* head, const BatchJob* jobs,
                                const unsigned long long* bctr, int grid, hipStream_t st) {
    hipLaunchKernelGGL(batch_rescore, dim3((unsigned)grid), dim3(256), 0, st, head, jobs, bctr);
    return hipGetLastError();
}

// Prefilter training targets: sim64 of every drawn pair (one lane each).
__global__ __launch_bounds__(256) void train_targets(const TrainJob* __restrict__ jobs,
                                                     const int4* __restrict__ samples, int B,
                                                     float* __restrict__ t) {
    __shared__ PairLds s_pairs[4];
    PairLds& lds = s_pairs[threadIdx.x >> 6];
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < B;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = base + (threadIdx.x & 63);
        const float* rp = nullptr;
        const float* sp = nullptr;
        int dim = 0;
        if (i < B) {
            const int4 smp = samples[i];
            const TrainJob& J = jobs[smp.x];
            int64_t r = smp.z, c = smp.w;
            if (smp.y == 1) {
                const Pair p = J.out[smp.z];
                r = p.r;
                c = p.s;
            }
            rp = J.R + r * J.ldR;
            sp = J.S + c * J.ldS;
            dim = J.dim;
        }
        const double sim = wave_sim64(rp, sp, dim, i < B, lds);
        if (i < B) t[i] = (float)sim;
    }
}

hipError_t launch_train_targets(const TrainJob* jobs, const int4* samples, int B, float* t,
                                hipStream_t st) {
    const int blocks = std::max(1, std::min(1024, (B + 255) / 256));
    hipLaunchKernelGGL(train_targets, dim3((unsigned)blocks), dim3(256), 0, st, jobs, samples, B,
                       t);
    return hipGetLastError();
}

// The measured band: the same bound as the rigorous one with the error norms
// the prep pass measured instead of their worst case (each read as float,
// widened by 0.1% for the FP32 evaluation of the norms).
__global__ void band_edges(unsigned long long* hdr, double theta, double f, double rigorous,
                           int alias, int all64) {
    if (threadIdx.x != 0) return;
    const double er = (double)__uint_as_float((uint32_t)hdr[H_ENORM_R]) * 1.001 + 1e-7;
    // a self-join prepares one copy: its rows' norms serve both sides
    const double es =
        (double)__uint_as_float((uint32_t)hdr[alias ? H_ENORM_R : H_ENORM_S]) * 1.001 + 1e-7;
    double d = er * (1.0 + es) + es + f * (1.0 + er) * (1.0 + es);
    if (!(d <= rigorous)) d = rigorous;
    const double lo = theta - d, hi = theta + d;
    float flo = (float)lo, fhi = (float)hi;
    if ((double)flo > lo) flo = nextafterf(flo, -INFINITY);
    if ((double)fhi < hi) fhi = nextafterf(fhi, INFINITY);
    if (all64) fhi = INFINITY;  // every candidate goes to the rescore
    hdr[H_LO] = (unsigned long long)__float_as_uint(flo);
    hdr[H_HI] = (unsigned long long)__float_as_uint(fhi);
    hdr[H_BAND_W] = (unsigned long long)__double_as_longlong(d);
}

hipError_t launch_band_edges(unsigned long long* hdr, double theta, double fp32_terms,
                             double rigorous, bool alias, bool all64, hipStream_t st) {
    hipLaunchKernelGGL(band_edges, dim3(1), dim3(64), 0, st, hdr, theta, fp32_terms, rigorous,
                       alias ? 1 : 0, all64 ? 1 : 0);
    return hipGetLastError();
}

// Device-side copy of the output count (asynchronous mode): the count, or
// minus the status code of a failure found on the device.
__global__ void copy_count(const unsigned long long* hdr, int64_t band_cap, int64_t* dst) {
    if (threadIdx.x != 0) return;
    int64_t v = (int64_t)hdr[H_OUT];
    if (hdr[H_FLAGS] & F_BADSEL) v = -1;                // EJOIN_E_INVAL
    else if (hdr[H_FLAGS] & F_NONFINITE) v = -4;        // EJOIN_E_NONFINITE
    else if (hdr[H_FLAGS] & F_RANGE) v = -7;            // EJOIN_E_RANGE
    else if ((int64_t)hdr[H_BAND] > band_cap) v = -3;   // EJOIN_E_WORKSPACE
    dst[0] = v;
}

hipError_t launch_copy_count(const unsigned long long* hdr, int64_t band_cap, int64_t* dst,
                             hipStream_t st) {
    hipLaunchKernelGGL(copy_count, dim3(1), dim3(64), 0, st, hdr, band_cap, dst);
    return hipGetLastError();
}

}  // namespace ej
