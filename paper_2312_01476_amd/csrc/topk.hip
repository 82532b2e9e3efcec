// topk.hip -- exact top-k E-join: candidate floor, certification, FP64
// rescoring and ordered selection.
//
// The top-k join condition (Section VI.E, the scan side of the scan-versus-
// probe study) asks, for every R tuple, for the k most similar S tuples.  The
// result here is exact with respect to the canonical FP64 similarity
// (sequential sums from the float32 inputs, dot / sqrt(|r|^2 |s|^2)), ordered
// by (similarity desc, S index asc):
//
//  1. a pilot computes the exact k-th similarity T_k of a few sample rows and
//     sets the candidate floor F = min T_k - 2 D (D: largest error bound of
//     the approximate scores);
//  2. the contraction sweep (panel kernel, candidate epilogue) stores every
//     column with approximate score a >= F in its row's candidate slots;
//  3. per row: A_k = k-th largest candidate score, D_i = the row's error
//     bound.  Any true top-k column j has a_ij >= A_k - 2 D_i.  If no slot
//     overflowed and A_k - 2 D_i >= F, every such column is a candidate: they
//     are rescored in FP64 and sorted, which gives the exact answer;
//  4. rows that fail the certificate take an exact FP64 scan of all S.
#include <math.h>

#include "common.hpp"
#include "launch.hpp"

namespace ej {

// canonical FP64 pieces: sums in order k = 0..d-1, one rounding per product
// and per sum (this file is compiled without FP contraction)
__device__ __forceinline__ double dot64_seq(const float* __restrict__ a,
                                            const float* __restrict__ b, int d) {
    double acc = 0.0;
    for (int k = 0; k < d; ++k) acc = acc + (double)a[k] * (double)b[k];
    return acc;
}
__device__ __forceinline__ double sim64_from(double dot, double nr, double ns) {
    if (nr == 0.0 || ns == 0.0) return 0.0;
    return dot / __builtin_sqrt(nr * ns);
}
// largest float below x (x finite)
__device__ __forceinline__ float next_down(float x) {
    if (x == 0.0f) return -1.401298464e-45f;
    const uint32_t u = __float_as_uint(x);
    return __uint_as_float(x > 0.0f ? u - 1u : u + 1u);
}
// strict top-k order: higher similarity first, then smaller index
__device__ __forceinline__ bool better(double va, int ja, double vb, int jb) {
    return va > vb || (va == vb && ja < jb);
}

// Squared FP64 norms of all rows (one lane per row).
__global__ __launch_bounds__(256) void norms64(const float* __restrict__ X, int64_t rows, int dim,
                                               int64_t ld, double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = dot64_seq(X + i * ld, X + i * ld, dim);
}

// Exact FP64 top-k of the rows in `rows_list` (one workgroup per row).  A
// block-wide buffer of 512 (score, index) entries collects every column that
// beats the current k-th best; when it fills it is sorted (bitonic) and cut to
// k.  k <= 256.
constexpr int XK_BUF = 512;

__device__ void bitonic_sort_desc(double* v, int* j, int n_pow2) {
    // sorts (v desc, j asc) over n_pow2 entries with 256 threads
    for (int size = 2; size <= n_pow2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < n_pow2 / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);  // first half of each block: descending
                const bool hi_better = better(v[hi], j[hi], v[lo], j[lo]);
                if (hi_better == up) {
                    const double tv = v[lo];
                    v[lo] = v[hi];
                    v[hi] = tv;
                    const int tj = j[lo];
                    j[lo] = j[hi];
                    j[hi] = tj;
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(256) void exact_topk_rows(
    const float* __restrict__ R, int64_t ldR, const float* __restrict__ S, int64_t ldS, int dim,
    int64_t nS, const double* __restrict__ nr64, const double* __restrict__ ns64, int k,
    const int* __restrict__ rows_list, const unsigned long long* __restrict__ n_rows_ptr,
    int n_rows_fixed, int32_t* __restrict__ out_idx, float* __restrict__ out_score,
    double* __restrict__ kth_out) {
    __shared__ double bv[XK_BUF];
    __shared__ int bj[XK_BUF];
    __shared__ int s_n;
    __shared__ double s_thr_v;
    __shared__ int s_thr_j;
    __shared__ int s_wcnt[4];

    const int n_rows = n_rows_ptr ? (int)*n_rows_ptr : n_rows_fixed;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int rr = blockIdx.x; rr < n_rows; rr += gridDim.x) {
        const int64_t i = rows_list[rr];
        const float* r = R + i * ldR;
        const double nr = nr64[i];
        if (threadIdx.x == 0) {
            s_n = 0;
            s_thr_v = -INFINITY;
            s_thr_j = 0x7fffffff;
        }
        __syncthreads();
        for (int64_t j0 = 0; j0 < nS; j0 += 256) {
            const int64_t jj = j0 + threadIdx.x;
            double v = -INFINITY;
            bool cand = false;
            if (jj < nS) {
                v = sim64_from(dot64_seq(r, S + jj * ldS, dim), nr, ns64[jj]);
                cand = better(v, (int)jj, s_thr_v, s_thr_j);
            }
            // block compaction into the buffer
            const uint64_t m = __ballot(cand);
            if (lane == 0) s_wcnt[wave] = __popcll(m);
            __syncthreads();
            int off = s_n;
            for (int w = 0; w < wave; ++w) off += s_wcnt[w];
            const int total = s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3];
            if (cand) {
                const int p = off + (int)lanes_below(m);
                bv[p] = v;
                bj[p] = (int)jj;
            }
            __syncthreads();
            if (threadIdx.x == 0) s_n += total;
            __syncthreads();
            // keep room for the next chunk: sort and cut to k
            if (s_n > XK_BUF - 256) {
                for (int t = s_n + threadIdx.x; t < XK_BUF; t += blockDim.x) {
                    bv[t] = -INFINITY;
                    bj[t] = 0x7fffffff;
                }
                __syncthreads();
                bitonic_sort_desc(bv, bj, XK_BUF);
                if (threadIdx.x == 0) {
                    s_n = min(s_n, k);
                    if (s_n == k) {
                        s_thr_v = bv[k - 1];
                        s_thr_j = bj[k - 1];
                    }
                }
                __syncthreads();
            }
        }
        for (int t = s_n + threadIdx.x; t < XK_BUF; t += blockDim.x) {
            bv[t] = -INFINITY;
            bj[t] = 0x7fffffff;
        }
        __syncthreads();
        bitonic_sort_desc(bv, bj, XK_BUF);
        const int have = min(s_n, k);
        for (int t = threadIdx.x; t < k; t += blockDim.x) {
            if (out_idx) {
                out_idx[i * k + t] = t < have ? bj[t] : -1;
                out_score[i * k + t] = t < have ? (float)bv[t] : -INFINITY;
            }
        }
        if (kth_out && threadIdx.x == 0) kth_out[rr] = have == k ? bv[k - 1] : -INFINITY;
        __syncthreads();
    }
}

// Floor of the candidate sweep: F = min over pilot rows of their exact k-th
// similarity, minus twice the largest error bound of any approximate score.
// With few S rows every column is a candidate (F = -inf).
__global__ void topk_floor(unsigned long long* hdr, const double* __restrict__ kth, int n_pilot,
                           double fp32_terms, int all_columns) {
    if (threadIdx.x != 0) return;
    const double er = (double)__uint_as_float((uint32_t)hdr[H_ENORM_R]) * 1.001 + 1e-7;
    const double es = (double)__uint_as_float((uint32_t)hdr[H_ENORM_S]) * 1.001 + 1e-7;
    const double dmax = er * (1.0 + es) + es + fp32_terms * (1.0 + er) * (1.0 + es);
    double m = INFINITY;
    for (int p = 0; p < n_pilot; ++p) m = fmin(m, kth[p]);
    double F = m - 2.0 * dmax - 1e-6;
    if (all_columns || !(F > -1e30)) F = -INFINITY;
    float Ff = (float)F;
    if ((double)Ff > F) Ff = next_down(Ff);
    hdr[H_TOPK_F] = (unsigned long long)__float_as_uint(Ff);
    hdr[H_TOPK_EMAX] = (unsigned long long)__float_as_uint((float)dmax);
}

// Per-row finalize (one wave per row, Kc <= 256 candidate slots).
constexpr int FZ_SLOTS = 256;

// wave-level bitonic sort of 256 (key desc, j asc) entries in LDS
__device__ void wave_sort256(double* v, int* j) {
    const int lane = threadIdx.x & 63;
    for (int size = 2; size <= FZ_SLOTS; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < FZ_SLOTS / 2; t += 64) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);
                const bool hi_better = better(v[hi], j[hi], v[lo], j[lo]);
                if (hi_better == up) {
                    const double tv = v[lo];
                    v[lo] = v[hi];
                    v[hi] = tv;
                    const int tj = j[lo];
                    j[lo] = j[hi];
                    j[hi] = tj;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
}

__global__ __launch_bounds__(256) void topk_finalize(
    const float* __restrict__ R, int64_t ldR, const float* __restrict__ S, int64_t ldS, int dim,
    int64_t nR, int64_t nS, const double* __restrict__ nr64, const double* __restrict__ ns64,
    const RowInfo* __restrict__ info_r, const int* __restrict__ cnt,
    const int2* __restrict__ cand, int Kc, int k, double fp32_terms,
    unsigned long long* __restrict__ hdr, int* __restrict__ fb_rows,
    int32_t* __restrict__ out_idx, float* __restrict__ out_score) {
    __shared__ double sv[4][FZ_SLOTS];
    __shared__ int sj[4][FZ_SLOTS];
    if (hdr[H_FLAGS] != 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double* v = sv[wave];
    int* jv = sj[wave];
    const float F = __uint_as_float((uint32_t)hdr[H_TOPK_F]);
    const double es = (double)__uint_as_float((uint32_t)hdr[H_ENORM_S]) * 1.001 + 1e-7;
    const int kk = (int)min((int64_t)k, nS);

    for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < nR; i += (int64_t)gridDim.x * 4) {
        if (nS == 0) {  // nothing to join: every slot is padding
            for (int t = lane; t < k; t += 64) {
                out_idx[i * k + t] = -1;
                out_score[i * k + t] = -INFINITY;
            }
            continue;
        }
        const int c = cnt[i];
        const int n = min(c, Kc);
        const double er = (double)info_r[i].enorm * 1.001 + 1e-7;
        const double di = er * (1.0 + es) + es + fp32_terms * (1.0 + er) * (1.0 + es);
        // load the candidates (approximate score, index)
        for (int t = lane; t < FZ_SLOTS; t += 64) {
            if (t < n) {
                const int2 e = cand[i * (int64_t)Kc + t];
                v[t] = (double)__int_as_float(e.y);
                jv[t] = e.x;
            } else {
                v[t] = -INFINITY;
                jv[t] = 0x7fffffff;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        bool ok = c <= Kc;
        double lim = -INFINITY;
        if (ok) {
            if (F == -INFINITY) {
                ok = (int64_t)n == nS;  // every column present
            } else {
                ok = n >= kk;
                if (ok) {
                    wave_sort256(v, jv);
                    const double ak = v[kk - 1];
                    lim = ak - 2.0 * di;
                    ok = lim >= (double)F;
                }
            }
        }
        if (!ok) {
            if (lane == 0) {
                const unsigned long long p = atomicAdd(hdr + H_TOPK_FB, 1ull);
                fb_rows[p] = (int)i;
            }
            continue;
        }
        // rescore every candidate that can still be in the top k
        const float* r = R + i * ldR;
        const double nr = nr64[i];
        for (int t = lane; t < FZ_SLOTS; t += 64) {
            if (t < n && v[t] >= lim) {
                const int j = jv[t];
                v[t] = sim64_from(dot64_seq(r, S + (int64_t)j * ldS, dim), nr, ns64[j]);
            } else {
                v[t] = -INFINITY;
                jv[t] = 0x7fffffff;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        wave_sort256(v, jv);
        for (int t = lane; t < k; t += 64) {
            const bool have = t < kk;
            out_idx[i * k + t] = have ? jv[t] : -1;
            out_score[i * k + t] = have ? (float)v[t] : -INFINITY;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// pilot rows: evenly spaced sample of R
__global__ void pilot_rows(int* rows, int n_pilot, int64_t nR) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n_pilot) rows[p] = (int)(((int64_t)p * nR) / n_pilot);
}

hipError_t launch_norms64(const float* X, int64_t rows, int dim, int64_t ld, double* out,
                          hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    int64_t nb = (rows + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(norms64, dim3((unsigned)nb), dim3(256), 0, st, X, rows, dim, ld, out);
    return hipGetLastError();
}

hipError_t launch_topk_pilot(const TopkArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(pilot_rows, dim3((a.n_pilot + 255) / 256), dim3(256), 0, st, a.pilot_rows,
                       a.n_pilot, a.nR);
    hipLaunchKernelGGL(exact_topk_rows, dim3(a.n_pilot), dim3(256), 0, st, a.R, a.ldR, a.S, a.ldS,
                       a.dim, a.nS, a.nr64, a.ns64, a.k, (const int*)a.pilot_rows,
                       (const unsigned long long*)nullptr, a.n_pilot, (int32_t*)nullptr,
                       (float*)nullptr, a.pilot_kth);
    hipLaunchKernelGGL(topk_floor, dim3(1), dim3(64), 0, st, a.hdr, a.pilot_kth, a.n_pilot,
                       a.fp32_terms, a.all_columns ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_topk_finalize(const TopkArgs& a, hipStream_t st) {
    int64_t nb = (a.nR + 3) / 4;
    if (nb > 16384) nb = 16384;
    if (nb > 0)
        hipLaunchKernelGGL(topk_finalize, dim3((unsigned)nb), dim3(256), 0, st, a.R, a.ldR, a.S,
                           a.ldS, a.dim, a.nR, a.nS, a.nr64, a.ns64, a.info_r, a.cnt, a.cand,
                           a.Kc, a.k, a.fp32_terms, a.hdr, a.fb_rows, a.out_idx, a.out_score);
    // exact scan of the rows that failed the certificate (count read on the
    // device; a fixed grid loops over them)
    hipLaunchKernelGGL(exact_topk_rows, dim3(1024), dim3(256), 0, st, a.R, a.ldR, a.S, a.ldS,
                       a.dim, a.nS, a.nr64, a.ns64, a.k, (const int*)a.fb_rows,
                       (const unsigned long long*)(a.hdr + H_TOPK_FB), 0, a.out_idx,
                       a.out_score, (double*)nullptr);
    return hipGetLastError();
}

}  // namespace ej
