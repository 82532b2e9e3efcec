// topk.hip -- exact top-k E-join: candidate floor, certification, FP64
// rescoring and ordered selection.
//
// The top-k join condition (Section VI.E, the scan side of the scan-versus-
// probe study) asks, for every R tuple, for the k most similar S tuples.  The
// result here is exact with respect to the canonical FP64 similarity
// (sequential sums from the float32 inputs, dot / sqrt(|r|^2 |s|^2)), ordered
// by (similarity desc, S index asc):
//
//  1. a pilot computes the exact k-th similarity T_k of a few sample rows
//     (over a strided sample of the columns when S is large, which can only
//     lower T_k) and sets the candidate floor F = min T_k - 2 D (D: largest
//     error bound of the approximate scores);
//  2. the contraction sweep (panel kernel, candidate epilogue) stores every
//     column with approximate score a >= F in its row's candidate slots;
//  3. per row: A_k = k-th largest candidate score, D_i = the row's error
//     bound.  Any true top-k column j has a_ij >= A_k - 2 D_i.  If no slot
//     overflowed and A_k - 2 D_i >= F, every such column is a candidate: they
//     are rescored in FP64 and sorted, which gives the exact answer;
//  4. rows that fail the certificate take an exact FP64 scan of all S.
//
// All FP64 dot products keep the canonical sequential order.  Each thread
// owns one (row, column) dot; the column rows are staged through LDS in
// 32-float chunks loaded with coalesced reads, and every thread sums its own
// row chunk by chunk, so the order of the sum stays k = 0, 1, ..., d-1.
// Each step is one fused multiply-add: the product of two float32 values is
// exact in float64, so the single rounding is the sum's, as in the
// sequential definition.
#include <math.h>

#include "common.hpp"
#include "launch.hpp"

namespace ej {

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

// The m best of a wave's entries (v[t], j[t]), t < n <= 256, in LDS, by
// `better` (value, then the lower index), among those with v >= floor: m
// rounds each take the best entry not taken yet (a per-lane best of the
// lane's four entries, then across the wave); emit(r, v, j) receives the
// entry of rank r.  Stops early when fewer than m entries pass.  The indices
// are distinct (columns of one row).  Returns the number of ranks emitted.
// (k rounds instead of each entry counting the entries above it: O(k n)
// work instead of O(n^2).)
template <typename Emit>
__device__ __forceinline__ int wave_best_m(const double* v, const int* jv, int n, int m,
                                           double floor, Emit emit) {
    const int lane = threadIdx.x & 63;
    double mv[4];
    int mj[4];
    bool mine[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = lane + 64 * q;
        mine[q] = t < n;
        mv[q] = mine[q] ? v[t] : 0.0;
        mj[q] = mine[q] ? jv[t] : 0;
        mine[q] = mine[q] && mv[q] >= floor;
    }
    for (int r = 0; r < m; ++r) {
        bool found = false;
        double bv = 0.0;
        int bj = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (mine[q] && (!found || better(mv[q], mj[q], bv, bj))) {
                bv = mv[q];
                bj = mj[q];
                found = true;
            }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o, 64);
            const int oj = __shfl_xor(bj, o, 64);
            const bool of = __shfl_xor(found ? 1 : 0, o, 64) != 0;
            if (of && (!found || better(ov, oj, bv, bj))) {
                bv = ov;
                bj = oj;
                found = true;
            }
        }
        if (!found) return r;  // wave-uniform after the reduction
        emit(r, bv, bj);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (mine[q] && mj[q] == bj) mine[q] = false;
    }
    return m;
}

// ---------------------------------------------------------------------------
// block-wide canonical FP64 dots (256 threads)
// ---------------------------------------------------------------------------
constexpr int SD_CH = 32;
struct StageSmem {
    float tile[256][SD_CH + 1];  // +1: conflict-free column reads
    float rch[SD_CH];
    int64_t row_of[256];
};

// Thread t returns the sequential FP64 dot of X[row_of[t]] with r (with
// itself when r is null).  row_of[t] < 0: no row (returns 0).  Must be
// called by all 256 threads.
__device__ double block_dots(const float* __restrict__ X, int64_t ldX,
                             const float* __restrict__ r, int dim, StageSmem& sm) {
    const int tid = threadIdx.x;
    const int64_t mine = sm.row_of[tid];
    double acc = 0.0;
    for (int k0 = 0; k0 < dim; k0 += SD_CH) {
        const int kn = min(SD_CH, dim - k0);
        // 16 loads in flight per thread before their values go to LDS
        for (int q0 = 0; q0 < 256 * SD_CH; q0 += 16 * 256) {
            float vals[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int q = q0 + u * 256 + tid;
                const int ri = q / SD_CH, kk = q - ri * SD_CH;
                const int64_t row = sm.row_of[ri];
                vals[u] = (row >= 0 && kk < kn) ? X[row * ldX + k0 + kk] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int q = q0 + u * 256 + tid;
                const int ri = q / SD_CH, kk = q - ri * SD_CH;
                sm.tile[ri][kk] = vals[u];
            }
        }
        if (r && tid < kn) sm.rch[tid] = r[k0 + tid];
        __syncthreads();
        if (mine >= 0) {
            for (int kk = 0; kk < kn; ++kk) {
                const double a = (double)sm.tile[tid][kk];
                const double b = r ? (double)sm.rch[kk] : a;
                acc = __builtin_fma(a, b, acc);  // a * b exact in FP64
            }
        }
        __syncthreads();
    }
    return acc;
}

// bitonic sort of n_pow2 (v desc, j asc) entries in LDS by 256 threads
__device__ void bitonic_sort_desc(double* v, int* j, int n_pow2) {
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

// Squared FP64 norms of all rows, 256 rows per workgroup.
__global__ __launch_bounds__(256) void norms64(const float* __restrict__ X, int64_t rows, int dim,
                                               int64_t ld, double* __restrict__ out) {
    __shared__ StageSmem sm;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < rows; base += (int64_t)gridDim.x * 256) {
        const int64_t i = base + threadIdx.x;
        sm.row_of[threadIdx.x] = i < rows ? i : -1;
        __syncthreads();
        const double n = block_dots(X, ld, nullptr, dim, sm);
        if (i < rows) out[i] = n;
        __syncthreads();
    }
}

// Exact FP64 top-k of the rows in `rows_list` (one workgroup per row).  A
// 512-entry buffer collects every column that beats the current k-th best;
// when it fills it is sorted and cut to k.  k <= 256.
constexpr int XK_BUF = 512;

//
// The S columns may be split into n_rg ranges (blockIdx.y): each workgroup
// then writes its range's top-k of list entry rr to part_v/part_j at
// [(rr - row_base) * n_rg + range] * k, and exact_topk_merge combines them.
// With n_rg == 1 the list's rows are written to the outputs directly.
__global__ __launch_bounds__(256) void exact_topk_rows(
    const float* __restrict__ R, int64_t ldR, const float* __restrict__ S, int64_t ldS, int dim,
    int64_t nS, const double* __restrict__ nr64, const double* __restrict__ ns64, int k,
    const int* __restrict__ rows_list, const unsigned long long* __restrict__ n_rows_ptr,
    int n_rows_fixed, int row_base, int row_limit, int32_t* __restrict__ out_idx,
    float* __restrict__ out_score, double* __restrict__ kth_out, double* __restrict__ part_v,
    int* __restrict__ part_j, int col_stride, double min_sim) {
    __shared__ StageSmem sm;
    __shared__ double bv[XK_BUF];
    __shared__ int bj[XK_BUF];
    __shared__ int s_n;
    __shared__ double s_thr_v;
    __shared__ int s_thr_j;
    __shared__ int s_wcnt[4];

    const int n_rows_all = n_rows_ptr ? (int)*n_rows_ptr : n_rows_fixed;
    const int n_rows = min(n_rows_all, row_limit);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // the scanned columns are c * col_stride for c < n_col (every column
    // with col_stride 1), split into n_rg ranges of c
    const int64_t n_col = (nS + col_stride - 1) / col_stride;
    const int n_rg = gridDim.y, rg = blockIdx.y;
    const int64_t per = (n_col + n_rg - 1) / n_rg;
    const int64_t s_lo = rg * per, s_hi = min(n_col, s_lo + per);
    for (int rr = row_base + blockIdx.x; rr < n_rows; rr += gridDim.x) {
        const int64_t i = rows_list[rr];
        const float* r = R + i * ldR;
        const double nr = nr64[i];
        if (threadIdx.x == 0) {
            s_n = 0;
            s_thr_v = -INFINITY;
            s_thr_j = 0x7fffffff;
        }
        __syncthreads();
        for (int64_t c0 = s_lo; c0 < s_hi; c0 += 256) {
            const int64_t jj = (c0 + threadIdx.x) * col_stride;
            sm.row_of[threadIdx.x] = c0 + threadIdx.x < s_hi ? jj : -1;
            __syncthreads();
            const double dot = block_dots(S, ldS, r, dim, sm);
            double v = -INFINITY;
            bool cand = false;
            if (c0 + threadIdx.x < s_hi) {
                v = sim64_from(dot, nr, ns64[jj]);
                cand = v >= min_sim && better(v, (int)jj, s_thr_v, s_thr_j);
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
        if (part_v) {
            const int64_t o = ((int64_t)(rr - row_base) * n_rg + rg) * k;
            for (int t = threadIdx.x; t < k; t += blockDim.x) {
                part_v[o + t] = t < have ? bv[t] : -INFINITY;
                part_j[o + t] = t < have ? bj[t] : 0x7fffffff;
            }
        } else {
            for (int t = threadIdx.x; t < k; t += blockDim.x) {
                if (out_idx) {
                    out_idx[i * k + t] = t < have ? bj[t] : -1;
                    out_score[i * k + t] = t < have ? (float)bv[t] : -INFINITY;
                }
            }
            if (kth_out && threadIdx.x == 0) kth_out[rr] = have == k ? bv[k - 1] : -INFINITY;
        }
        __syncthreads();
    }
}

// Combine the per-range lists of exact_topk_rows (one workgroup per list
// entry): the exact top-k of the row is the top-k of the union.
__global__ __launch_bounds__(256) void exact_topk_merge(
    const int* __restrict__ rows_list, const unsigned long long* __restrict__ n_rows_ptr,
    int n_rows_fixed, int row_base, int row_limit, int n_rg, int k, int64_t nS,
    const double* __restrict__ part_v, const int* __restrict__ part_j,
    int32_t* __restrict__ out_idx, float* __restrict__ out_score, double* __restrict__ kth_out) {
    __shared__ double bv[XK_BUF];
    __shared__ int bj[XK_BUF];
    const int n_rows_all = n_rows_ptr ? (int)*n_rows_ptr : n_rows_fixed;
    const int n_rows = min(n_rows_all, row_limit);
    for (int rr = row_base + blockIdx.x; rr < n_rows; rr += gridDim.x) {
        const int64_t i = rows_list[rr];
        const int64_t o = (int64_t)(rr - row_base) * n_rg * k;
        int n = 0;  // entries held (block-uniform)
        for (int g = 0; g < n_rg; ++g) {
            for (int t = threadIdx.x; t < k; t += blockDim.x) {
                bv[n + t] = part_v[o + (int64_t)g * k + t];
                bj[n + t] = part_j[o + (int64_t)g * k + t];
            }
            n += k;
            __syncthreads();
            if (n > XK_BUF - k || g == n_rg - 1) {
                for (int t = n + threadIdx.x; t < XK_BUF; t += blockDim.x) {
                    bv[t] = -INFINITY;
                    bj[t] = 0x7fffffff;
                }
                __syncthreads();
                bitonic_sort_desc(bv, bj, XK_BUF);
                n = k;
            }
        }
        // sorted descending: the entries are the finite ones (the ranges'
        // lists hold only columns that passed the minimum similarity)
        (void)nS;
        for (int t = threadIdx.x; t < k; t += blockDim.x) {
            if (out_idx) {
                const bool have = bv[t] > -INFINITY;
                out_idx[i * k + t] = have ? bj[t] : -1;
                out_score[i * k + t] = have ? (float)bv[t] : -INFINITY;
            }
        }
        if (kth_out && threadIdx.x == 0) kth_out[rr] = bv[k - 1];
        __syncthreads();
    }
}

// Floor of the candidate sweep: F = min over pilot rows of their exact k-th
// similarity, minus twice the largest error bound of any approximate score.
// With few S rows every column is a candidate (F = -inf).
__global__ void topk_floor(unsigned long long* hdr, const double* __restrict__ kth, int n_pilot,
                           double fp32_terms, int all_columns, double min_sim) {
    if (threadIdx.x != 0) return;
    const double er = (double)__uint_as_float((uint32_t)hdr[H_ENORM_R]) * 1.001 + 1e-7;
    const double es = (double)__uint_as_float((uint32_t)hdr[H_ENORM_S]) * 1.001 + 1e-7;
    const double dmax = er * (1.0 + es) + es + fp32_terms * (1.0 + er) * (1.0 + es);
    double m = INFINITY;
    for (int p = 0; p < n_pilot; ++p) m = fmin(m, kth[p]);
    double F = m - 2.0 * dmax - 1e-6;
    // a column with sim64 >= min_sim has an approximate score >= min_sim - dmax
    if (min_sim > -INFINITY) F = fmax(F, min_sim - dmax - 1e-6);
    if (all_columns || !(F > -1e30)) F = -INFINITY;
    float Ff = (float)F;
    if ((double)Ff > F) Ff = next_down(Ff);
    hdr[H_TOPK_F] = (unsigned long long)__float_as_uint(Ff);
    hdr[H_TOPK_EMAX] = (unsigned long long)__float_as_uint((float)dmax);
}

// ---------------------------------------------------------------------------
// finalize order: rows grouped by their best candidate, so that rows with the
// same neighbourhood rescore the same S rows one after the other (L2 reuse)
// ---------------------------------------------------------------------------
__global__ void fill_int(int* p, int64_t n, int v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// key[i] = smallest candidate index of row i (nS if none); counts[key]++.
// Rows whose candidate sets coincide (one neighbourhood) get the same key.
// Nothing runs after a failed input check: the sweep then left the candidate
// counters unwritten.
__global__ __launch_bounds__(256) void topk_keys(const int* __restrict__ cnt,
                                                 const int2* __restrict__ cand, int Kc,
                                                 int64_t nR, int64_t nS, int* __restrict__ key,
                                                 int* __restrict__ counts,
                                                 const unsigned long long* __restrict__ hdr) {
    if (hdr[H_FLAGS] != 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t i = (int64_t)blockIdx.x * 4 + wave; i < nR; i += (int64_t)gridDim.x * 4) {
        const int n = max(0, min(cnt[i], Kc));
        int bj = (int)nS;
        for (int t = lane; t < n; t += 64) bj = min(bj, cand[i * (int64_t)Kc + t].x);
        for (int o = 32; o > 0; o >>= 1) bj = min(bj, __shfl_xor(bj, o, 64));
        bj = max(bj, 0);  // candidate columns lie in [0, nS)
        if (lane == 0) {
            key[i] = bj;
            atomicAdd(counts + bj, 1);
        }
    }
}

// exclusive scan of counts[0..n) in place (one workgroup)
__global__ __launch_bounds__(256) void scan_counts(int* counts, int64_t n) {
    __shared__ int part[256];
    const int64_t per = (n + 255) / 256;
    const int64_t b = threadIdx.x * per, e = min(n, b + per);
    int s = 0;
    for (int64_t q = b; q < e; ++q) s += counts[q];
    part[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int t = 0; t < 256; ++t) {
            const int v = part[t];
            part[t] = acc;
            acc += v;
        }
    }
    __syncthreads();
    int acc = part[threadIdx.x];
    for (int64_t q = b; q < e; ++q) {
        const int v = counts[q];
        counts[q] = acc;
        acc += v;
    }
}

__global__ void scatter_order(const int* __restrict__ key, int64_t nR, int* __restrict__ offs,
                              int* __restrict__ order, const unsigned long long* __restrict__ hdr) {
    if (hdr[H_FLAGS] != 0) return;  // keys were not written
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nR;
         i += (int64_t)gridDim.x * blockDim.x)
        order[atomicAdd(offs + key[i], 1)] = (int)i;
}

// ---------------------------------------------------------------------------
// per-row finalize: one workgroup per row, Kc <= 256 candidate slots
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void topk_finalize(
    const float* __restrict__ R, int64_t ldR, const float* __restrict__ S, int64_t ldS, int dim,
    int64_t nR, int64_t nS, const double* __restrict__ nr64, const double* __restrict__ ns64,
    const RowInfo* __restrict__ info_r, const int* __restrict__ cnt,
    const int2* __restrict__ cand, int Kc, int k, double fp32_terms,
    const int* __restrict__ order, unsigned long long* __restrict__ hdr,
    int* __restrict__ fb_rows, int32_t* __restrict__ out_idx, float* __restrict__ out_score) {
    __shared__ StageSmem sm;
    __shared__ double v[256];
    __shared__ int jv[256];
    if (hdr[H_FLAGS] != 0) return;
    const int tid = threadIdx.x;
    const float F = __uint_as_float((uint32_t)hdr[H_TOPK_F]);
    const double es = (double)__uint_as_float((uint32_t)hdr[H_ENORM_S]) * 1.001 + 1e-7;
    const int kk = (int)min((int64_t)k, nS);

    for (int64_t rr = blockIdx.x; rr < nR; rr += gridDim.x) {
        const int64_t i = order ? order[rr] : rr;
        if (nS == 0) {  // nothing to join: every slot is padding
            for (int t = tid; t < k; t += 256) {
                out_idx[i * k + t] = -1;
                out_score[i * k + t] = -INFINITY;
            }
            continue;
        }
        const int c = cnt[i];
        const int n = min(c, Kc);
        const double er = (double)info_r[i].enorm * 1.001 + 1e-7;
        const double di = er * (1.0 + es) + es + fp32_terms * (1.0 + er) * (1.0 + es);
        if (tid < n) {
            const int2 e = cand[i * (int64_t)Kc + tid];
            v[tid] = (double)__int_as_float(e.y);
            jv[tid] = e.x;
        } else {
            v[tid] = -INFINITY;
            jv[tid] = 0x7fffffff;
        }
        __syncthreads();
        bool ok = c <= Kc;
        double lim = -INFINITY;
        if (ok) {
            if (F == -INFINITY) {
                ok = (int64_t)n == nS;  // every column present
            } else {
                ok = n >= kk;
                if (ok) {
                    bitonic_sort_desc(v, jv, 256);
                    lim = v[kk - 1] - 2.0 * di;
                    ok = lim >= (double)F;
                }
            }
        }
        if (!ok) {  // uniform: every value above is block-uniform
            if (tid == 0) {
                const unsigned long long p = atomicAdd(hdr + H_TOPK_FB, 1ull);
                fb_rows[p] = (int)i;
            }
            __syncthreads();
            continue;
        }
        // rescore every candidate that can still be in the top k
        const bool live = tid < n && v[tid] >= lim;
        sm.row_of[tid] = live ? (int64_t)jv[tid] : -1;
        __syncthreads();
        const double dot = block_dots(S, ldS, R + i * ldR, dim, sm);
        const double sim = live ? sim64_from(dot, nr64[i], ns64[jv[tid]]) : -INFINITY;
        __syncthreads();
        v[tid] = sim;
        if (!live) jv[tid] = 0x7fffffff;
        __syncthreads();
        bitonic_sort_desc(v, jv, 256);
        for (int t = tid; t < k; t += 256) {
            const bool have = t < kk;
            out_idx[i * k + t] = have ? jv[t] : -1;
            out_score[i * k + t] = have ? (float)v[t] : -INFINITY;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// wave-per-row finalize
// ---------------------------------------------------------------------------
// One wave owns one R row: no workgroup barriers.  The k-th best candidate
// and the final order come from ranks (each lane counts the entries that beat
// its own); the FP64 dots stage the row chunk and the 64 candidate rows of a
// pass through the wave's LDS, so global reads are whole row segments while
// each lane keeps the sequential order of its own sum.
constexpr int FW_WAVES = 4;
constexpr int FW_CH = 32;
constexpr int FW_STRIDE = FW_CH + 1;

struct alignas(16) FinSmem {
    double v[FW_WAVES][256];
    int j[FW_WAVES][256];
    int live[FW_WAVES][256];
    float rows[FW_WAVES][64 * FW_STRIDE];
    float rch[FW_WAVES][FW_CH];
    double lim[FW_WAVES];
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

typedef __attribute__((address_space(1))) const float* gfloat_ptr;

// Lane l: sequential FP64 dot of the row `r` with S row live[p0 + l] (lanes
// with p0 + l >= n_live get 0; p0 < n_live).  Candidate chunks of 32
// elements go through LDS, two candidate rows per load instruction (lanes
// 0-31 one, 32-63 the next) at the row the lane half reads from the live list,
// all 32 loads of a chunk in flight together.  Chunk entries past dim are
// zero on both sides, so the unrolled sum adds exact zeros: the sequential
// FP64 sum over k < dim is unchanged.
__device__ __forceinline__ double wave_dot64(const float* __restrict__ r,
                                             const float* __restrict__ S, int64_t ldS,
                                             const int* live, int p0, int n_live, int dim,
                                             float* rows, float* rch) {
    const int lane = threadIdx.x & 63;
    const int kk = lane & 31, hl = lane >> 5;
    const gfloat_ptr Sg = (gfloat_ptr)S;
    double acc = 0.0;
    for (int k0 = 0; k0 < dim; k0 += FW_CH) {
        const int kn = min(FW_CH, dim - k0);
        if (lane < FW_CH) rch[lane] = lane < kn ? r[k0 + lane] : 0.0f;
        const bool kin = kk < kn;
        const int kq = k0 + (kin ? kk : 0);
        float vals[32];
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            const int i = p0 + 2 * q + hl;
            const bool have = i < n_live;
            const int c = live[have ? i : p0];
            const float x = Sg[(int64_t)c * ldS + kq];
            vals[q] = (have && kin) ? x : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < 32; ++q) rows[(2 * q + hl) * FW_STRIDE + kk] = vals[q];
        wave_sync();
        const float* mine = rows + lane * FW_STRIDE;
#pragma unroll
        for (int q = 0; q < FW_CH; ++q)
            acc = __builtin_fma((double)rch[q], (double)mine[q], acc);  // exact product
        wave_sync();
    }
    return p0 + lane < n_live ? acc : 0.0;
}

// The four waves of a workgroup take four consecutive rows of the
// neighbourhood order, which mostly share their candidates.  When every wave
// with live candidates holds the same live list, the workgroup rescores that
// list together: each wave loads a quarter of every candidate chunk into LDS
// and all four multiply it with their own row, so each candidate row is read
// once per workgroup instead of once per wave.  Otherwise every wave rescores
// its own list (wave_dot64).  Each lane's FP64 sum keeps the sequential order
// of the canonical definition in both cases.
__global__ __launch_bounds__(256) void topk_finalize_w(
    const float* __restrict__ R, int64_t ldR, const float* __restrict__ S, int64_t ldS, int dim,
    int64_t nR, int64_t nS, const double* __restrict__ nr64, const double* __restrict__ ns64,
    const RowInfo* __restrict__ info_r, const int* __restrict__ cnt,
    const int2* __restrict__ cand, int Kc, int k, double fp32_terms,
    const int* __restrict__ order, unsigned long long* __restrict__ hdr,
    int* __restrict__ fb_rows, int32_t* __restrict__ out_idx, float* __restrict__ out_score,
    const float* __restrict__ floors, int64_t n_rows, double min_sim) {
    __shared__ FinSmem sm;
    __shared__ int s_nl[FW_WAVES], s_same[FW_WAVES];
    if (hdr[H_FLAGS] != 0) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double* v = sm.v[w];
    int* jv = sm.j[w];
    int* live = sm.live[w];
    const float F0 = __uint_as_float((uint32_t)hdr[H_TOPK_F]);
    const double es = (double)__uint_as_float((uint32_t)hdr[H_ENORM_S]) * 1.001 + 1e-7;
    const int kk = (int)min((int64_t)k, nS);

    // With a minimum similarity (min_sim > -inf) only columns with
    // sim64 >= min_sim count: a certified row needs every such column of its
    // top k among its candidates, i.e. no overflow and the larger of
    // (k-th candidate score - 2 D_i) and (min_sim - D_i) at or above the
    // floor; fewer than k passing columns are then a complete answer.
    // workgroup-uniform loop: the barriers below need all four waves.  Rows
    // order[0 .. n_rows) (all rows without an order); with `floors` the
    // candidates of position rr were swept with floor floors[rr].
    for (int64_t base = (int64_t)blockIdx.x * FW_WAVES; base < n_rows;
         base += (int64_t)gridDim.x * FW_WAVES) {
        const int64_t rr = base + w;
        int n_live = 0;  // wave-uniform: candidates this wave rescores
        bool done = false;  // wave-uniform: the row is certified (outputs below)
        int64_t i = 0;
        if (rr < n_rows) {
            i = order ? order[rr] : rr;
            const float F = floors ? floors[rr] : F0;
            if (nS == 0) {  // nothing to join: every slot is padding
                for (int t = lane; t < k; t += 64) {
                    out_idx[i * k + t] = -1;
                    out_score[i * k + t] = -INFINITY;
                }
            } else {
                const int c = cnt[i];
                const int n = min(c, Kc);
                const double er = (double)info_r[i].enorm * 1.001 + 1e-7;
                const double di = er * (1.0 + es) + es + fp32_terms * (1.0 + er) * (1.0 + es);
                for (int t = lane; t < 256; t += 64) {
                    if (t < n) {
                        const int2 e = cand[i * (int64_t)Kc + t];
                        v[t] = (double)__int_as_float(e.y);
                        jv[t] = e.x;
                    } else {
                        v[t] = -INFINITY;
                        jv[t] = 0x7fffffff;
                    }
                }
                if (lane == 0) sm.lim[w] = -INFINITY;
                wave_sync();
                bool ok = c <= Kc;
                if (ok) {
                    if (F == -INFINITY) {
                        ok = (int64_t)n == nS;  // every column present
                    } else {
                        if (n >= kk) {
                            // the entry of rank kk-1 among the n candidates
                            if (kk <= 32) {
                                wave_best_m(v, jv, n, kk, -INFINITY, [&](int r, double bv, int) {
                                    if (r == kk - 1 && lane == 0) sm.lim[w] = bv - 2.0 * di;
                                });
                            } else {
                                for (int t = lane; t < n; t += 64) {
                                    const double vt = v[t];
                                    const int jt = jv[t];
                                    int rank = 0;
                                    for (int u = 0; u < n; ++u)
                                        rank += better(v[u], jv[u], vt, jt);
                                    if (rank == kk - 1) sm.lim[w] = vt - 2.0 * di;
                                }
                            }
                            wave_sync();
                        }
                        if (min_sim > -INFINITY && lane == 0)
                            sm.lim[w] = fmax(sm.lim[w], min_sim - di);
                        wave_sync();
                        ok = sm.lim[w] >= (double)F;
                    }
                }
                if (!ok) {  // wave-uniform
                    if (lane == 0) {
                        const unsigned long long p = atomicAdd(hdr + H_TOPK_FB, 1ull);
                        fb_rows[p] = (int)i;
                    }
                } else {
                    done = true;
                    const double lim = sm.lim[w];
                    // compact the candidates that can still be in the top k
                    for (int t0 = 0; t0 < n; t0 += 64) {
                        const int t = t0 + lane;
                        const bool lv = t < n && v[t] >= lim;
                        const uint64_t m = __ballot(lv);
                        if (lv) live[n_live + lanes_below(m)] = jv[t];
                        n_live += __popcll(m);
                    }
                }
            }
        }
        if (lane == 0) s_nl[w] = n_live;
        __syncthreads();
        // shared list: that of the first wave with one, if every other wave
        // with a list holds the same
        int ref = -1;
        for (int u = 0; u < FW_WAVES; ++u)
            if (ref < 0 && s_nl[u] > 0) ref = u;
        if (n_live > 0) {
            bool same = n_live == s_nl[ref];
            if (same && w != ref) {
                const int* L = sm.live[ref];
                bool eq = true;
                for (int t = lane; t < n_live; t += 64) eq = eq && live[t] == L[t];
                same = __ballot(!eq) == 0;
            }
            if (lane == 0) s_same[w] = same ? 1 : 0;
        } else if (lane == 0) {
            s_same[w] = 1;
        }
        __syncthreads();
        const bool coop =
            ref >= 0 && s_same[0] && s_same[1] && s_same[2] && s_same[3];  // workgroup-uniform
        const float* rrow = R + i * ldR;
        if (coop) {
            const int n = s_nl[ref];
            const int* L = sm.live[ref];
            // two chunk buffers (the candidate chunks of the workgroup and
            // this wave's row chunk): chunk c + 1 is loaded while chunk c is
            // multiplied.  The candidate chunks stay float32 in LDS (36
            // floats per candidate: 16-byte reads of 16 lanes hit 16
            // different bank groups) and are widened as each lane reads
            // them; the row chunk is widened once, when stored
            constexpr int FWS = FW_CH + 4;
            static_assert(2 * 64 * FWS * sizeof(float) <= sizeof(sm.rows),
                          "chunk buffers do not fit");
            float* const rows0 = &sm.rows[0][0];
            float* const rows1 = rows0 + 64 * FWS;
            __shared__ double s_rch[2][FW_WAVES][FW_CH];
            double* const rch0 = s_rch[0][w];
            double* const rch1 = s_rch[1][w];
            const int kk2 = lane & 31;
            const int nch = (dim + FW_CH - 1) / FW_CH;
            // Two chunks' loads in flight, in two register sets used in turn
            // (the loop is unrolled by two).  Every load is issued, so that
            // the compiler can wait for one chunk while the next loads: past
            // the pass's candidates, the row's end or the last chunk the
            // loads repeat valid addresses and the values are zeroed when
            // stored.  This wave's 16 of the pass's 64 candidate rows, two
            // rows per load instruction (lanes 0-31 one, 32-63 the next).
            auto load = [&](int p0, int c, float (&vals)[8], float& rv) {
                const int k0 = min(c, nch - 1) * FW_CH;
                rv = rrow[min(k0 + kk2, dim - 1)];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int tb = min(p0 + 16 * w + 2 * q + (lane >> 5), n - 1);
                    vals[q] = S[(int64_t)L[tb] * ldS + min(k0 + kk2, dim - 1)];
                }
            };
            auto store = [&](int p0, int c, const float (&vals)[8], float rv) {
                const int k0 = c * FW_CH;
                const bool in_row = k0 + kk2 < dim;
                float* r = (c & 1) ? rows1 : rows0;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int tb = p0 + 16 * w + 2 * q + (lane >> 5);
                    r[(16 * w + 2 * q + (lane >> 5)) * FWS + kk2] =
                        (tb < n && in_row) ? vals[q] : 0.0f;
                }
                if (lane < FW_CH)
                    ((c & 1) ? rch1 : rch0)[lane] = (n_live > 0 && in_row) ? (double)rv : 0.0;
            };
            auto dot_chunk = [&](int c, bool valid, double& acc) {
                if (n_live > 0 && valid) {
                    typedef float v4f __attribute__((ext_vector_type(4)));
                    const v4f* mine = (const v4f*)(((c & 1) ? rows1 : rows0) + lane * FWS);
                    const double* rc = (c & 1) ? rch1 : rch0;
                    // (the chunks are zero past dim: the extra terms add exact zeros;
                    // the products of the widened float32 values are exact)
#pragma unroll
                    for (int q4 = 0; q4 < FW_CH / 4; ++q4) {
                        const v4f m = mine[q4];
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc = __builtin_fma(rc[4 * q4 + e], (double)m[e], acc);
                    }
                }
            };
            float va[8], vb[8];
            float ra, rb;
            for (int p0 = 0; p0 < n; p0 += 64) {
                const int t = p0 + lane;
                const bool valid = t < n;
                double acc = 0.0;
                load(p0, 0, va, ra);
                load(p0, 1, vb, rb);
                store(p0, 0, va, ra);
                __syncthreads();
                // buffer (c + 1) & 1 is written after chunk c is multiplied;
                // it was last read for chunk c - 1, before the previous barrier
                for (int c = 0; c < nch; c += 2) {
                    load(p0, c + 2, va, ra);
                    dot_chunk(c, valid, acc);
                    if (c + 1 < nch) store(p0, c + 1, vb, rb);
                    __syncthreads();
                    if (c + 1 >= nch) break;
                    load(p0, c + 3, vb, rb);
                    dot_chunk(c + 1, valid, acc);
                    if (c + 2 < nch) store(p0, c + 2, va, ra);
                    __syncthreads();
                }
                if (n_live > 0 && valid) {
                    const int sj = L[t];
                    v[t] = sim64_from(acc, nr64[i], ns64[sj]);
                    jv[t] = sj;
                }
            }
        } else if (n_live > 0) {
            // FP64 rescore of this wave's live candidates, 64 per pass
            for (int p0 = 0; p0 < n_live; p0 += 64) {
                const int t = p0 + lane;
                const bool valid = t < n_live;
                const int sj = valid ? live[t] : 0;
                const double dot =
                    wave_dot64(rrow, S, ldS, live, p0, n_live, dim, sm.rows[w], sm.rch[w]);
                if (valid) {
                    v[t] = sim64_from(dot, nr64[i], ns64[sj]);
                    jv[t] = sj;
                }
            }
        }
        if (done) {
            wave_sync();
            // final order by rank among the live entries that pass min_sim
            int n_pass = 0;
            if (kk <= 32) {
                n_pass = wave_best_m(v, jv, n_live, kk, min_sim, [&](int r, double bv, int bj) {
                    if (lane == 0) {
                        out_idx[i * k + r] = bj;
                        out_score[i * k + r] = (float)bv;
                    }
                });
            } else {
                for (int t = lane; t < n_live; t += 64) {
                    const double vt = v[t];
                    if (!(vt >= min_sim)) continue;
                    ++n_pass;
                    const int jt = jv[t];
                    int rank = 0;
                    for (int u = 0; u < n_live; ++u)
                        rank += v[u] >= min_sim && better(v[u], jv[u], vt, jt);
                    if (rank < kk) {
                        out_idx[i * k + rank] = jt;
                        out_score[i * k + rank] = (float)vt;
                    }
                }
                for (int o = 32; o > 0; o >>= 1) n_pass += __shfl_xor(n_pass, o, 64);
            }
            for (int t = min(kk, n_pass) + lane; t < k; t += 64) {
                out_idx[i * k + t] = -1;
                out_score[i * k + t] = -INFINITY;
            }
        }
        __syncthreads();  // the lists and buffers are reused by the next rows
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

// number of S ranges per exact row scan (enough workgroups per row to use
// the GPU, with the merged lists fitting the merge buffer in a few rounds)
static int exact_ranges(int64_t nS) {
    int64_t g = (nS + 4095) / 4096;
    if (g > 64) g = 64;
    if (g < 1) g = 1;
    return (int)g;
}

// exact top-k of list entries [row_base, row_base + n) (n <= part rows)
// (col_stride > 1: over the columns c * col_stride only)
static hipError_t exact_topk_batch(const TopkArgs& a, const int* rows,
                                   const unsigned long long* n_ptr, int n_fixed, int row_base,
                                   int n_rows_max, int32_t* oi, float* os, double* kth,
                                   hipStream_t st, int col_stride = 1,
                                   double min_sim = -INFINITY) {
    const int64_t n_col = (a.nS + col_stride - 1) / col_stride;
    const int n_rg = exact_ranges(n_col);
    hipLaunchKernelGGL(exact_topk_rows, dim3(n_rows_max, n_rg), dim3(256), 0, st, a.R, a.ldR,
                       a.S, a.ldS, a.dim, a.nS, a.nr64, a.ns64, a.k, rows, n_ptr, n_fixed,
                       row_base, row_base + n_rows_max, (int32_t*)nullptr, (float*)nullptr,
                       (double*)nullptr, a.part_v, a.part_j, col_stride, min_sim);
    hipLaunchKernelGGL(exact_topk_merge, dim3(n_rows_max), dim3(256), 0, st, rows, n_ptr,
                       n_fixed, row_base, row_base + n_rows_max, n_rg, a.k, n_col,
                       (const double*)a.part_v, (const int*)a.part_j, oi, os, kth);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int, dim3(1024), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_topk_pilot(const TopkArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(pilot_rows, dim3((a.n_pilot + 255) / 256), dim3(256), 0, st, a.pilot_rows,
                       a.n_pilot, a.nR);
    // the pilot scans every 4th column of a large S: the k-th similarity over
    // that sample is a lower bound of the k-th over all of S, and any floor
    // keeps the result exact (a lower floor only admits more candidates)
    const int stride = a.nS >= 65536 ? 4 : 1;
    hipError_t e = exact_topk_batch(a, a.pilot_rows, nullptr, a.n_pilot, 0, a.n_pilot, nullptr,
                                    nullptr, a.pilot_kth, st, stride);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(topk_floor, dim3(1), dim3(64), 0, st, a.hdr, a.pilot_kth, a.n_pilot,
                       a.fp32_terms, a.all_columns ? 1 : 0, a.min_sim);
    return hipGetLastError();
}

hipError_t launch_topk_finalize(const TopkArgs& a, hipStream_t st) {
    if (a.nR <= 0) return hipSuccess;
    const int* order = nullptr;
    if (a.nS > 0) {
        // rows grouped by their best candidate
        hipLaunchKernelGGL(fill_int, dim3(256), dim3(256), 0, st, a.counts, a.nS + 1, 0);
        int64_t nb = (a.nR + 3) / 4;
        if (nb > 16384) nb = 16384;
        hipLaunchKernelGGL(topk_keys, dim3((unsigned)nb), dim3(256), 0, st, a.cnt, a.cand, a.Kc,
                           a.nR, a.nS, a.keys, a.counts, (const unsigned long long*)a.hdr);
        hipLaunchKernelGGL(scan_counts, dim3(1), dim3(256), 0, st, a.counts, a.nS + 1);
        hipLaunchKernelGGL(scatter_order, dim3(1024), dim3(256), 0, st, a.keys, a.nR, a.counts,
                           a.order, (const unsigned long long*)a.hdr);
        order = a.order;
    }
    int64_t nb = (a.nR + FW_WAVES - 1) / FW_WAVES;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(topk_finalize_w, dim3((unsigned)nb), dim3(256), 0, st, a.R, a.ldR, a.S,
                       a.ldS, a.dim, a.nR, a.nS, a.nr64, a.ns64, a.info_r, a.cnt, a.cand, a.Kc,
                       a.k, a.fp32_terms, order, a.hdr, a.fb_rows, a.out_idx, a.out_score,
                       (const float*)nullptr, a.nR, a.min_sim);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// refinement of rows whose candidate slots overflowed
// ---------------------------------------------------------------------------
// A row that saw more than Kc columns at or above the global floor F holds
// Kc of them (whichever came first).  Their k-th best approximate score A'_k
// is at most the row's k-th best over all columns A_k, and every column of
// the exact top k has an approximate score >= A_k - 2 D_i >= A'_k - 2 D_i,
// so F_i = A'_k - 2 D_i (rounded down to float) is a valid floor for that
// row alone, usually far above F.  One wave per listed row: rows that
// overflowed get F_i and their counter reset; the others (too few good
// candidates: no better floor exists) get +inf and keep their state, so the
// second finalize sends them to the exact scan again.
__global__ __launch_bounds__(256) void topk_refine_floor(
    const int* __restrict__ rows, int64_t n, int* __restrict__ cnt,
    const int2* __restrict__ cand, int Kc, int k, int64_t nS,
    const RowInfo* __restrict__ info_r, double fp32_terms,
    const unsigned long long* __restrict__ hdr, float* __restrict__ floors, double min_sim) {
    __shared__ double sv[4][256];
    __shared__ int sj[4][256];
    __shared__ double s_lim[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double es = (double)__uint_as_float((uint32_t)hdr[H_ENORM_S]) * 1.001 + 1e-7;
    const int kk = (int)min((int64_t)k, nS);
    for (int64_t c = (int64_t)blockIdx.x * 4 + w; c < n; c += (int64_t)gridDim.x * 4) {
        const int64_t i = rows[c];
        const int cn = cnt[i];
        if (cn <= Kc) {  // wave-uniform
            if (lane == 0) floors[c] = INFINITY;
            continue;
        }
        for (int t = lane; t < Kc; t += 64) {
            const int2 e = cand[i * (int64_t)Kc + t];
            sv[w][t] = (double)__int_as_float(e.y);
            sj[w][t] = e.x;
        }
        if (lane == 0) s_lim[w] = -INFINITY;
        wave_sync();
        for (int t = lane; t < Kc; t += 64) {
            const double vt = sv[w][t];
            const int jt = sj[w][t];
            int rank = 0;
            for (int u = 0; u < Kc; ++u) rank += better(sv[w][u], sj[w][u], vt, jt);
            if (rank == kk - 1) s_lim[w] = vt;
        }
        wave_sync();
        if (lane == 0) {
            const double er = (double)info_r[i].enorm * 1.001 + 1e-7;
            const double di = er * (1.0 + es) + es + fp32_terms * (1.0 + er) * (1.0 + es);
            const double f = fmax(s_lim[w] - 2.0 * di, min_sim - di);
            float ff = (float)f;
            if ((double)ff > f) ff = next_down(ff);
            floors[c] = ff;
            cnt[i] = 0;
        }
        wave_sync();
    }
}

hipError_t launch_topk_refine_floor(const TopkArgs& a, const int* rows, int64_t n, float* floors,
                                    hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + 3) / 4;
    if (nb > 16384) nb = 16384;
    hipLaunchKernelGGL(topk_refine_floor, dim3((unsigned)nb), dim3(256), 0, st, rows, n,
                       (int*)a.cnt, a.cand, a.Kc, a.k, a.nS, a.info_r, a.fp32_terms,
                       (const unsigned long long*)a.hdr, floors, a.min_sim);
    return hipGetLastError();
}

// The second finalize: rows order[0 .. n) swept with per-position floors.
hipError_t launch_topk_finalize_rows(const TopkArgs& a, const int* order, int64_t n,
                                     const float* floors, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t nb = (n + FW_WAVES - 1) / FW_WAVES;
    if (nb > 65536) nb = 65536;
    hipLaunchKernelGGL(topk_finalize_w, dim3((unsigned)nb), dim3(256), 0, st, a.R, a.ldR, a.S,
                       a.ldS, a.dim, a.nR, a.nS, a.nr64, a.ns64, a.info_r, a.cnt, a.cand, a.Kc,
                       a.k, a.fp32_terms, order, a.hdr, a.fb_rows, a.out_idx, a.out_score, floors,
                       n, a.min_sim);
    return hipGetLastError();
}

// Prepared rows rows[0 .. n) of X (row_bytes each, a multiple of 16) copied
// into a compact buffer of n_pad rows (rows n .. n_pad - 1 zero).
__global__ __launch_bounds__(256) void gather_prepared(const char* __restrict__ X,
                                                       int row_bytes, const int* __restrict__ rows,
                                                       int64_t n, int64_t n_pad,
                                                       char* __restrict__ dst) {
    const int per = row_bytes / 16;
    const int64_t total = n_pad * per;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = q / per, o = q - c * per;
        v4i v = {0, 0, 0, 0};
        if (c < n) v = *(const v4i*)(X + (int64_t)rows[c] * row_bytes + o * 16);
        *(v4i*)(dst + c * row_bytes + o * 16) = v;
    }
}

hipError_t launch_gather_prepared(const void* X, int row_bytes, const int* rows, int64_t n,
                                  int64_t n_pad, void* dst, hipStream_t st) {
    if (n_pad <= 0) return hipSuccess;
    int64_t nb = (n_pad * (row_bytes / 16) + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(gather_prepared, dim3((unsigned)nb), dim3(256), 0, st, (const char*)X,
                       row_bytes, rows, n, n_pad, (char*)dst);
    return hipGetLastError();
}

// Exact scan of the rows that failed the certificate.  n_fb is the count read
// back by the host (-1: unknown, asynchronous call): with a known count the
// rows go in batches through the split scan; otherwise one workgroup per row
// loops over the device-side list.
hipError_t launch_topk_fallback(const TopkArgs& a, int64_t n_fb, hipStream_t st) {
    if (a.nR <= 0 || a.nS <= 0) return hipSuccess;
    const unsigned long long* cnt = a.hdr + H_TOPK_FB;
    if (n_fb < 0) {
        hipLaunchKernelGGL(exact_topk_rows, dim3(1024, 1), dim3(256), 0, st, a.R, a.ldR, a.S,
                           a.ldS, a.dim, a.nS, a.nr64, a.ns64, a.k, (const int*)a.fb_rows, cnt,
                           0, 0, 0x7fffffff, a.out_idx, a.out_score, (double*)nullptr,
                           (double*)nullptr, (int*)nullptr, 1, a.min_sim);
        return hipGetLastError();
    }
    for (int64_t b = 0; b < n_fb; b += a.part_rows) {
        hipError_t e = exact_topk_batch(a, a.fb_rows, cnt, 0, (int)b, a.part_rows, a.out_idx,
                                        a.out_score, nullptr, st, 1, a.min_sim);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ej
