// prune.hip -- exact pruning of tile pairs for the batched join.
//
// The certified counterpart of the learned prefilter: every relation of the
// batch is put in an order that keeps similar rows together, cut into tiles
// of 128 rows, and a tile pair (T, U) is skipped only when a rigorous upper
// bound of the cosine of every one of its pairs, taken in the original
// embedding space, lies below theta.  The skipped pairs then all have
// sim64 < theta and the result is the exact join.
//
//  * Order: the prepared rows are coded by a fixed random +-1 projection to
//    64 dimensions (no training), normalised; the anchor keys and the stable
//    per-relation sort of the prefilter follow (prefilter.hip).  The order
//    only decides how tight the tiles are, never what is returned.
//  * Per tile T of prepared rows x_r (BF16, in tile order): the direction d_T
//    of the rows' mean and the angular radius A_T, an upper bound of the
//    angle between d_T and every exact unit row r / |r| of T: the largest
//    angle measured on the prepared rows, plus the angle their rounding can
//    hide (|x_r - r/|r|| <= e_r, the row's quantisation error norm plus the
//    FP32 normalisation error), plus slack for the FP32 acos.
//  * Tile to rows (on the matrix cores): M1 = max over the rows s of U of
//    d_T . x_s, M2 = max over the rows r of T of d_U . x_r.  Raised by the
//    BF16 rounding of d and the rows' error norms, m1 bounds d_T . s/|s| for
//    every s of U; the angle between r and s is then at least
//    acos(m1) - A_T (triangle inequality for angles), so
//        cos(r, s) <= cos(max(0, acos(m1) - A_T))
//    and the same with (M2, A_U).  The pair of tiles is kept when the smaller
//    bound reaches theta (minus slack for the FP32 cos).
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "mma.hpp"
#include "prefilter.hpp"
#include "tile_body.hpp"

namespace ej {

namespace {

__device__ __forceinline__ int xp_seg_of(const PrepSeg* __restrict__ segs, int nseg,
                                         int64_t row) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].row_base <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int xp_job_of(const BatchJob* __restrict__ jobs, int n_jobs,
                                         int64_t item, bool side) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((side ? jobs[mid].side_base : jobs[mid].tile_base) <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace

// The projection: P[o][k] = +-1/8 for k < dim (sign from a SplitMix64-style
// mix of the index), 0 beyond; BF16, 64 x Dp.
__global__ void xp_proj(int dim, int Dp, uint16_t* __restrict__ P) {
    const int64_t n = (int64_t)MLP_OUT * Dp;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(q % Dp);
        uint64_t z = (uint64_t)q * 0x9E3779B97F4A7C15ull + 0x5EEDull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const float v = k < dim ? ((z & 1ull) ? 0.125f : -0.125f) : 0.0f;
        P[q] = f32_to_bf16_rne(v);
    }
}

// Z = X P^T over the flat row space (128-row tiles of the prepared rows of
// every segment, 64 code columns).
__global__ __launch_bounds__(256) void xp_codes(const BatchHead* __restrict__ head,
                                                const PrepSeg* __restrict__ segs,
                                                const uint16_t* __restrict__ P, int Dp,
                                                float* __restrict__ Z) {
    constexpr int BM = 128, BN = 64, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    __shared__ int s_seg;
    const int64_t tile = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int64_t row0 = tile * BM;
    if (row0 >= head->n_rows) return;
    if (threadIdx.x == 0) s_seg = xp_seg_of(segs, head->n_segs, row0);
    __syncthreads();
    const PrepSeg& g = segs[s_seg];
    const int tm = (int)((row0 - g.row_base) / BM);
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)g.Xq, (const char*)P, nullptr,
                                          nullptr, Dp * 2, tm, 0, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
#pragma unroll
    for (int j = 0; j < TG::FN; ++j) {
        const int col = wn * TG::WTN + j * 32 + r32;
#pragma unroll
        for (int i = 0; i < TG::FM; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t row = row0 + wm * TG::WTM + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                Z[row * MLP_OUT + col] = acc[i][j][e];
            }
    }
}

// One wave per 128-row tile of the ordered prepared rows: direction d_T (BF16
// into Dir, zero for an empty or directionless tile), the angular radius
// A_T with its margins (alpha; 4 for a directionless tile: the bound is void;
// -1 for an empty tile) and the largest row error e_T (err).
__global__ __launch_bounds__(256) void xp_tile_stats(const BatchHead* __restrict__ head,
                                                     const PrepSeg* __restrict__ segs, int Dp,
                                                     uint16_t* __restrict__ Dir,
                                                     float* __restrict__ alpha,
                                                     float* __restrict__ err) {
    constexpr int NV = 16;  // Dp <= 1024
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t row0 = tile * 128;
    if (row0 >= head->n_rows) return;
    const PrepSeg& g = segs[xp_seg_of(segs, head->n_segs, row0)];
    const int64_t l0 = row0 - g.row_base;
    const int cnt = (int)max<int64_t>(0, min<int64_t>(128, g.rows - l0));
    const uint16_t* X = (const uint16_t*)g.Xq + l0 * Dp;
    float c[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = 0.0f;
    float emax = 0.0f;
    for (int i = 0; i < cnt; ++i) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int k = lane + 64 * v;
            if (k < Dp) c[v] += bf16_to_f32(X[(int64_t)i * Dp + k]);
        }
        emax = fmaxf(emax, g.info[l0 + i].enorm);
    }
    float cc = 0.0f;
#pragma unroll
    for (int v = 0; v < NV; ++v) cc += c[v] * c[v];
    const float cn = sqrtf(wave_sum(cc));
    const bool dir = cnt > 0 && cn > 1e-3f * (float)cnt;
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = dir ? c[v] / cn : 0.0f;
    // largest angle between a prepared row and the direction
    float cmin = 1.0f;
    if (dir) {
        for (int i = 0; i < cnt; ++i) {
            float dot = 0.0f, nn = 0.0f;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int k = lane + 64 * v;
                if (k < Dp) {
                    const float x = bf16_to_f32(X[(int64_t)i * Dp + k]);
                    dot = fmaf(x, c[v], dot);
                    nn = fmaf(x, x, nn);
                }
            }
            dot = wave_sum(dot);
            nn = wave_sum(nn);
            if (nn > 0.0f) cmin = fminf(cmin, dot / sqrtf(nn));  // zero rows: cos 0 with all
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int k = lane + 64 * v;
        if (k < Dp) Dir[tile * Dp + k] = f32_to_bf16_rne(c[v]);
    }
    if (lane == 0) {
        // rows are the exact unit rows up to e: quantisation error norm plus
        // the FP32 normalisation (relative (d + 8) 2^-24, counted 1.5 times)
        const float e = emax + 1.5f * (float)(g.dim + 8) * 5.9604645e-8f + 1e-6f;
        err[tile] = e;
        float a;
        if (cnt == 0) a = -1.0f;
        else if (!dir) a = 4.0f;
        else a = acosf(fmaxf(-1.0f, fminf(1.0f, cmin))) + 1.1f * e + 1e-3f;
        alpha[tile] = a;
    }
}

// Tile-to-rows maxima (as the prefilter's pf_sidemax, in the original
// space): one item multiplies the directions of 128 tiles of one side by
// the 128 prepared rows of one tile of the other side (K = Dp) and keeps
// the row maxima.
__global__ __launch_bounds__(256) void xp_sidemax(const BatchHead* __restrict__ head,
                                                  const BatchJob* __restrict__ jobs, int Dp,
                                                  const uint16_t* __restrict__ Dir,
                                                  float* __restrict__ M1,
                                                  float* __restrict__ M2) {
    constexpr int BM = 128, BN = 128, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    __shared__ float s_v[WN][BM];
    const int64_t item = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (item >= head->n_side) return;
    const int jb = xp_job_of(jobs, head->n_jobs, item, true);
    const BatchJob& J = jobs[jb];
    int64_t local = item - J.side_base;
    const int64_t n0 = (int64_t)((J.tiles_m + 127) / 128) * J.tiles_n;
    const bool side0 = local < n0;
    int ag, b;
    int64_t a_first, n_a;
    const char* rows;
    if (side0) {  // R tile directions x S tile rows
        ag = (int)(local / J.tiles_n);
        b = (int)(local % J.tiles_n);
        a_first = J.rtile0 + (int64_t)ag * 128;
        n_a = J.tiles_m;
        rows = J.B;
    } else {      // S tile directions x R tile rows
        local -= n0;
        ag = (int)(local / J.tiles_m);
        b = (int)(local % J.tiles_m);
        a_first = J.stile0 + (int64_t)ag * 128;
        n_a = J.tiles_n;
        rows = J.A;
    }
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)(Dir + a_first * Dp), rows, nullptr,
                                          nullptr, Dp * 2, 0, b, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
    // rows past the end of the relation are zero rows of the padded copy:
    // a product 0 never raises a maximum above the real rows' only when some
    // real row is larger, so they are left out explicitly
    const int64_t n_rows_b = side0 ? J.nS : J.nR;
#pragma unroll
    for (int i = 0; i < TG::FM; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            float v = -2.0f;
#pragma unroll
            for (int j = 0; j < TG::FN; ++j) {
                const int64_t col = (int64_t)b * BN + wn * TG::WTN + j * 32 + r32;
                if (col < n_rows_b) v = fmaxf(v, acc[i][j][e]);
            }
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
            if (r32 == 0) s_v[wn][wm * TG::WTM + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3)] = v;
        }
    __syncthreads();
    if (threadIdx.x < BM) {
        const int t = threadIdx.x;
        const int64_t a = (int64_t)ag * 128 + t;
        if (a < n_a) {
            const float v = fmaxf(s_v[0][t], s_v[1][t]);
            if (side0) M1[J.tile_base + a * J.tiles_n + b] = v;
            else M2[J.tile_base + (int64_t)b * J.tiles_n + a] = v;
        }
    }
}

__device__ __forceinline__ float xp_rows_bound(float m, float e_other, float a) {
    // m: the computed maximum of d . x over the other tile's rows; raised by
    // the BF16 rounding of d (2^-9, counted twice), the rows' error norm and
    // the FP32 accumulation, it bounds d . s/|s| for every exact row s
    const float mu = fminf(1.0f, m + 0.0078125f + 1.1f * e_other + 1e-4f);
    const float gap = acosf(fmaxf(-1.0f, mu)) - a - 1e-3f;
    return gap > 0.0f ? cosf(gap) + 1e-5f : 1.0f + 1e-5f;
}

// Every tile pair of every job: keep it unless the smaller tile-to-rows bound
// lies below theta.  Output as pf_bounds: a compacted work list, or a flag
// per tile pair for the panel form's chunks.
__global__ __launch_bounds__(256) void xp_bounds(const BatchHead* __restrict__ head,
                                                 const BatchJob* __restrict__ jobs,
                                                 const float* __restrict__ alpha,
                                                 const float* __restrict__ err,
                                                 const float* __restrict__ M1,
                                                 const float* __restrict__ M2,
                                                 int64_t* __restrict__ work,
                                                 unsigned long long* __restrict__ n_work,
                                                 uint8_t* __restrict__ keep_flags) {
    const int lane = threadIdx.x & 63;
    const int64_t total = head->n_tiles;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < total;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = base + lane;
        bool keep = false;
        int64_t packed = 0;
        if (item < total) {
            const int jb = xp_job_of(jobs, head->n_jobs, item, false);
            const BatchJob& J = jobs[jb];
            const int64_t local = item - J.tile_base;
            const int tm = (int)(local / J.tiles_n), tn = (int)(local % J.tiles_n);
            const int64_t a = J.rtile0 + tm, b = J.stile0 + tn;
            const float aa = alpha[a], ab = alpha[b];
            if (aa >= 0.0f && ab >= 0.0f) {
                float bound = 1.0f + 1e-5f;
                if (aa < 3.5f) bound = fminf(bound, xp_rows_bound(M1[item], err[b], aa));
                if (ab < 3.5f) bound = fminf(bound, xp_rows_bound(M2[item], err[a], ab));
                // theta <= 0: a zero row's pairs (similarity 0) match, and
                // the bound does not cover them; such jobs are not pruned
                keep = J.theta <= 0.0 || (double)bound >= J.theta;
                packed = ((int64_t)jb << 48) | ((int64_t)tm << 24) | (int64_t)tn;
            }
        }
        if (keep_flags) {
            if (item < total) keep_flags[item] = keep ? 1 : 0;
            continue;
        }
        const uint64_t m = __ballot(keep);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            unsigned long long b0 = 0;
            if (lane == leader) b0 = atomicAdd(n_work, (unsigned long long)__popcll(m));
            const uint32_t blo = __shfl((uint32_t)b0, leader, 64);
            const uint32_t bhi = __shfl((uint32_t)(b0 >> 32), leader, 64);
            const unsigned long long bb = ((unsigned long long)bhi << 32) | blo;
            if (keep) work[bb + lanes_below(m)] = packed;
        }
    }
}

hipError_t launch_xp_codes(const BatchHead* head, const PrepSeg* segs, int64_t n_rows, int dim,
                           int Dp, uint16_t* P, float* Z, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    if (Dp > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xp_proj, dim3(64), dim3(256), 0, st, dim, Dp, P);
    const int64_t tiles = n_rows / 128;
    const int64_t gx = std::min<int64_t>(tiles, 65536), gy = (tiles + gx - 1) / gx;
    hipLaunchKernelGGL(xp_codes, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, head, segs,
                       (const uint16_t*)P, Dp, Z);
    return hipGetLastError();
}

hipError_t launch_xp_tiles(const BatchHead* head, const PrepSeg* segs, const BatchJob* jobs,
                           int64_t n_rows, int Dp, uint16_t* Dir, float* alpha, float* err,
                           float* M1, float* M2, int64_t n_side, int64_t* work,
                           unsigned long long* n_work, int64_t n_tiles, uint8_t* keep,
                           hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    if (Dp > 1024) return hipErrorInvalidValue;
    const int64_t tiles = n_rows / 128;
    hipLaunchKernelGGL(xp_tile_stats, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, head,
                       segs, Dp, Dir, alpha, err);
    if (n_side > 0) {
        const int64_t gx = std::min<int64_t>(n_side, 65536), gy = (n_side + gx - 1) / gx;
        hipLaunchKernelGGL(xp_sidemax, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, head,
                           jobs, Dp, (const uint16_t*)Dir, M1, M2);
    }
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_tiles + 255) / 256, 8192));
    hipLaunchKernelGGL(xp_bounds, dim3((unsigned)blocks), dim3(256), 0, st, head, jobs,
                       (const float*)alpha, (const float*)err, (const float*)M1,
                       (const float*)M2, work, n_work, keep);
    return hipGetLastError();
}

}  // namespace ej
