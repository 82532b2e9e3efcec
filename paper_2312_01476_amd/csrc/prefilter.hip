// prefilter.hip -- the approximate mode of the batched join: code every
// prepared row with the prefilter network, order the rows of each relation
// by a locality-sensitive key of its code, bound the predicted similarity of
// every 128 x 128 tile pair from per-tile centroids and radii, and keep only
// the tile pairs whose bound reaches theta - eps as the work list of the
// persistent contraction kernel.  The pairs it finds are exact (they come
// from the same contraction and FP64 band rescore); only tile pairs are
// skipped, so the result is a subset of the exact join.
//
// Flat row space: the relations of a batch are concatenated, each padded to
// a multiple of 256 rows (PrepSeg.row_base), so every 128-row tile and every
// 256-row block lies inside one relation.
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "mlp.hpp"
#include "mma.hpp"
#include "prefilter.hpp"
#include "tile_body.hpp"

namespace ej {

__device__ __forceinline__ int seg_of(const PrepSeg* __restrict__ segs, int nseg, int64_t row) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].row_base <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ float bf16v(float x) { return bf16_to_f32(f32_to_bf16_rne(x)); }

// ---------------------------------------------------------------------------
// codes of all prepared rows (the network's inference form)
// ---------------------------------------------------------------------------

// layer 1 over the flat row space: H = BF16(ReLU(X W1 + b1))
__global__ __launch_bounds__(256) void pf_l1(const BatchHead* __restrict__ head,
                                             const PrepSeg* __restrict__ segs,
                                             const uint16_t* __restrict__ W1t,
                                             const float* __restrict__ b1, int Dp,
                                             uint16_t* __restrict__ Hb) {
    constexpr int BM = 128, BN = 128, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    __shared__ TileSmem<BM, BN, WM * WN> sm;
    __shared__ int s_seg;
    const int64_t tile = (int64_t)blockIdx.y * gridDim.x / 2 + blockIdx.x / 2;
    const int tn = blockIdx.x & 1;
    const int64_t row0 = tile * BM;
    if (row0 >= head->n_rows) return;
    if (threadIdx.x == 0) s_seg = seg_of(segs, head->n_segs, row0);
    __syncthreads();
    const PrepSeg& g = segs[s_seg];
    const int tm = (int)((row0 - g.row_base) / BM);
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)g.Xq, (const char*)W1t, nullptr,
                                          nullptr, Dp * 2, tm, tn, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
#pragma unroll
    for (int j = 0; j < TG::FN; ++j) {
        const int col = tn * BN + wn * TG::WTN + j * 32 + r32;
        const float bias = bf16v(b1[col]);
#pragma unroll
        for (int i = 0; i < TG::FM; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t row = row0 + wm * TG::WTM + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                Hb[row * MLP_HIDDEN + col] = f32_to_bf16_rne(fmaxf(acc[i][j][e] + bias, 0.0f));
            }
    }
}

// layer 2 over the flat row space: Z = H W2 + b2
__global__ __launch_bounds__(256) void pf_l2(int64_t n_rows, const uint16_t* __restrict__ Hb,
                                             const uint16_t* __restrict__ W2t,
                                             const float* __restrict__ b2, float* __restrict__ Z) {
    constexpr int BM = 128, BN = 64, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    __shared__ TileSmem<BM, BN, WM * WN> sm;
    const int64_t tm = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (tm * BM >= n_rows) return;
    v16f acc[TG::FM][TG::FN];
    // the mainloop addresses tile tm of A from its base; pass the tile's rows
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)(Hb + tm * BM * MLP_HIDDEN),
                                          (const char*)W2t, nullptr, nullptr, MLP_HIDDEN * 2, 0,
                                          0, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
#pragma unroll
    for (int j = 0; j < TG::FN; ++j) {
        const int col = wn * TG::WTN + j * 32 + r32;
        const float bias = bf16v(b2[col]);
#pragma unroll
        for (int i = 0; i < TG::FM; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t row = tm * BM + wm * TG::WTM + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                Z[row * MLP_OUT + col] = acc[i][j][e] + bias;
            }
    }
}

// u = z / ||z|| and the ordering key: bit b set iff u . plane_b >= 0;
// padding rows get the key PF_PAD_KEY so that they sort last
__global__ __launch_bounds__(256) void pf_code(const BatchHead* __restrict__ head,
                                               const PrepSeg* __restrict__ segs,
                                               const float* __restrict__ Z,
                                               const float* __restrict__ planes,
                                               float* __restrict__ U, int32_t* __restrict__ key) {
    const int lane = threadIdx.x & 63;
    const int64_t n = head->n_rows;
    for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n;
         row += (int64_t)gridDim.x * 4) {
        const PrepSeg& g = segs[seg_of(segs, head->n_segs, row)];
        const bool real = row - g.row_base < g.rows;
        const float z = Z[row * MLP_OUT + lane];
        const float nz = sqrtf(wave_sum(z * z));
        const float u = real && nz > 0.0f ? z / nz : 0.0f;
        U[row * MLP_OUT + lane] = u;
        int code = 0;
#pragma unroll
        for (int b = 0; b < MLP_PLANES; ++b)
            code |= (wave_sum(u * planes[b * MLP_OUT + lane]) >= 0.0f ? 1 : 0) << b;
        if (lane == 0) key[row] = real ? code : PF_PAD_KEY;
    }
}

// ---------------------------------------------------------------------------
// stable radix sort of every relation's rows by key: 3 passes of 6 bits,
// blocks of 256 rows (one workgroup each) inside one relation
// ---------------------------------------------------------------------------

// rank of this thread's digit among the lower threads of the block with the
// same digit, and the block's digit counts in s_cnt[4][64]
__device__ __forceinline__ int block_rank(int digit, int (*s_cnt)[64]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t same = ~0ull;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const uint64_t m = __ballot((digit >> b) & 1);
        same &= ((digit >> b) & 1) ? m : ~m;
    }
    for (int i = threadIdx.x; i < 4 * 64; i += blockDim.x) s_cnt[i >> 6][i & 63] = 0;
    __syncthreads();
    const int below = (int)lanes_below(same);
    if (below == 0) s_cnt[wave][digit] = __popcll(same);
    __syncthreads();
    int r = below;
    for (int w = 0; w < wave; ++w) r += s_cnt[w][digit];
    return r;
}

__device__ __forceinline__ int pass_digit(const BatchHead* head, const PrepSeg* segs, int pass,
                                          const int32_t* key, const int32_t* perm_in,
                                          int64_t flat, int& seg_out, int32_t& src) {
    const int seg = seg_of(segs, head->n_segs, flat);
    const int64_t local = flat - segs[seg].row_base;
    src = perm_in ? perm_in[flat] : (int32_t)local;
    seg_out = seg;
    return (key[segs[seg].row_base + src] >> (6 * pass)) & 63;
}

__global__ __launch_bounds__(256) void pf_hist(const BatchHead* __restrict__ head,
                                               const PrepSeg* __restrict__ segs, int pass,
                                               const int32_t* __restrict__ key,
                                               const int32_t* __restrict__ perm_in,
                                               int32_t* __restrict__ hist) {
    __shared__ int s_cnt[4][64];
    const int64_t flat = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int seg;
    int32_t src;
    const int d = pass_digit(head, segs, pass, key, perm_in, flat, seg, src);
    block_rank(d, s_cnt);
    if (threadIdx.x < 64)
        hist[(int64_t)blockIdx.x * 64 + threadIdx.x] =
            s_cnt[0][threadIdx.x] + s_cnt[1][threadIdx.x] + s_cnt[2][threadIdx.x] +
            s_cnt[3][threadIdx.x];
}

// per relation: offsets in (digit, block) order, local to the relation
__global__ void pf_scan(const BatchHead* __restrict__ head, const PrepSeg* __restrict__ segs,
                        const int32_t* __restrict__ hist, int32_t* __restrict__ offs) {
    __shared__ int s_tot[64];
    const int seg = blockIdx.x;
    if (seg >= head->n_segs) return;
    const int64_t b0 = segs[seg].row_base / 256, nb = segs[seg].rows_pad / 256;
    const int d = threadIdx.x;  // 64 threads, one digit each
    int tot = 0;
    for (int64_t b = 0; b < nb; ++b) tot += hist[(b0 + b) * 64 + d];
    s_tot[d] = tot;
    __syncthreads();
    int run = 0;
    for (int e = 0; e < d; ++e) run += s_tot[e];
    for (int64_t b = 0; b < nb; ++b) {
        offs[(b0 + b) * 64 + d] = run;
        run += hist[(b0 + b) * 64 + d];
    }
}

__global__ __launch_bounds__(256) void pf_scatter(const BatchHead* __restrict__ head,
                                                  const PrepSeg* __restrict__ segs, int pass,
                                                  const int32_t* __restrict__ key,
                                                  const int32_t* __restrict__ perm_in,
                                                  const int32_t* __restrict__ offs,
                                                  int32_t* __restrict__ perm_out) {
    __shared__ int s_cnt[4][64];
    const int64_t flat = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int seg;
    int32_t src;
    const int d = pass_digit(head, segs, pass, key, perm_in, flat, seg, src);
    const int r = block_rank(d, s_cnt);
    const int64_t dest = offs[(int64_t)blockIdx.x * 64 + d] + r;
    perm_out[segs[seg].row_base + dest] = src;
}

// ---------------------------------------------------------------------------
// tile statistics and the tile-pair bound
// ---------------------------------------------------------------------------

// one wave per 128-row tile of the ordered rows: centroid c of the codes of
// its real rows, radius rho = max ||u - c||, ||c||; rho < 0 marks an empty tile
__global__ __launch_bounds__(256) void pf_tile_stats(const BatchHead* __restrict__ head,
                                                     const PrepSeg* __restrict__ segs,
                                                     const float* __restrict__ U,
                                                     const int32_t* __restrict__ perm,
                                                     float* __restrict__ C,
                                                     float* __restrict__ rho,
                                                     float* __restrict__ cnorm) {
    const int lane = threadIdx.x & 63;
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t row0 = tile * 128;
    if (row0 >= head->n_rows) return;
    const PrepSeg& g = segs[seg_of(segs, head->n_segs, row0)];
    const int64_t l0 = row0 - g.row_base;
    const int cnt = (int)max<int64_t>(0, min<int64_t>(128, g.rows - l0));
    float c = 0.0f;
    for (int i = 0; i < cnt; ++i) c += U[(g.row_base + perm[row0 + i]) * MLP_OUT + lane];
    c = cnt ? c / (float)cnt : 0.0f;
    float r2 = 0.0f;
    for (int i = 0; i < cnt; ++i) {
        const float dlt = U[(g.row_base + perm[row0 + i]) * MLP_OUT + lane] - c;
        r2 = fmaxf(r2, wave_sum(dlt * dlt));
    }
    C[tile * MLP_OUT + lane] = c;
    const float cn = sqrtf(wave_sum(c * c));
    if (lane == 0) {
        // one FP32 ulp of slack per quantity for the rounding of the sums
        rho[tile] = cnt ? sqrtf(r2) * (1.0f + 1e-6f) + 1e-6f : -1.0f;
        cnorm[tile] = cn * (1.0f + 1e-6f);
    }
}

// every tile pair of every job: keep it when
//   c_T . c_U + rho_T ||c_U|| + rho_U ||c_T|| + rho_T rho_U >= theta - eps
__global__ __launch_bounds__(256) void pf_bounds(const BatchHead* __restrict__ head,
                                                 const BatchJob* __restrict__ jobs,
                                                 const float* __restrict__ C,
                                                 const float* __restrict__ rho,
                                                 const float* __restrict__ cnorm, float eps,
                                                 int64_t* __restrict__ work,
                                                 unsigned long long* __restrict__ n_work) {
    const int lane = threadIdx.x & 63;
    const int64_t total = head->n_tiles;
    const int n_jobs = head->n_jobs;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < total;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = base + lane;
        bool keep = false;
        int64_t packed = 0;
        if (item < total) {
            int lo = 0, hi = n_jobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].tile_base <= item) lo = mid;
                else hi = mid - 1;
            }
            const BatchJob& J = jobs[lo];
            const int64_t local = item - J.tile_base;
            const int tm = (int)(local / J.tiles_n), tn = (int)(local % J.tiles_n);
            const int64_t a = J.rtile0 + tm, b = J.stile0 + tn;
            const float ra = rho[a], rb = rho[b];
            if (ra >= 0.0f && rb >= 0.0f) {
                const float* ca = C + a * MLP_OUT;
                const float* cb = C + b * MLP_OUT;
                float dot = 0.0f;
                for (int k = 0; k < MLP_OUT; ++k) dot = fmaf(ca[k], cb[k], dot);
                // 1e-5 covers the FP32 rounding of the 64-term dot of
                // vectors of norm <= 1
                const float bound = dot + 1e-5f + ra * cnorm[b] + rb * cnorm[a] + ra * rb;
                keep = (double)bound >= J.theta - (double)eps;
                packed = ((int64_t)lo << 48) | ((int64_t)tm << 24) | (int64_t)tn;
            }
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

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_pf_codes(const BatchHead* head, const PrepSeg* segs, int64_t n_rows,
                           const MlpDev& m, uint16_t* Hb, float* Z, float* U, int32_t* key,
                           hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    const int64_t tiles = n_rows / 128;  // n_rows is a multiple of 256
    const float* b1 = m.P + (int64_t)m.dim * MLP_HIDDEN;
    const float* b2 = b1 + MLP_HIDDEN + (int64_t)MLP_HIDDEN * MLP_OUT;
    // 2-D grids: x = 2 column tiles x 32768 row tiles, y = row tile groups
    const int64_t gy1 = (tiles + 32767) / 32768;
    const int64_t gx1 = 2 * std::min<int64_t>(tiles, 32768);
    hipLaunchKernelGGL(pf_l1, dim3((unsigned)gx1, (unsigned)gy1), dim3(256), 0, st, head, segs,
                       m.W1t, b1, m.Dp, Hb);
    const int64_t gx2 = std::min<int64_t>(tiles, 65536), gy2 = (tiles + gx2 - 1) / gx2;
    hipLaunchKernelGGL(pf_l2, dim3((unsigned)gx2, (unsigned)gy2), dim3(256), 0, st, n_rows, Hb,
                       m.W2t, b2, Z);
    const int64_t blocks = std::min<int64_t>((n_rows + 3) / 4, 16384);
    hipLaunchKernelGGL(pf_code, dim3((unsigned)blocks), dim3(256), 0, st, head, segs, Z,
                       m.planes, U, key);
    return hipGetLastError();
}

hipError_t launch_pf_sort(const BatchHead* head, const PrepSeg* segs, int n_segs, int64_t n_rows,
                          const int32_t* key, int32_t* perm_a, int32_t* perm_b, int32_t* hist,
                          int32_t* offs, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    const int64_t blocks = n_rows / 256;
    const int32_t* in = nullptr;
    int32_t* bufs[2] = {perm_a, perm_b};
    // three passes end in perm_a: a, b, a
    for (int pass = 0; pass < 3; ++pass) {
        int32_t* out = bufs[pass & 1 ? 1 : 0];
        if (pass == 2) out = perm_a;
        hipLaunchKernelGGL(pf_hist, dim3((unsigned)blocks), dim3(256), 0, st, head, segs, pass,
                           key, in, hist);
        hipLaunchKernelGGL(pf_scan, dim3((unsigned)n_segs), dim3(64), 0, st, head, segs, hist,
                           offs);
        hipLaunchKernelGGL(pf_scatter, dim3((unsigned)blocks), dim3(256), 0, st, head, segs, pass,
                           key, in, offs, out);
        in = out;
    }
    return hipGetLastError();
}

hipError_t launch_pf_tiles(const BatchHead* head, const PrepSeg* segs, const BatchJob* jobs,
                           int64_t n_rows, const float* U, const int32_t* perm, float* C,
                           float* rho, float* cnorm, float eps, int64_t* work,
                           unsigned long long* n_work, int64_t n_tiles, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    const int64_t tiles = n_rows / 128;
    hipLaunchKernelGGL(pf_tile_stats, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, head,
                       segs, U, perm, C, rho, cnorm);
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_tiles + 255) / 256, 8192));
    hipLaunchKernelGGL(pf_bounds, dim3((unsigned)blocks), dim3(256), 0, st, head, jobs, C, rho,
                       cnorm, eps, work, n_work);
    return hipGetLastError();
}

}  // namespace ej
