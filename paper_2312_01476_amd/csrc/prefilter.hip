// prefilter.hip -- the approximate mode of the batched join: code every
// prepared row with the prefilter network, order the rows of each relation
// by a locality-sensitive key of its code, bound the predicted similarity of
// every 128 x 128 tile pair from per-tile centroids and radii, and keep only
// the tile pairs whose bound reaches theta - eps as the work list of the
// persistent contraction kernel.  The pairs it finds are exact (they come
// from the same contraction and FP64 band rescore); only tile pairs are
// skipped, so the result is a subset of the exact join.
//
// Ordering key: K anchor codes are sampled from the batch's rows, grouped by
// leader clustering (an anchor joins the first earlier leader within cosine
// tau), and every row takes the group of its nearest anchor; rows of one
// tight cluster of codes then share a key and become contiguous.
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
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
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

// one step of a transposed wave sum: values [H, 2H) cross lane bit M, the
// lower half keeps its values and adds the partner's
template <int N, int H, int M>
__device__ __forceinline__ void pf_fold(float (&v)[N], int lane) {
    const bool up = lane & M;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const float send = up ? v[i] : v[i + H];
        const float keep = up ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, M, 64);
    }
}

// layer 2 over the flat row space with the normalisation of the codes:
// z = H W2 + b2, u = z / ||z|| (FP32, and a BF16 copy for the anchor
// assignment; zero for padding, zero and non-finite codes).  A wave holds 32
// of a row's 64 columns: its squares are totalled over the 32 lanes of each
// half (lane r ends with value r of the wave's 32 rows) and the two column
// halves meet in LDS.
__global__ __launch_bounds__(256) void pf_l2(const BatchHead* __restrict__ head,
                                             const PrepSeg* __restrict__ segs,
                                             const uint16_t* __restrict__ Hb,
                                             const uint16_t* __restrict__ W2t,
                                             const float* __restrict__ b2, float* __restrict__ U,
                                             uint16_t* __restrict__ Ub) {
    constexpr int BM = 128, BN = 64, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    static_assert(TG::FM == 2 && TG::FN == 1, "one 32-column block per wave");
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    __shared__ float s_q[WN][BM];
    const int64_t tm = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (tm * BM >= head->n_rows) return;
    v16f acc[TG::FM][TG::FN];
    // the mainloop addresses tile tm of A from its base; pass the tile's rows
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)(Hb + tm * BM * MLP_HIDDEN),
                                          (const char*)W2t, nullptr, nullptr, MLP_HIDDEN * 2, 0,
                                          0, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
    const int col = wn * TG::WTN + r32;
    const float bias = bf16v(b2[col]);
    float q[32];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            acc[i][0][e] += bias;
            q[16 * i + e] = acc[i][0][e] * acc[i][0][e];
        }
    pf_fold<32, 16, 16>(q, lane);
    pf_fold<32, 8, 8>(q, lane);
    pf_fold<32, 4, 4>(q, lane);
    pf_fold<32, 2, 2>(q, lane);
    pf_fold<32, 1, 1>(q, lane);
    auto row_in_tile = [&](int i, int e) {
        return wm * TG::WTM + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
    };
    s_q[wn][row_in_tile(r32 >> 4, r32 & 15)] = q[0];
    __syncthreads();
    const PrepSeg& g = segs[seg_of(segs, head->n_segs, tm * BM)];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int rl = row_in_tile(i, e);
            const int64_t row = tm * BM + rl;
            const float nz = sqrtf(s_q[0][rl] + s_q[1][rl]);
            const bool real = row - g.row_base < g.rows;
            const float u = real && nz > 0.0f ? acc[i][0][e] / nz : 0.0f;
            U[row * MLP_OUT + col] = u;
            Ub[row * MLP_OUT + col] = f32_to_bf16_rne(u);
        }
}

// anchors: the codes of sampled rows (FP32, and BF16 zero-padded to a
// multiple of 128 anchors)
__global__ void pf_anchor_gather(const float* __restrict__ U, const int64_t* __restrict__ idx,
                                 int K, int Kpad, float* __restrict__ Af,
                                 uint16_t* __restrict__ Ab) {
    const int k = blockIdx.x, o = threadIdx.x;  // 64 threads
    if (k >= Kpad) return;
    const float v = k < K ? U[idx[k] * MLP_OUT + o] : 0.0f;
    if (k < K) Af[(int64_t)k * MLP_OUT + o] = v;
    Ab[(int64_t)k * MLP_OUT + o] = f32_to_bf16_rne(v);
}

// leader labels of the anchors, in anchor order: an anchor joins the first
// leader whose code has cosine >= tau with it, else becomes a leader; the
// label is the leader's rank.  Two steps: every anchor pair's test in
// parallel (a bit matrix: bit b of word w of row k is set when anchor
// 64 w + b passes with anchor k), then one wave walks the anchors in order
// holding the leader set as a bit mask (lane w: anchors 64 w .. 64 w + 63):
// the first leader an anchor passes with is the lowest set bit of its row
// masked by the leader set, since leaders are taken in anchor order.
__global__ __launch_bounds__(256) void pf_anchor_bits(const float* __restrict__ Af, int K, int W,
                                                      float tau, uint64_t* __restrict__ bits) {
    const int lane = threadIdx.x & 63;
    const int64_t word = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);  // k * W + w
    if (word >= (int64_t)K * W) return;  // whole waves
    const int k = (int)(word / W), j = (int)(word % W) * 64 + lane;
    bool pass = false;
    if (j < K) {
        const float* a = Af + (int64_t)k * MLP_OUT;
        const float* b = Af + (int64_t)j * MLP_OUT;
        float d = 0.0f;
        for (int o = 0; o < MLP_OUT; ++o) d = fmaf(a[o], b[o], d);
        pass = d >= tau;
    }
    const uint64_t m = __ballot(pass);
    if (lane == 0) bits[word] = m;
}

__global__ __launch_bounds__(256) void pf_leaders(const uint64_t* __restrict__ bits, int K, int W,
                                                  int32_t* __restrict__ label) {
    constexpr int CH = 64;  // anchor rows staged in LDS at a time
    __shared__ uint64_t s_rows[CH * 64];
    __shared__ int s_rank[PF_MAX_ANCHORS];
    const int tid = threadIdx.x, lane = tid & 63;
    uint64_t lead = 0;  // wave 0, lane w: leader bits of anchors 64 w .. 64 w + 63
    int n = 0;          // leaders so far (wave-uniform)
    for (int k0 = 0; k0 < K; k0 += CH) {
        const int rows = min(CH, K - k0);
        __syncthreads();  // the previous chunk has been walked
        for (int i = tid; i < rows * W; i += blockDim.x) s_rows[i] = bits[(int64_t)k0 * W + i];
        __syncthreads();
        if (tid < 64) {
            for (int r = 0; r < rows; ++r) {
                const int k = k0 + r;
                const uint64_t h = lane < W ? (s_rows[r * W + lane] & lead) : 0ull;
                const uint64_t any = __ballot(h != 0ull);
                if (any == 0ull) {
                    if (lane == (k >> 6)) lead |= 1ull << (k & 63);
                    if (lane == 0) {
                        s_rank[k] = n;
                        label[k] = n;
                    }
                    ++n;
                } else {
                    const int w = __ffsll((unsigned long long)any) - 1;
                    const uint32_t lo = __shfl((uint32_t)h, w, 64);
                    const uint32_t hi = __shfl((uint32_t)(h >> 32), w, 64);
                    const uint64_t hw = ((uint64_t)hi << 32) | lo;
                    const int j = w * 64 + __ffsll((unsigned long long)hw) - 1;
                    if (lane == 0) label[k] = s_rank[j];
                }
            }
        }
    }
}

// ordering key of every row: the label of its nearest anchor (largest code
// dot product, ties to the lower anchor), on the matrix cores.  A workgroup
// takes 128 rows, a wave 32 of them with their codes held in registers (one
// fragment per 16 code elements); the anchors pass through LDS 128 at a time
// (swizzled 128-byte rows) and every wave sweeps them in blocks of 32,
// keeping per lane the best anchor of each of its 16 accumulator rows.
// Every dot product is the same four matrix-core steps in the same order as
// any other tile kernel over these codes.  Padding rows get PF_PAD_KEY.
__global__ __launch_bounds__(256) void pf_assign(const BatchHead* __restrict__ head,
                                                 const PrepSeg* __restrict__ segs,
                                                 const uint16_t* __restrict__ Ub,
                                                 const uint16_t* __restrict__ Ab, int K, int Kpad,
                                                 const int32_t* __restrict__ label,
                                                 int32_t* __restrict__ key) {
    __shared__ __attribute__((aligned(16))) char s_a[128 * 128];
    const int64_t tm = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (tm * 128 >= head->n_rows) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rr = lane & 31, kh = lane >> 5;
    const int64_t row0 = tm * 128 + 32 * wave;
    typedef __attribute__((address_space(1))) const v4i* gv4_ptr;
    v4i a[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
        a[t] = *(gv4_ptr)(Ub + (row0 + rr) * MLP_OUT + 16 * t + 8 * kh);
    float bv[16];
    int bi[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        bv[e] = -3.0f;
        bi[e] = 0x7fffffff;
    }
    for (int c0 = 0; c0 < Kpad; c0 += 128) {
        __syncthreads();  // the previous chunk has been read
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = threadIdx.x + 256 * q;  // 16-byte piece: anchor idx / 8, chunk idx % 8
            const int ar = idx >> 3, ch = idx & 7;
            *(v4i*)(s_a + lds_off(ar, ch)) = *(gv4_ptr)(Ab + (int64_t)(c0 + ar) * MLP_OUT + 8 * ch);
        }
        __syncthreads();
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
            const int ar = 32 * blk + rr;
            v16f acc;
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[e] = 0.0f;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const v4i b = *(const v4i*)(s_a + lds_off(ar, 2 * t + kh));
                Mma<P_BF16>::mma(a[t], b, acc, 0, 0);
            }
            const int col = c0 + ar;
            if (col < K) {
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (acc[e] > bv[e]) {  // anchors ascend per lane: ties keep the lower
                        bv[e] = acc[e];
                        bi[e] = col;
                    }
            }
        }
    }
    // best over the 32 lanes of a half (same rows, different anchors)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) {
            const float ov = __shfl_xor(bv[e], o, 64);
            const int oi = __shfl_xor(bi[e], o, 64);
            if (ov > bv[e] || (ov == bv[e] && oi < bi[e])) {
                bv[e] = ov;
                bi[e] = oi;
            }
        }
    }
    // lane rr == e of each half writes row 8 (e / 4) + 4 kh + e % 4
    int best = bi[0];
#pragma unroll
    for (int e = 1; e < 16; ++e)
        if (rr == e) best = bi[e];
    if (rr < 16) {
        const int64_t row = row0 + 8 * (rr >> 2) + 4 * kh + (rr & 3);
        const PrepSeg& g = segs[seg_of(segs, head->n_segs, row)];
        const bool real = row - g.row_base < g.rows;
        key[row] = (real && best < K) ? label[best] : PF_PAD_KEY;
    }
}

// ---------------------------------------------------------------------------
// stable radix sort of every relation's rows by key: 2 passes of 6 bits,
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
                                                     float* __restrict__ cnorm,
                                                     float* __restrict__ alpha,
                                                     uint16_t* __restrict__ Up,
                                                     uint16_t* __restrict__ Dir) {
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
    const float cn = sqrtf(wave_sum(c * c));
    const float ch = cn > 0.0f ? c / cn : 0.0f;  // centroid direction
    float r2 = 0.0f, cmin = 1.0f;
    for (int i = 0; i < cnt; ++i) {
        const float u = U[(g.row_base + perm[row0 + i]) * MLP_OUT + lane];
        const float dlt = u - c;
        r2 = fmaxf(r2, wave_sum(dlt * dlt));
        cmin = fminf(cmin, wave_sum(u * ch));
        Up[(row0 + i) * MLP_OUT + lane] = f32_to_bf16_rne(u);  // codes in tile order
    }
    for (int i = cnt; i < 128; ++i) Up[(row0 + i) * MLP_OUT + lane] = 0;
    Dir[tile * MLP_OUT + lane] = f32_to_bf16_rne(cn > 1e-3f ? ch : 0.0f);
    C[tile * MLP_OUT + lane] = c;
    if (lane == 0) {
        // slack for the FP32 rounding of the sums
        rho[tile] = cnt ? sqrtf(r2) * (1.0f + 1e-6f) + 1e-6f : -1.0f;
        cnorm[tile] = cn * (1.0f + 1e-6f);
        // angular radius: largest angle between a code and the centroid
        // direction (pi: no direction, the angular bound is void)
        alpha[tile] = cn > 1e-3f ? acosf(fmaxf(-1.0f, fminf(1.0f, cmin))) + 1e-4f : 3.2f;
    }
}

// Tile-to-rows maxima, on the matrix cores: for every tile pair (T, U) of a
// job, M1 = max over the rows s of U of dir(T) . u_s and M2 = max over the
// rows r of T of dir(U) . u_r, with dir the unit centroid direction.  One
// item multiplies the directions of 128 tiles of one side by the 128 codes
// of one tile of the other side and keeps the row maxima.
__global__ __launch_bounds__(256) void pf_sidemax(const BatchHead* __restrict__ head,
                                                  const BatchJob* __restrict__ jobs,
                                                  const uint16_t* __restrict__ Up,
                                                  const uint16_t* __restrict__ Dir,
                                                  float* __restrict__ M1,
                                                  float* __restrict__ M2) {
    constexpr int BM = 128, BN = 128, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    __shared__ float s_v[WN][BM];
    const int64_t item = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (item >= head->n_side) return;
    const int n_jobs = head->n_jobs;
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].side_base <= item) lo = mid;
        else hi = mid - 1;
    }
    const BatchJob& J = jobs[lo];
    int64_t local = item - J.side_base;
    const int64_t n0 = (int64_t)((J.tiles_m + 127) / 128) * J.tiles_n;
    int64_t a_first, b_tile, n_a;  // direction tiles [a_first, +128), code tile b_tile
    bool side0 = local < n0;
    int ag, b;
    if (side0) {
        ag = (int)(local / J.tiles_n);
        b = (int)(local % J.tiles_n);
        a_first = J.rtile0 + (int64_t)ag * 128;
        b_tile = J.stile0 + b;
        n_a = J.tiles_m;
    } else {
        local -= n0;
        ag = (int)(local / J.tiles_m);
        b = (int)(local % J.tiles_m);
        a_first = J.stile0 + (int64_t)ag * 128;
        b_tile = J.rtile0 + b;
        n_a = J.tiles_n;
    }
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)(Dir + a_first * MLP_OUT),
                                          (const char*)(Up + b_tile * 128 * MLP_OUT), nullptr,
                                          nullptr, MLP_OUT * 2, 0, 0, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
#pragma unroll
    for (int i = 0; i < TG::FM; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            float v = acc[i][0][e];
#pragma unroll
            for (int j = 1; j < TG::FN; ++j) v = fmaxf(v, acc[i][j][e]);
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

// every tile pair of every job: keep it when the smallest of these upper
// bounds of the predicted similarity reaches theta - eps:
//   c_T . c_U + rho_T ||c_U|| + rho_U ||c_T|| + rho_T rho_U   (any codes),
//   cos(max(0, angle(c_T, c_U) - a_T - a_U))                  (unit codes),
//   cos(max(0, acos(M1) - a_T)) and cos(max(0, acos(M2) - a_U))
// (M1, M2: tile-to-rows maxima of pf_sidemax)
__global__ __launch_bounds__(256) void pf_bounds(const BatchHead* __restrict__ head,
                                                 const BatchJob* __restrict__ jobs,
                                                 const float* __restrict__ C,
                                                 const float* __restrict__ rho,
                                                 const float* __restrict__ cnorm,
                                                 const float* __restrict__ alpha,
                                                 const float* __restrict__ M1,
                                                 const float* __restrict__ M2, float eps,
                                                 int64_t* __restrict__ work,
                                                 unsigned long long* __restrict__ n_work,
                                                 uint8_t* __restrict__ keep_flags) {
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
                float bound = dot + 1e-5f + ra * cnorm[b] + rb * cnorm[a] + ra * rb;
                // codes are unit vectors: the angle between two of them is at
                // least the angle between the tile directions minus both
                // angular radii (1e-4 rad of slack for the FP32 acos/cos)
                const float na = cnorm[a], nb = cnorm[b];
                if (na > 1e-3f && nb > 1e-3f) {
                    const float cphi = fmaxf(-1.0f, fminf(1.0f, dot / (na * nb)));
                    const float gap = acosf(cphi) - alpha[a] - alpha[b] - 1e-4f;
                    if (gap > 0.0f) bound = fminf(bound, cosf(gap) + 1e-5f);
                }
                // one tile's rows against the other tile's direction: the
                // angle of u_r to u_s is at least the angle of dir(T) to u_s
                // minus a_T; 0.02 covers the BF16 codes of the product
                if (na > 1e-3f) {
                    const float m = fminf(1.0f, M1[item] + 0.02f);
                    const float gap = acosf(fmaxf(-1.0f, m)) - alpha[a] - 1e-4f;
                    bound = fminf(bound, gap > 0.0f ? cosf(gap) + 1e-5f : 1.0f + 1e-5f);
                }
                if (nb > 1e-3f) {
                    const float m = fminf(1.0f, M2[item] + 0.02f);
                    const float gap = acosf(fmaxf(-1.0f, m)) - alpha[b] - 1e-4f;
                    bound = fminf(bound, gap > 0.0f ? cosf(gap) + 1e-5f : 1.0f + 1e-5f);
                }
                keep = (double)bound >= J.theta - (double)eps;
                packed = ((int64_t)lo << 48) | ((int64_t)tm << 24) | (int64_t)tn;
            }
        }
        if (keep_flags) {  // per-tile flags for the panel form's chunks
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

// One lane per (job, panel, S chunk) item: the chunk's kept-tile mask from
// the per-tile flags, and a wave-compacted append of the items that keep any.
__global__ __launch_bounds__(256) void pf_chunks(const BatchHead* __restrict__ head,
                                                 const BatchJob* __restrict__ jobs,
                                                 const uint8_t* __restrict__ keep,
                                                 int64_t* __restrict__ work,
                                                 uint32_t* __restrict__ work_mask,
                                                 unsigned long long* __restrict__ n_work,
                                                 unsigned long long* __restrict__ n_kept) {
    const int lane = threadIdx.x & 63;
    const int64_t total = head->n_chunks;
    const int n_jobs = head->n_jobs;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < total;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = base + lane;
        uint32_t mask = 0;
        int64_t packed = 0;
        if (item < total) {
            int lo = 0, hi = n_jobs - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (jobs[mid].chunk_base <= item) lo = mid;
                else hi = mid - 1;
            }
            const BatchJob& J = jobs[lo];
            const int ct = J.chunk_tiles;
            const int nch = (J.tiles_n + ct - 1) / ct;
            const int64_t local = item - J.chunk_base;
            const int tm = (int)(local / nch);
            const int tn0 = (int)(local % nch) * ct;
            const int n = min(ct, J.tiles_n - tn0);
            const uint8_t* k = keep + J.tile_base + (int64_t)tm * J.tiles_n + tn0;
            for (int b = 0; b < n; ++b) mask |= (uint32_t)(k[b] != 0) << b;
            packed = ((int64_t)lo << 48) | ((int64_t)tm << 24) | (int64_t)tn0;
        }
        const uint64_t m = __ballot(mask != 0);
        int kept = __popc(mask);
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) kept += __shfl_xor(kept, o, 64);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            unsigned long long b0 = 0;
            if (lane == leader) {
                b0 = atomicAdd(n_work, (unsigned long long)__popcll(m));
                atomicAdd(n_kept, (unsigned long long)kept);
            }
            const uint32_t blo = __shfl((uint32_t)b0, leader, 64);
            const uint32_t bhi = __shfl((uint32_t)(b0 >> 32), leader, 64);
            const unsigned long long bb = ((unsigned long long)bhi << 32) | blo;
            if (mask) {
                const unsigned long long at = bb + lanes_below(m);
                work[at] = packed;
                work_mask[at] = mask;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_pf_codes(const BatchHead* head, const PrepSeg* segs, int64_t n_rows,
                           const MlpDev& m, uint16_t* Hb, float* U, uint16_t* Ub,
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
    hipLaunchKernelGGL(pf_l2, dim3((unsigned)gx2, (unsigned)gy2), dim3(256), 0, st, head, segs,
                       Hb, m.W2t, b2, U, Ub);
    return hipGetLastError();
}

hipError_t launch_pf_keys(const BatchHead* head, const PrepSeg* segs, int64_t n_rows,
                          const float* U, const uint16_t* Ub, const int64_t* anchor_idx, int K,
                          float tau, float* Af, uint16_t* Ab, uint64_t* abits, int32_t* label,
                          int32_t* key, hipStream_t st) {
    if (n_rows <= 0 || K <= 0) return hipSuccess;
    if (K > PF_MAX_ANCHORS) return hipErrorInvalidValue;
    const int Kpad = (K + 127) / 128 * 128;
    hipLaunchKernelGGL(pf_anchor_gather, dim3((unsigned)Kpad), dim3(64), 0, st, U, anchor_idx, K,
                       Kpad, Af, Ab);
    const int W = pf_anchor_words(K);
    hipLaunchKernelGGL(pf_anchor_bits, dim3((unsigned)(((int64_t)K * W + 3) / 4)), dim3(256), 0, st,
                       Af, K, W, tau, abits);
    hipLaunchKernelGGL(pf_leaders, dim3(1), dim3(256), 0, st, abits, K, W, label);
    const int64_t tiles = n_rows / 128;
    const int64_t gx = std::min<int64_t>(tiles, 65536), gy = (tiles + gx - 1) / gx;
    hipLaunchKernelGGL(pf_assign, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, head, segs,
                       Ub, Ab, K, Kpad, label, key);
    return hipGetLastError();
}

hipError_t launch_pf_sort(const BatchHead* head, const PrepSeg* segs, int n_segs, int64_t n_rows,
                          const int32_t* key, int32_t* perm_a, int32_t* perm_b, int32_t* hist,
                          int32_t* offs, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    const int64_t blocks = n_rows / 256;
    const int32_t* in = nullptr;
    // two passes of 6 bits cover keys below 4096 and end in perm_a: b, a
    for (int pass = 0; pass < 2; ++pass) {
        int32_t* out = pass == 0 ? perm_b : perm_a;
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
                           float* rho, float* cnorm, float* alpha, uint16_t* Up, uint16_t* Dir,
                           float* M1, float* M2, int64_t n_side, float eps, int64_t* work,
                           unsigned long long* n_work, int64_t n_tiles, uint8_t* keep,
                           hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    const int64_t tiles = n_rows / 128;
    hipLaunchKernelGGL(pf_tile_stats, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, head,
                       segs, U, perm, C, rho, cnorm, alpha, Up, Dir);
    if (n_side > 0) {
        const int64_t gx = std::min<int64_t>(n_side, 65536), gy = (n_side + gx - 1) / gx;
        hipLaunchKernelGGL(pf_sidemax, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, head,
                           jobs, Up, Dir, M1, M2);
    }
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_tiles + 255) / 256, 8192));
    hipLaunchKernelGGL(pf_bounds, dim3((unsigned)blocks), dim3(256), 0, st, head, jobs, C, rho,
                       cnorm, alpha, M1, M2, eps, work, n_work, keep);
    return hipGetLastError();
}

hipError_t launch_pf_chunks(const BatchHead* head, const BatchJob* jobs, const uint8_t* keep,
                            int64_t* work, uint32_t* work_mask, unsigned long long* n_work,
                            unsigned long long* n_kept, int64_t n_chunks, hipStream_t st) {
    if (n_chunks <= 0) return hipSuccess;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_chunks + 255) / 256, 8192));
    hipLaunchKernelGGL(pf_chunks, dim3((unsigned)blocks), dim3(256), 0, st, head, jobs, keep, work,
                       work_mask, n_work, n_kept);
    return hipGetLastError();
}

}  // namespace ej
