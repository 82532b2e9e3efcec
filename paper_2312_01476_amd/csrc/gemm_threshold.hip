// gemm_threshold.hip -- the tensor-join contraction with the threshold
// predicate applied to each block as it is produced.
//
// Section IV.C writes the join as the block-matrix product
// D_tv = sum_i R_ti S_iv of the normalised relations, partitioned along tuple
// lines, with every block of D mapped back to tuple-offset pairs through the
// partitions' start offsets.  Here a block is one BM x BN output tile of a
// matrix-core kernel: operand slices stream through LDS (double buffered),
// the accumulators never leave registers, and the epilogue keeps only the
// pairs that can satisfy the predicate, so the dense intermediate of
// Section V.B never exists.
//
// Exactness: an accumulator a with a >= hi is a certain match, a < lo a
// certain miss, and lo <= a < hi goes to the band list for the FP64 rescore;
// [lo, hi] contains [theta - delta, theta + delta] for a rigorous bound delta
// on |a - sim64|.
//
// Output compaction: each wave counts its hits with ballots, the workgroup
// sums the wave counts in LDS and issues ONE atomicAdd per output list per
// tile; lanes then write their pairs at base + (hits of earlier waves) +
// (hits of lower lanes, mbcnt).
#include "common.hpp"
#include "launch.hpp"
#include "mma.hpp"

namespace ej {

template <int PREC, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(WM* WN * 64) void threshold_tile(
    const char* __restrict__ A, const char* __restrict__ B, const RowInfo* __restrict__ info_r,
    const RowInfo* __restrict__ info_s, int Kp_bytes, int64_t nR, int64_t nS,
    int tiles_m, int tiles_n, int ntiles, float lo, float hi, Pair* __restrict__ out,
    int64_t capacity,
    int2* __restrict__ band, int64_t band_cap, unsigned long long* __restrict__ hdr) {
    constexpr int NT = WM * WN * 64;
    constexpr int NW = WM * WN;
    constexpr int WTM = BM / WM;  // rows per wave
    constexpr int WTN = BN / WN;  // cols per wave
    constexpr int FM = WTM / 32;  // 32x32 blocks per wave
    constexpr int FN = WTN / 32;
    constexpr int CA = BM * 8 / NT;  // 16-byte chunks per thread per slice
    constexpr int CB = BN * 8 / NT;
    static_assert(CA * NT == BM * 8 && CB * NT == BN * 8, "tile/thread mismatch");
    typedef Mma<PREC> M;

    __shared__ __attribute__((aligned(16))) char sA[2][BM * 128];
    __shared__ __attribute__((aligned(16))) char sB[2][BN * 128];
    __shared__ uint32_t s_cnt[2 * NW];
    __shared__ unsigned long long s_base[2];

    // 2-D grid (a 1-D grid of this many workgroups would overflow the 32-bit
    // dispatch size); workgroups past the last tile leave at once
    int bid = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (bid >= ntiles) return;
    if (hdr[H_FLAGS] != 0) return;  // bad input rows: nothing to compute

    // ---- tile index: XCD-aware remap, then grouped rasterisation ----
    // Workgroups are dispatched to the 8 XCDs round-robin; remapping gives
    // each XCD a contiguous range of tiles, so the tiles that run together
    // on one XCD share operand panels in that XCD's L2.
    const int full = ntiles & ~7;
    if (bid < full) bid = (bid & 7) * (full >> 3) + (bid >> 3);
    constexpr int GROUP_M = 8;
    const int per_group = GROUP_M * tiles_n;
    const int grp = bid / per_group;
    const int first_m = grp * GROUP_M;
    const int gsize = min(tiles_m - first_m, GROUP_M);
    const int in_grp = bid - grp * per_group;
    const int tm = first_m + in_grp % gsize;
    const int tn = in_grp / gsize;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int h = lane >> 5, r32 = lane & 31;

    const char* Ag = A + (int64_t)tm * BM * Kp_bytes;
    const char* Bg = B + (int64_t)tn * BN * Kp_bytes;
    const int nk = Kp_bytes >> 7;

    v16f acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    // FP8 operand scales (E8M0 byte 127 - p for a row stored as x * 2^p)
    int sa[FM], sb[FN];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        sa[i] = 127;
        if (PREC == P_FP8)
            sa[i] = 127 - ilogbf(info_r[(int64_t)tm * BM + wm * WTM + i * 32 + r32].qscale);
    }
#pragma unroll
    for (int j = 0; j < FN; ++j) {
        sb[j] = 127;
        if (PREC == P_FP8)
            sb[j] = 127 - ilogbf(info_s[(int64_t)tn * BN + wn * WTN + j * 32 + r32].qscale);
    }

    v4i ra[CA], rb[CB];
    auto gload = [&](int kb) {
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            int q = tid + i * NT;
            ra[i] = *(const v4i*)(Ag + (int64_t)(q >> 3) * Kp_bytes + kb * 128 + (q & 7) * 16);
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            int q = tid + i * NT;
            rb[i] = *(const v4i*)(Bg + (int64_t)(q >> 3) * Kp_bytes + kb * 128 + (q & 7) * 16);
        }
    };
    auto lstore = [&](int st) {
#pragma unroll
        for (int i = 0; i < CA; ++i) {
            int q = tid + i * NT;
            *(v4i*)(&sA[st][lds_off(q >> 3, q & 7)]) = ra[i];
        }
#pragma unroll
        for (int i = 0; i < CB; ++i) {
            int q = tid + i * NT;
            *(v4i*)(&sB[st][lds_off(q >> 3, q & 7)]) = rb[i];
        }
    };

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kb = 0; kb < nk; ++kb) {
        const int st = kb & 1;
        if (kb + 1 < nk) gload(kb + 1);
#pragma unroll
        for (int g = 0; g < M::GROUPS; ++g) {
            typename M::Frag fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int row = wm * WTM + i * 32 + r32;
#pragma unroll
                for (int c = 0; c < M::CPL; ++c) {
                    v4i v = *(const v4i*)(&sA[st][lds_off(row, M::chunk(g, h, c))]);
#pragma unroll
                    for (int e = 0; e < 4; ++e) fa[i][c * 4 + e] = v[e];
                }
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int row = wn * WTN + j * 32 + r32;
#pragma unroll
                for (int c = 0; c < M::CPL; ++c) {
                    v4i v = *(const v4i*)(&sB[st][lds_off(row, M::chunk(g, h, c))]);
#pragma unroll
                    for (int e = 0; e < 4; ++e) fb[j][c * 4 + e] = v[e];
                }
            }
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) M::mma(fa[i], fb[j], acc[i][j], sa[i], sb[j]);
        }
        if (kb + 1 < nk) lstore(st ^ 1);
        __syncthreads();
    }

    // ---- epilogue ----
    // accumulator element e of block (i, j) of this lane sits at
    // row 8*(e/4) + 4*h + e%4 and column r32 of that 32x32 block
    const int64_t i0 = (int64_t)tm * BM + wm * WTM;
    const int64_t j0 = (int64_t)tn * BN + wn * WTN;
    const bool edge = ((int64_t)(tm + 1) * BM > nR) || ((int64_t)(tn + 1) * BN > nS);

    uint32_t nc = 0, nbnd = 0;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float a = acc[i][j][e];
                bool v = true;
                if (edge) {
                    const int64_t gi = i0 + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                    const int64_t gj = j0 + j * 32 + r32;
                    v = gi < nR && gj < nS;
                }
                const uint64_t mlo = __ballot(v && a >= lo);
                if (mlo) {
                    const uint64_t mhi = __ballot(v && a >= hi);
                    nc += __popcll(mhi);
                    nbnd += __popcll(mlo & ~mhi);
                }
            }
    if (lane == 0) {
        s_cnt[2 * wave] = nc;
        s_cnt[2 * wave + 1] = nbnd;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long tc = 0, tb = 0;
        for (int w = 0; w < NW; ++w) {
            tc += s_cnt[2 * w];
            tb += s_cnt[2 * w + 1];
        }
        s_base[0] = tc ? atomicAdd(hdr + H_OUT, tc) : 0ull;
        s_base[1] = tb ? atomicAdd(hdr + H_BAND, tb) : 0ull;
    }
    __syncthreads();
    if (nc + nbnd == 0) return;
    unsigned long long oc = s_base[0], ob = s_base[1];
    for (int w = 0; w < wave; ++w) {
        oc += s_cnt[2 * w];
        ob += s_cnt[2 * w + 1];
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const float a = acc[i][j][e];
                const int64_t gi = i0 + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                const int64_t gj = j0 + j * 32 + r32;
                const bool v = !edge || (gi < nR && gj < nS);
                const uint64_t mlo = __ballot(v && a >= lo);
                if (mlo) {
                    const uint64_t mhi = __ballot(v && a >= hi);
                    const uint64_t mb = mlo & ~mhi;
                    if ((mhi >> lane) & 1ull) {
                        const unsigned long long p = oc + lanes_below(mhi);
                        if ((int64_t)p < capacity) {
                            Pair pr;
                            pr.r = (int32_t)gi;
                            pr.s = (int32_t)gj;
                            pr.score = a;
                            out[p] = pr;
                        }
                    }
                    if ((mb >> lane) & 1ull) {
                        const unsigned long long p = ob + lanes_below(mb);
                        if ((int64_t)p < band_cap) band[p] = make_int2((int)gi, (int)gj);
                    }
                    oc += __popcll(mhi);
                    ob += __popcll(mb);
                }
            }
}

// ---------------------------------------------------------------------------
// tile table and launcher
// ---------------------------------------------------------------------------
static const TileDesc kTiles[] = {
    {1, P_FP32, 128, 128, 32, "fp32:128x128x32"},
    {2, P_FP32, 64, 64, 32, "fp32:64x64x32"},
    {3, P_BF16, 128, 128, 64, "bf16:128x128x64"},
    {4, P_BF16, 256, 128, 64, "bf16:256x128x64"},
    {5, P_FP8, 128, 128, 128, "fp8:128x128x128"},
    {6, P_FP8, 256, 128, 128, "fp8:256x128x128"},
    {7, P_BF16, 256, 256, 64, "bf16:256x256x64/4w"},
    {8, P_BF16, 256, 256, 64, "bf16:256x256x64/8w"},
    {9, P_FP8, 256, 256, 128, "fp8:256x256x128/4w"},
    {10, P_FP8, 256, 256, 128, "fp8:256x256x128/8w"},
    {11, P_FP32, 256, 128, 32, "fp32:256x128x32"},
    // register-resident R panels (K up to 768 bytes per row)
    {12, P_BF16, 0, 0, 64, "bf16:panel"},
    {13, P_FP8, 0, 0, 128, "fp8:panel"},
    {14, P_BF16, 0, 0, 64, "bf16:panel/2wg"},
    {15, P_FP8, 0, 0, 128, "fp8:panel/2wg"},
};

int tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const TileDesc* tile_get(int id) {
    for (const auto& t : kTiles)
        if (t.id == id) return &t;
    return nullptr;
}

template <int PREC, int BM, int BN, int WM, int WN>
static hipError_t run(const ThresholdArgs& a, hipStream_t st) {
    const int64_t tm = (a.nR + BM - 1) / BM, tn = (a.nS + BN - 1) / BN;
    const int64_t nblocks = tm * tn;
    if (nblocks == 0) return hipSuccess;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const int64_t gx = nblocks < 65536 ? nblocks : 65536;
    const int64_t gy = (nblocks + gx - 1) / gx;
    if (gy > 65535) return hipErrorInvalidValue;
    const int kpb = a.Kp * (PREC == P_FP32 ? 4 : PREC == P_BF16 ? 2 : 1);
    hipLaunchKernelGGL((threshold_tile<PREC, BM, BN, WM, WN>), dim3((unsigned)gx, (unsigned)gy),
                       dim3(WM * WN * 64), 0, st, (const char*)a.A, (const char*)a.B, a.info_r,
                       a.info_s, kpb, a.nR,
                       a.nS, (int)tm, (int)tn, (int)nblocks, a.lo, a.hi, a.out, a.capacity, a.band, a.band_cap,
                       a.hdr);
    return hipGetLastError();
}

hipError_t launch_threshold(int tile_id, const ThresholdArgs& a, hipStream_t st) {
    switch (tile_id) {
        case 1: return run<P_FP32, 128, 128, 2, 2>(a, st);
        case 2: return run<P_FP32, 64, 64, 2, 2>(a, st);
        case 3: return run<P_BF16, 128, 128, 2, 2>(a, st);
        case 4: return run<P_BF16, 256, 128, 2, 2>(a, st);
        case 5: return run<P_FP8, 128, 128, 2, 2>(a, st);
        case 6: return run<P_FP8, 256, 128, 2, 2>(a, st);
        case 7: return run<P_BF16, 256, 256, 2, 2>(a, st);
        case 8: return run<P_BF16, 256, 256, 2, 4>(a, st);
        case 9: return run<P_FP8, 256, 256, 2, 2>(a, st);
        case 10: return run<P_FP8, 256, 256, 2, 4>(a, st);
        case 11: return run<P_FP32, 256, 128, 2, 2>(a, st);
        case 12: return launch_threshold_panel(P_BF16, false, a, st);
        case 13: return launch_threshold_panel(P_FP8, false, a, st);
        case 14: return launch_threshold_panel(P_BF16, true, a, st);
        case 15: return launch_threshold_panel(P_FP8, true, a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ej
