// gemm_threshold.hip -- the single-join threshold contraction kernel (LDS
// tile form; the tile body is in tile_body.hpp) and the table of tile shapes.
#include "common.hpp"
#include "launch.hpp"
#include "mma.hpp"
#include "tile_body.hpp"

namespace ej {

// Tiles of up to 128 x 128 are held to two resident workgroups per CU
// (256 registers per lane), which their accumulators allow.
template <int PREC, int BM, int BN, int WM, int WN, bool BIG = false>
__global__ __launch_bounds__(WM* WN * 64, (BM * BN <= 128 * 128) ? 2 : 1) void threshold_tile(
    const char* __restrict__ A, const char* __restrict__ B, const RowInfo* __restrict__ info_r,
    const RowInfo* __restrict__ info_s, int Kp_bytes, int64_t nR, int64_t nS,
    int tiles_m, int tiles_n, int ntiles, float lo, float hi, Pair* __restrict__ out,
    int64_t capacity, int2* __restrict__ band, int64_t band_cap,
    unsigned long long* __restrict__ hdr, int kg_last, int lohi_dev) {
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    // 2-D grid (a 1-D grid of this many workgroups would overflow the 32-bit
    // dispatch size); workgroups past the last tile leave at once
    int bid = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (bid >= ntiles) return;
    if (hdr[H_FLAGS] != 0) return;  // bad input rows: nothing to compute
    if (lohi_dev) {  // band edges measured on the device after prep
        lo = __uint_as_float((uint32_t)hdr[H_LO]);
        hi = __uint_as_float((uint32_t)hdr[H_HI]);
    }
    // Workgroups are dispatched to the 8 XCDs round-robin; remapping gives
    // each XCD a contiguous range of tiles, so the tiles that run together
    // on one XCD share operand panels in that XCD's L2.
    const int full = ntiles & ~7;
    if (bid < full) bid = (bid & 7) * (full >> 3) + (bid >> 3);
    int tm, tn;
    raster_tile(bid, tiles_m, tiles_n, tm, tn);
    if constexpr (BIG)
        big_tile_body<PREC>(sm, A, B, info_r, info_s, Kp_bytes, nR, nS, tm, tn, lo, hi, out,
                            capacity, hdr + H_OUT, band, band_cap, hdr + H_BAND, 0, nullptr,
                            nullptr, kg_last);
    else
        tile_body<PREC, BM, BN, WM, WN>(sm, A, B, info_r, info_s, Kp_bytes, nR, nS, tm, tn, lo,
                                        hi, out, capacity, hdr + H_OUT, band, band_cap,
                                        hdr + H_BAND, 0, nullptr, nullptr, kg_last);
}

// ---------------------------------------------------------------------------
// top-k candidate sweep on the LDS tile kernel (any row depth)
// ---------------------------------------------------------------------------
// Every accumulator at or above the floor F (float bits in hdr[H_TOPK_F])
// becomes a candidate (column, score) of its R row: the row's counter is
// raised by one atomicAdd per half-wave (the 32 lanes of a half hold one row
// of a 32x32 block, at different columns) and each hit takes the next slot;
// hits past Kc slots are counted, not written.  Counters start at zero.
template <int PREC>
__global__ __launch_bounds__(256, 2) void topk_cand_tile(
    const char* __restrict__ A, const char* __restrict__ B, const RowInfo* __restrict__ info_r,
    const RowInfo* __restrict__ info_s, int Kp_bytes, int64_t nR, int64_t nS, int tiles_m,
    int tiles_n, int ntiles, const unsigned long long* __restrict__ hdr, int* __restrict__ cnt,
    int2* __restrict__ cand, int Kc, const int* __restrict__ row_map,
    const float* __restrict__ floors) {
    constexpr int BM = 128, BN = 128, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    int bid = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (bid >= ntiles) return;
    if (hdr[H_FLAGS] != 0) return;
    const int full = ntiles & ~7;
    if (bid < full) bid = (bid & 7) * (full >> 3) + (bid >> 3);
    int tm, tn;
    raster_tile(bid, tiles_m, tiles_n, tm, tn);
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<PREC, BM, BN, WM, WN>(sm, A, B, info_r, info_s, Kp_bytes, tm, tn, acc);
    // with a row map, A holds gathered rows: row gi is R row row_map[gi],
    // swept with its own floor floors[gi]
    const float F0 = __uint_as_float((uint32_t)hdr[H_TOPK_F]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
    const uint32_t below_half = (1u << r32) - 1u;
#pragma unroll
    for (int i = 0; i < TG::FM; ++i)
#pragma unroll
        for (int j = 0; j < TG::FN; ++j) {
            const int64_t gj = (int64_t)tn * BN + wn * TG::WTN + j * 32 + r32;
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t gi =
                    (int64_t)tm * BM + wm * TG::WTM + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3);
                const float a = acc[i][j][e];
                const bool rin = gi < nR;
                const float F = (floors && rin) ? floors[gi] : F0;
                const bool hit = rin && gj < nS && a >= F;
                const uint64_t m = __ballot(hit);
                if (!m) continue;
                const int64_t ri = (row_map && rin) ? (int64_t)row_map[gi] : gi;
                const uint32_t mh = h ? (uint32_t)(m >> 32) : (uint32_t)m;
                // the lowest hitting lane of each half takes the half's slots
                const int leader = mh ? 32 * h + __builtin_ctz(mh) : lane;
                int base = 0;
                if (hit && lane == leader) base = atomicAdd(cnt + ri, __popc(mh));
                base = __shfl(base, leader, 64);
                if (hit) {
                    const int pos = base + __popc(mh & below_half);
                    if (pos < Kc) cand[ri * Kc + pos] = make_int2((int)gj, __float_as_int(a));
                }
            }
        }
}

template <int PREC>
static hipError_t run_cand_tile(const CandArgs& a, hipStream_t st) {
    const int64_t tm = (a.nR + 127) / 128, tn = (a.nS + 127) / 128;
    const int64_t nblocks = tm * tn;
    if (nblocks == 0) return hipSuccess;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const int64_t gx = nblocks < 65536 ? nblocks : 65536;
    const int64_t gy = (nblocks + gx - 1) / gx;
    if (gy > 65535) return hipErrorInvalidValue;
    const int kpb = a.Kp * (PREC == P_FP32 ? 4 : PREC == P_BF16 ? 2 : 1);
    hipLaunchKernelGGL((topk_cand_tile<PREC>), dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st,
                       (const char*)a.A, (const char*)a.B, a.info_r, a.info_s, kpb, a.nR, a.nS,
                       (int)tm, (int)tn, (int)nblocks, a.hdr, a.cnt, a.cand, a.Kc, a.row_map,
                       a.floors);
    return hipGetLastError();
}

hipError_t launch_topk_candidates_tile(int prec, const CandArgs& a, hipStream_t st) {
    switch (prec) {
        case P_FP32: return run_cand_tile<P_FP32>(a, st);
        case P_BF16: return run_cand_tile<P_BF16>(a, st);
        case P_FP8: return run_cand_tile<P_FP8>(a, st);
        default: return hipErrorInvalidValue;
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
    // 256 x 256 tiles, 128 x 128 per wave, staged single-pass epilogue
    {16, P_BF16, 256, 256, 64, "bf16:256x256x64/4w/staged"},
    {17, P_FP8, 256, 256, 128, "fp8:256x256x128/4w/staged"},
    {18, P_FP32, 256, 256, 32, "fp32:256x256x32/4w/staged"},
    // batches only: BF16 register panels of 128 rows, 128-column S tiles
    {19, P_BF16, 128, 128, 64, "bf16:panel/batch"},
    {20, P_FP32, 0, 0, 32, "fp32:panel"},
    {21, P_FP32, 0, 0, 32, "fp32:panel/2wg"},
    {22, P_BF16, 128, 128, 64, "bf16:panel/batch/2wg"},
    // the nested-loop comparator: one pair per wavefront, no tiling
    {kTileNlj, P_FP32, 0, 0, 32, "fp32:nlj"},
    // register panels with two 32-row blocks per wave (rows of 3-6 K slices)
    {24, P_BF16, 0, 0, 64, "bf16:panel/rb2"},
    {25, P_FP8, 0, 0, 128, "fp8:panel/rb2"},
};

int tile_count() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const TileDesc* tile_get(int id) {
    for (const auto& t : kTiles)
        if (t.id == id) return &t;
    return nullptr;
}

template <int PREC, int BM, int BN, int WM, int WN, bool BIG = false>
static hipError_t run(const ThresholdArgs& a, hipStream_t st) {
    const int64_t tm = (a.nR + BM - 1) / BM, tn = (a.nS + BN - 1) / BN;
    const int64_t nblocks = tm * tn;
    if (nblocks == 0) return hipSuccess;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const int64_t gx = nblocks < 65536 ? nblocks : 65536;
    const int64_t gy = (nblocks + gx - 1) / gx;
    if (gy > 65535) return hipErrorInvalidValue;
    const int kpb = a.Kp * (PREC == P_FP32 ? 4 : PREC == P_BF16 ? 2 : 1);
    hipLaunchKernelGGL((threshold_tile<PREC, BM, BN, WM, WN, BIG>), dim3((unsigned)gx, (unsigned)gy),
                       dim3(WM * WN * 64), 0, st, (const char*)a.A, (const char*)a.B, a.info_r,
                       a.info_s, kpb, a.nR,
                       a.nS, (int)tm, (int)tn, (int)nblocks, a.lo, a.hi, a.out, a.capacity, a.band, a.band_cap,
                       a.hdr, a.kg_last, a.lohi ? 1 : 0);
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
        case 12: return launch_threshold_panel(P_BF16, 0, a, st);
        case 13: return launch_threshold_panel(P_FP8, 0, a, st);
        case 14: return launch_threshold_panel(P_BF16, 1, a, st);
        case 15: return launch_threshold_panel(P_FP8, 1, a, st);
        case 20: return launch_threshold_panel(P_FP32, 0, a, st);
        case 21: return launch_threshold_panel(P_FP32, 1, a, st);
        case 24: return launch_threshold_panel(P_BF16, 2, a, st);
        case 25: return launch_threshold_panel(P_FP8, 2, a, st);
        case 16: return run<P_BF16, 256, 256, 2, 2, true>(a, st);
        case 17: return run<P_FP8, 256, 256, 2, 2, true>(a, st);
        case 18: return run<P_FP32, 256, 256, 2, 2, true>(a, st);
        case kTileNlj: return launch_threshold_nlj(a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace ej
