// tile_body.hpp -- one BM x BN output tile of the threshold contraction
// (shared by the single-join kernel and the persistent batch kernel).
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
#pragma once

#include <type_traits>

#include "common.hpp"
#include "epi_stage.hpp"
#include "mma.hpp"

namespace ej {

template <int BM, int BN, int NW>
struct TileSmem {
    __attribute__((aligned(16))) char sA[2][BM * 128];
    __attribute__((aligned(16))) char sB[2][BN * 128];
    uint32_t s_cnt[2 * NW];
    unsigned long long s_base[2];
};

// Grouped rasterisation of a tile index: GROUP_M tile rows at a time.
__device__ __forceinline__ void raster_tile(int bid, int tiles_m, int tiles_n, int& tm, int& tn) {
    constexpr int GROUP_M = 8;
    const int per_group = GROUP_M * tiles_n;
    const int grp = bid / per_group;
    const int first_m = grp * GROUP_M;
    const int gsize = min(tiles_m - first_m, GROUP_M);
    const int in_grp = bid - grp * per_group;
    tm = first_m + in_grp % gsize;
    tn = in_grp / gsize;
}

// Shape constants of a BM x BN tile computed by WM x WN waves.
template <int BM, int BN, int WM, int WN>
struct TileGeom {
    static constexpr int NT = WM * WN * 64;
    static constexpr int NW = WM * WN;
    static constexpr int WTM = BM / WM;  // rows per wave
    static constexpr int WTN = BN / WN;  // cols per wave
    static constexpr int FM = WTM / 32;  // 32x32 blocks per wave
    static constexpr int FN = WTN / 32;
    static constexpr int CA = BM * 8 / NT;  // 16-byte chunks per thread per slice
    static constexpr int CB = BN * 8 / NT;
    static_assert(CA * NT == BM * 8 && CB * NT == BN * 8, "tile/thread mismatch");
};

// Contraction of tile (tm, tn): acc[i][j] receives the 32x32 block (i, j)
// of this wave's WTM x WTN part of A_tile B_tile^T.  Both operands are
// K-contiguous rows of Kp_bytes bytes (a multiple of 128); rows up to the
// end of the tile must be readable.  info_r / info_s give the FP8 row scales
// (unused otherwise).  Only the first kg_last k-groups of the last slice are
// contracted (the rest of it is zero padding).  All threads of the workgroup
// call this.
template <int PREC, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void tile_mainloop(
    TileSmem<BM, BN, WM * WN>& sm, const char* __restrict__ A, const char* __restrict__ B,
    const RowInfo* __restrict__ info_r, const RowInfo* __restrict__ info_s, int Kp_bytes, int tm,
    int tn, v16f (&acc)[TileGeom<BM, BN, WM, WN>::FM][TileGeom<BM, BN, WM, WN>::FN],
    int kg_last = Mma<PREC>::GROUPS) {
    typedef TileGeom<BM, BN, WM, WN> TG;
    constexpr int NT = TG::NT;
    constexpr int WTM = TG::WTM, WTN = TG::WTN, FM = TG::FM, FN = TG::FN;
    constexpr int CA = TG::CA, CB = TG::CB;
    typedef Mma<PREC> M;
    auto& sA = sm.sA;
    auto& sB = sm.sB;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int h = lane >> 5, r32 = lane & 31;

    const char* Ag = A + (int64_t)tm * BM * Kp_bytes;
    const char* Bg = B + (int64_t)tn * BN * Kp_bytes;
    const int nk = Kp_bytes >> 7;

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

    // the matrix-core steps of the first NG k-groups of the slice in stage st
    auto compute = [&](int st, auto ng_c) {
        constexpr int NG = decltype(ng_c)::value;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
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
            // sub-steps outermost: consecutive matrix-core steps go to
            // different accumulators, none waits on the previous one
#pragma unroll
            for (int u = 0; u < M::SUB; ++u)
#pragma unroll
                for (int i = 0; i < FM; ++i)
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        M::mma_sub(fa[i], fb[j], acc[i][j], sa[i], sb[j], u);
        }
    };

    gload(0);
    lstore(0);
    __syncthreads();
    for (int kb = 0; kb + 1 < nk; ++kb) {
        const int st = kb & 1;
        gload(kb + 1);
        compute(st, std::integral_constant<int, M::GROUPS>{});
        lstore(st ^ 1);
        __syncthreads();
    }
    const int st_last = (nk - 1) & 1;
    if constexpr (BM * BN > 128 * 128) {
        // the largest tiles have no registers to spare for more copies of
        // the slice code: they contract the last slice whole
        compute(st_last, std::integral_constant<int, M::GROUPS>{});
    } else {
        // last slice: only its k-groups that hold data (a uniform switch, so
        // the steady-state loop above keeps its fully unrolled schedule)
        switch (kg_last) {
            case 1: compute(st_last, std::integral_constant<int, 1>{}); break;
            case 2:
                if constexpr (M::GROUPS >= 2) compute(st_last, std::integral_constant<int, 2>{});
                break;
            case 3:
                if constexpr (M::GROUPS >= 3) compute(st_last, std::integral_constant<int, 3>{});
                break;
            default: compute(st_last, std::integral_constant<int, M::GROUPS>{}); break;
        }
    }
    __syncthreads();
}

// All threads of the workgroup call this for tile (tm, tn).  out_ctr and
// band_ctr count the pairs appended to `out` and to the band list.  Band
// entries are int2 {r, s}, or, with TAG, int4 {r, s, job, 0} (one band list
// shared by the jobs of a batch).  perm_r / perm_s (may be null) map the
// operand rows back to the caller's rows when the operands were reordered.
template <int PREC, int BM, int BN, int WM, int WN, bool TAG = false>
__device__ __forceinline__ void tile_body(
    TileSmem<BM, BN, WM * WN>& sm, const char* __restrict__ A, const char* __restrict__ B,
    const RowInfo* __restrict__ info_r, const RowInfo* __restrict__ info_s, int Kp_bytes,
    int64_t nR, int64_t nS, int tm, int tn, float lo, float hi, Pair* __restrict__ out,
    int64_t capacity, unsigned long long* __restrict__ out_ctr, void* __restrict__ band,
    int64_t band_cap, unsigned long long* __restrict__ band_ctr, int job = 0,
    const int32_t* __restrict__ perm_r = nullptr, const int32_t* __restrict__ perm_s = nullptr,
    int kg_last = Mma<PREC>::GROUPS) {
    typedef TileGeom<BM, BN, WM, WN> TG;
    constexpr int NW = TG::NW;
    constexpr int WTM = TG::WTM, WTN = TG::WTN, FM = TG::FM, FN = TG::FN;
    auto& s_cnt = sm.s_cnt;
    auto& s_base = sm.s_base;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int h = lane >> 5, r32 = lane & 31;

    v16f acc[FM][FN];
    tile_mainloop<PREC, BM, BN, WM, WN>(sm, A, B, info_r, info_s, Kp_bytes, tm, tn, acc, kg_last);

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
        s_base[0] = tc ? atomicAdd(out_ctr, tc) : 0ull;
        s_base[1] = tb ? atomicAdd(band_ctr, tb) : 0ull;
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
                    const bool hit = (mlo >> lane) & 1ull;
                    int32_t ri = (int32_t)gi, si = (int32_t)gj;
                    if (hit && perm_r) {
                        ri = perm_r[gi];
                        si = perm_s[gj];
                    }
                    if ((mhi >> lane) & 1ull) {
                        const unsigned long long p = oc + lanes_below(mhi);
                        if ((int64_t)p < capacity) {
                            Pair pr;
                            pr.r = ri;
                            pr.s = si;
                            pr.score = a;
                            out[p] = pr;
                        }
                    }
                    if ((mb >> lane) & 1ull) {
                        const unsigned long long p = ob + lanes_below(mb);
                        if ((int64_t)p < band_cap) {
                            if (TAG)
                                ((int4*)band)[p] = make_int4(ri, si, job, 0);
                            else
                                ((int2*)band)[p] = make_int2(ri, si);
                        }
                    }
                    oc += __popcll(mhi);
                    ob += __popcll(mb);
                }
            }
}

// 256 x 256 tiles computed by 4 waves of 128 x 128 each: per K slice a wave
// reads 32 KB of fragments from LDS for 64 matrix-core steps, which keeps
// the LDS below the matrix cores' pace; the 256 accumulators per lane fill
// the accumulation registers, so the epilogue works in one pass and stages
// its hits in the operand LDS, which is idle once the contraction is done.
template <int PREC, bool TAG = false>
__device__ __forceinline__ void big_tile_body(
    TileSmem<256, 256, 4>& sm, const char* __restrict__ A, const char* __restrict__ B,
    const RowInfo* __restrict__ info_r, const RowInfo* __restrict__ info_s, int Kp_bytes,
    int64_t nR, int64_t nS, int tm, int tn, float lo, float hi, Pair* __restrict__ out,
    int64_t capacity, unsigned long long* __restrict__ out_ctr, void* __restrict__ band,
    int64_t band_cap, unsigned long long* __restrict__ band_ctr, int job = 0,
    const int32_t* __restrict__ perm_r = nullptr, const int32_t* __restrict__ perm_s = nullptr,
    int kg_last = Mma<PREC>::GROUPS) {
    typedef TileGeom<256, 256, 2, 2> TG;
    typedef typename BandEntryT<TAG>::type BE;
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<PREC, 256, 256, 2, 2>(sm, A, B, info_r, info_s, Kp_bytes, tm, tn, acc, kg_last);
    // the mainloop ends on a barrier: the operand LDS is free for staging
    constexpr int PER_WAVE = ST_OUT * (int)sizeof(Pair) + ST_BAND * (int)sizeof(BE);
    static_assert(4 * PER_WAVE <= (int)sizeof(sm.sA), "staging does not fit");
    const int wave = threadIdx.x >> 6;
    const int wm = wave / 2, wn = wave % 2;
    char* base = &sm.sA[0][0] + wave * PER_WAVE;
    const bool edge = ((int64_t)(tm + 1) * 256 > nR) || ((int64_t)(tn + 1) * 256 > nS);
    stage_epilogue<TG::FM, TG::FN, TAG>(acc, (int64_t)tm * 256 + wm * TG::WTM,
                                        (int64_t)tn * 256 + wn * TG::WTN, edge, nR, nS, lo, hi,
                                        out, capacity, out_ctr, band, band_cap, band_ctr, job,
                                        perm_r, perm_s, (Pair*)base,
                                        (BE*)(base + ST_OUT * sizeof(Pair)));
    __syncthreads();  // staging area is the next tile's operand buffer
}

}  // namespace ej

