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

// LDS of one tile: two slots per operand for the K slices.  The four slots
// are separate LDS arrays (declared by EJ_TILE_SMEM in the kernel), so the
// compiler can tell the slot being filled by direct loads from the slot being
// read and does not wait for the fills before every LDS read.
template <int BM, int BN, int NW>
struct TileSmem {
    char* a[2];
    char* b[2];
    uint32_t* s_cnt;             // 2 * NW wave counts
    unsigned long long* s_base;  // 2 list bases
};

#define EJ_TILE_SMEM(BM_, BN_, NW_, name)                                                  \
    __shared__ __attribute__((aligned(16))) char name##_a0[(BM_) * 128];                   \
    __shared__ __attribute__((aligned(16))) char name##_a1[(BM_) * 128];                   \
    __shared__ __attribute__((aligned(16))) char name##_b0[(BN_) * 128];                   \
    __shared__ __attribute__((aligned(16))) char name##_b1[(BN_) * 128];                   \
    __shared__ uint32_t name##_cnt[2 * (NW_)];                                             \
    __shared__ unsigned long long name##_base[2];                                          \
    TileSmem<BM_, BN_, NW_> name = {{name##_a0, name##_a1}, {name##_b0, name##_b1}, name##_cnt, \
                                    name##_base}

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
//
// K slices (128 bytes per row) go from global memory straight into LDS
// (direct loads, no staging registers): slice kb + 1 is filled into one slot
// while slice kb is multiplied out of the other.  A slice of R rows is R / 8
// blocks of 1 KB; instruction i of wave w fills block NW i + w, lane l writing
// the 16 bytes at l * 16, so the lane loads the chunk that the XOR swizzle of
// lds_off places there (its row is 8 (NW i + w) + l / 8, its chunk
// (l % 8) ^ ((row / 2) % 8), which does not depend on i for an even NW).
template <int PREC, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void tile_mainloop(
    TileSmem<BM, BN, WM * WN>& sm, const char* __restrict__ A, const char* __restrict__ B,
    const RowInfo* __restrict__ info_r, const RowInfo* __restrict__ info_s, int Kp_bytes, int tm,
    int tn, v16f (&acc)[TileGeom<BM, BN, WM, WN>::FM][TileGeom<BM, BN, WM, WN>::FN],
    int kg_last = Mma<PREC>::GROUPS) {
    typedef TileGeom<BM, BN, WM, WN> TG;
    constexpr int NW = TG::NW;
    constexpr int WTM = TG::WTM, WTN = TG::WTN, FM = TG::FM, FN = TG::FN;
    constexpr int NFA = BM / (8 * NW), NFB = BN / (8 * NW);  // fills per wave and slice
    static_assert(NFA * 8 * NW == BM && NFB * 8 * NW == BN && NW % 2 == 0,
                  "the tile rows must spread evenly over the waves' fills");
    typedef Mma<PREC> M;

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

    // the wave index as a wave-uniform value: the LDS address of a direct
    // load goes through m0
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    const int frow = wave_u * 8 + (lane >> 3);
    const int64_t loff = (int64_t)frow * Kp_bytes + (((lane & 7) ^ ((frow >> 1) & 7)) << 4);
    const int64_t istride = (int64_t)8 * NW * Kp_bytes;
    auto fill = [&](auto st_c, int kb) {
        constexpr int st = decltype(st_c)::value;
        const char* ga = Ag + kb * 128 + loff;
        const char* gb = Bg + kb * 128 + loff;
#pragma unroll
        for (int i = 0; i < NFA; ++i) lds_fill16(ga + i * istride, sm.a[st] + (NW * i + wave_u) * 1024);
#pragma unroll
        for (int i = 0; i < NFB; ++i) lds_fill16(gb + i * istride, sm.b[st] + (NW * i + wave_u) * 1024);
    };

    // the matrix-core steps of the first NG k-groups of the slice in slot st
    auto compute = [&](auto st_c, auto ng_c) {
        constexpr int st = decltype(st_c)::value;
        constexpr int NG = decltype(ng_c)::value;
        const char* la = sm.a[st];
        const char* lb = sm.b[st];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            typename M::Frag fa[FM], fb[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int row = wm * WTM + i * 32 + r32;
#pragma unroll
                for (int c = 0; c < M::CPL; ++c) {
                    v4i v = *(const v4i*)(la + lds_off(row, M::chunk(g, h, c)));
#pragma unroll
                    for (int e = 0; e < 4; ++e) fa[i][c * 4 + e] = v[e];
                }
            }
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int row = wn * WTN + j * 32 + r32;
#pragma unroll
                for (int c = 0; c < M::CPL; ++c) {
                    v4i v = *(const v4i*)(lb + lds_off(row, M::chunk(g, h, c)));
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
    // last slice: only its k-groups that hold data (a uniform switch, so the
    // steady-state steps keep their fully unrolled schedule); the largest
    // tiles have no registers to spare for more copies of the slice code and
    // contract it whole
    auto last = [&](auto st_c) {
        if constexpr (BM * BN > 128 * 128) {
            compute(st_c, std::integral_constant<int, M::GROUPS>{});
        } else {
            switch (kg_last) {
                case 1: compute(st_c, std::integral_constant<int, 1>{}); break;
                case 2:
                    if constexpr (M::GROUPS >= 2) compute(st_c, std::integral_constant<int, 2>{});
                    break;
                case 3:
                    if constexpr (M::GROUPS >= 3) compute(st_c, std::integral_constant<int, 3>{});
                    break;
                default: compute(st_c, std::integral_constant<int, M::GROUPS>{}); break;
            }
        }
    };
    typedef std::integral_constant<int, 0> S0;
    typedef std::integral_constant<int, 1> S1;
    typedef std::integral_constant<int, M::GROUPS> GALL;

    // Step over slice kb in slot kb % 2: its fills (issued one step earlier)
    // have landed once this wave's loads are done; the barrier publishes every
    // wave's part and retires the reads of slice kb - 1, whose slot slice
    // kb + 1 takes.
    fill(S0{}, 0);
    if constexpr (BM * BN > 128 * 128) {
        // largest tiles: a branch-free loop over pairs of slices (the 256
        // accumulators per lane leave the register allocator no room for
        // the copies that merging branches would need); past the last slice
        // the fill reloads it (never read)
        const int nk2 = nk & ~1;
        for (int kb = 0; kb < nk2; kb += 2) {
            wait_vmcnt_lgkm0<0>();
            bare_barrier();
            fill(S1{}, kb + 1);
            compute(S0{}, GALL{});
            wait_vmcnt_lgkm0<0>();
            bare_barrier();
            fill(S0{}, min(kb + 2, nk - 1));
            compute(S1{}, GALL{});
        }
        wait_vmcnt_lgkm0<0>();
        bare_barrier();
        if (nk & 1) compute(S0{}, GALL{});
    } else {
        for (int kb = 0; kb < nk; kb += 2) {
            wait_vmcnt_lgkm0<0>();
            bare_barrier();
            if (kb + 1 < nk) {
                fill(S1{}, kb + 1);
                compute(S0{}, GALL{});
                wait_vmcnt_lgkm0<0>();
                bare_barrier();
                if (kb + 2 < nk) {
                    fill(S0{}, kb + 2);
                    compute(S1{}, GALL{});
                } else {
                    last(S1{});
                }
            } else {
                last(S0{});
            }
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
    // (two waves per 32 KB operand slot)
    constexpr int PER_WAVE = ST_OUT * (int)sizeof(Pair) + ST_BAND * (int)sizeof(BE);
    static_assert(2 * PER_WAVE <= 256 * 128, "staging does not fit");
    const int wave = threadIdx.x >> 6;
    const int wm = wave / 2, wn = wave % 2;
    char* base = (wave < 2 ? sm.a[0] : sm.b[0]) + (wave & 1) * PER_WAVE;
    const bool edge = ((int64_t)(tm + 1) * 256 > nR) || ((int64_t)(tn + 1) * 256 > nS);
    stage_epilogue<TG::FM, TG::FN, TAG>(acc, (int64_t)tm * 256 + wm * TG::WTM,
                                        (int64_t)tn * 256 + wn * TG::WTN, edge, nR, nS, lo, hi,
                                        out, capacity, out_ctr, band, band_cap, band_ctr, job,
                                        perm_r, perm_s, (Pair*)base,
                                        (BE*)(base + ST_OUT * sizeof(Pair)));
    __syncthreads();  // staging area is the next tile's operand buffer
}

}  // namespace ej

