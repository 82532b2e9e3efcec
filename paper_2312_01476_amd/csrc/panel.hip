// panel.hip -- register-resident R panels for the narrow-format contraction.
//
// The tensor join's cache argument (Section IV.C: a block of vectors stays in
// cache and is reused across many products) is taken here to the register
// file.  A workgroup of NW waves owns a panel of 32 * RB * NW R rows (32 * RB
// per wave); each wave loads its rows' BF16 or FP8 MFMA operand fragments
// into VGPRs once and keeps them while the workgroup sweeps a range of S
// tiles (32 * CB columns each).  S slices (128 bytes of K per row) stream
// through an LDS ring shared by the waves, so per MFMA only the S operand is
// read from LDS and only S traffic reaches L2.  With K short (a few hundred),
// this removes the per-output-tile prologue that a classic tile kernel pays
// for every block of D (Section V.B's mini-batch slowdown, at tile scale).
//
// The ring is filled either through registers (two slots, one slice ahead)
// or by direct global->LDS loads into NSLOT slots, NSLOT - 1 slices ahead of
// the MFMAs.
//
// The accumulators of each S tile go to an epilogue policy:
//  * ThresholdEpi -- the threshold predicate of the E-theta-join: groups of
//    four scores that may reach the band are staged per wave in LDS as
//    records and split into certain and band pairs when the stage is
//    written out, with one atomicAdd per list and stage;
//  * CandEpi -- top-k candidates: every column with score >= a floor goes to
//    its row's candidate slots (the workgroup sweeps all of S, so each row is
//    owned by one wave and its counter lives in LDS).
#include "batch.hpp"
#include "common.hpp"
#include "epi_stage.hpp"
#include "launch.hpp"
#include "mma.hpp"

namespace ej {

// Staged candidate records per wave.  A record is one lane's group of four
// accumulators (four rows of one S column) whose maximum reaches the band;
// records are split into certain pairs and band pairs only when the stage
// is written out.
constexpr int PN_RECCAP = 320;   // threshold epilogue
constexpr int PN_CANDCAP = 256;  // top-k candidate epilogue

// Exclusive prefix sum over the lanes of a wave of a per-lane count in
// [0, 7] (one ballot per bit), and the wave's total.
__device__ __forceinline__ uint32_t lane_prefix7(uint32_t c, uint32_t& total) {
    const uint64_t b0 = __ballot(c & 1u), b1 = __ballot(c & 2u), b2 = __ballot(c & 4u);
    total = (uint32_t)__popcll(b0) + 2u * (uint32_t)__popcll(b1) + 4u * (uint32_t)__popcll(b2);
    return lanes_below(b0) + 2u * lanes_below(b1) + 4u * lanes_below(b2);
}

// Screening of one wave's S tile against lo: one wave mask per group of
// four accumulators (four rows of one column) from a compare of their
// maximum, no branches.  Each flagged lane of a group then stages the group
// as one record (the four scores; the first row and the column) at
// val/pos[n]; pre() runs between the screening and the staging, and a
// 32 x 32 block first calls make_room() when its records would not fit in
// CAP, so that call is inlined once per block.
template <int RB, int CB, int CAP, class Pre, class MakeRoom>
__device__ __forceinline__ void stage_records(v16f (&acc)[RB][CB], float lo, float4* val,
                                              int2* pos, int& n, int gi0, int gj0, Pre&& pre,
                                              MakeRoom&& make_room) {
    bool hit[RB][CB][4];
    uint64_t gmask[RB][CB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                const int e4 = 4 * q4;
                const float m4 =
                    __builtin_fmaxf(__builtin_fmaxf(acc[rb][cb][e4], acc[rb][cb][e4 + 1]),
                                    __builtin_fmaxf(acc[rb][cb][e4 + 2], acc[rb][cb][e4 + 3]));
                hit[rb][cb][q4] = m4 >= lo;
                gmask[rb][cb][q4] = __ballot(hit[rb][cb][q4]);
            }
    pre();
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const uint64_t* g = gmask[rb][cb];
            if (!(g[0] | g[1] | g[2] | g[3])) continue;
            const int need = __popcll(g[0]) + __popcll(g[1]) + __popcll(g[2]) + __popcll(g[3]);
            if (n + need > CAP) make_room();
#pragma unroll
            for (int q4 = 0; q4 < 4; ++q4) {
                if (!g[q4]) continue;
                if (hit[rb][cb][q4]) {
                    const int e = n + (int)lanes_below(g[q4]);
                    const int e4 = 4 * q4;
                    val[e] = make_float4(acc[rb][cb][e4], acc[rb][cb][e4 + 1], acc[rb][cb][e4 + 2],
                                         acc[rb][cb][e4 + 3]);
                    pos[e] = make_int2(gi0 + rb * 32 + 8 * q4, gj0 + cb * 32);
                }
                n += __popcll(g[q4]);
            }
        }
}

// Position of the accumulators: element e of 32x32 block (rb, cb) of a lane
// is row 8*(e/4) + 4*h + e%4 of the block and column r32 (h = lane / 32).
struct TileCtx {
    int lane, wave, h, r32;
    int r0;       // first R row of the wave
    int rows;     // R rows per wave (32 * RB)
    int t;        // S tile index
    int bn;       // columns per S tile
    bool edge;    // tile touches the end of R or S
    int64_t nR, nS;
};

// ---------------------------------------------------------------------------
// threshold epilogue (NW waves per workgroup)
// ---------------------------------------------------------------------------
struct ThresholdParams {
    float lo, hi;
    // when set: the band edges are read from lohi[0], lohi[1] (float bits)
    // at the start of the sweep instead of lo, hi
    const unsigned long long* lohi;
    Pair* out;
    int64_t capacity;
    unsigned long long* out_ctr;   // pairs appended to out
    void* band;                    // int2 {r, s}, or int4 {r, s, job, 0} with TAG
    int64_t band_cap;
    unsigned long long* band_ctr;  // band entries found
    int job;
    // with PERM (prefiltered batch): prepared row -> caller's row maps of
    // the prefilter order
    const int32_t* perm_r;
    const int32_t* perm_s;
};

template <int NW, bool TAG, bool PERM = false>
struct ThresholdEpiT {
    typedef ThresholdParams Params;
    typedef typename BandEntryT<TAG>::type BE;
    struct Smem {
        float4 val[NW][PN_RECCAP];  // a record's four scores (rows r .. r + 3)
        int2 pos[NW][PN_RECCAP];    // its first row r and its column
        int flush_at;               // the tile step at which every wave writes out
    };
    struct State {
        int n_rec;       // staged records of this wave (wave-uniform)
        int step;        // S tiles of the sweep so far (the same in every wave)
        float lo, hi;    // band edges of this sweep
    };
    // staged records from which a wave asks the workgroup to write out
    static constexpr int kWriteOutAt = PN_RECCAP / 2;

    __device__ static __forceinline__ void init(const Params& p, Smem& sm, State& s, const TileCtx&) {
        s.n_rec = 0;
        s.step = 0;
        __hip_atomic_store(&sm.flush_at, -1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        s.lo = p.lohi ? __uint_as_float((uint32_t)p.lohi[0]) : p.lo;
        s.hi = p.lohi ? __uint_as_float((uint32_t)p.lohi[1]) : p.hi;
    }

    // Certain (score >= hi) and band (lo <= score < hi) masks of the four
    // rows of staged record e, for rows inside R and a column inside S.
    __device__ static __forceinline__ void record_masks(const Smem& sm, const State& s,
                                                        const TileCtx& c, int e, int nR32,
                                                        int nS32, float (&a)[4], int2& rc,
                                                        uint32_t& mo, uint32_t& mb) {
        const bool have = e < s.n_rec;
        const float4 a4 = sm.val[c.wave][have ? e : 0];
        rc = sm.pos[c.wave][have ? e : 0];
        a[0] = a4.x;
        a[1] = a4.y;
        a[2] = a4.z;
        a[3] = a4.w;
        const bool col = have && rc.y < nS32;
        mo = 0;
        mb = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool ok = col && rc.x + k < nR32;
            mo |= (uint32_t)(ok && a[k] >= s.hi) << k;
            mb |= (uint32_t)(ok && a[k] >= s.lo && a[k] < s.hi) << k;
        }
    }

    // Write the staged records out, one per lane: the rows inside R and S
    // are split into certain pairs and band pairs.  A first pass over the
    // records sizes both lists' shares, so that each list takes one
    // atomicAdd (both in flight together); one more pass per list writes
    // its entries.
    // Entries past a list's capacity are dropped (its counter still counts
    // them, so the caller learns the true size).
    __device__ static __forceinline__ void flush(const Params& p, Smem& sm, State& s,
                                                 const TileCtx& c) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int nR32 = c.nR < 0x7fffffff ? (int)c.nR : 0x7fffffff;
        const int nS32 = c.nS < 0x7fffffff ? (int)c.nS : 0x7fffffff;
        uint32_t tot_o = 0, tot_b = 0;  // wave-uniform
        for (int e0 = 0; e0 < s.n_rec; e0 += 64) {
            float a[4];
            int2 rc;
            uint32_t mo, mb, no, nb;
            record_masks(sm, s, c, e0 + c.lane, nR32, nS32, a, rc, mo, mb);
            lane_prefix7(__popc(mo), no);
            lane_prefix7(__popc(mb), nb);
            tot_o += no;
            tot_b += nb;
        }
        unsigned long long bo = 0, bb = 0;
        if (c.lane == 0) {
            if (tot_o) bo = atomicAdd(p.out_ctr, (unsigned long long)tot_o);
            if (tot_b) bb = atomicAdd(p.band_ctr, (unsigned long long)tot_b);
        }
        bo = ((unsigned long long)__builtin_amdgcn_readlane((uint32_t)(bo >> 32), 0) << 32) |
             __builtin_amdgcn_readlane((uint32_t)bo, 0);
        bb = ((unsigned long long)__builtin_amdgcn_readlane((uint32_t)(bb >> 32), 0) << 32) |
             __builtin_amdgcn_readlane((uint32_t)bb, 0);
        for (int e0 = 0; tot_o && e0 < s.n_rec; e0 += 64) {
            float a[4];
            int2 rc;
            uint32_t mo, mb, no;
            record_masks(sm, s, c, e0 + c.lane, nR32, nS32, a, rc, mo, mb);
            uint32_t po = lane_prefix7(__popc(mo), no);
            const int32_t sj = PERM && mo ? p.perm_s[rc.y] : rc.y;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((mo >> k) & 1u) {
                    const unsigned long long q = bo + po++;
                    if ((int64_t)q < p.capacity) {
                        Pair pr;
                        pr.r = PERM ? p.perm_r[rc.x + k] : rc.x + k;
                        pr.s = sj;
                        pr.score = a[k];
                        p.out[q] = pr;
                    }
                }
            }
            bo += no;
        }
        for (int e0 = 0; tot_b && e0 < s.n_rec; e0 += 64) {
            float a[4];
            int2 rc;
            uint32_t mo, mb, nb;
            record_masks(sm, s, c, e0 + c.lane, nR32, nS32, a, rc, mo, mb);
            uint32_t pb = lane_prefix7(__popc(mb), nb);
            const int32_t sj = PERM && mb ? p.perm_s[rc.y] : rc.y;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((mb >> k) & 1u) {
                    const unsigned long long q = bb + pb++;
                    if ((int64_t)q < p.band_cap) {
                        const int32_t ri = PERM ? p.perm_r[rc.x + k] : rc.x + k;
                        BE be;
                        if constexpr (TAG)
                            be = make_int4(ri, sj, p.job, 0);
                        else
                            be = make_int2(ri, sj);
                        ((BE*)p.band)[q] = be;
                    }
                }
            }
            bb += nb;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        s.n_rec = 0;
    }

    template <int RB, int CB>
    __device__ static __forceinline__ void tile(const Params& p, Smem& sm, State& s,
                                                v16f (&acc)[RB][CB], const TileCtx& c) {
        // the row numbers are the same for every tile of the sweep; an opaque
        // copy keeps the compiler from computing all of them once before the
        // sweep and holding them (or spilling them) across the matrix loop
        int gi0 = c.r0 + 4 * c.h;
        __asm__ volatile("" : "+v"(gi0));
        // The waves of a single join's workgroup write out together: a wave
        // whose stage passes kWriteOutAt names the next tile step, and at
        // that step every wave writes out what it holds.  Apart, each wave's
        // write-out would hold the other waves at the next barrier; together
        // they overlap.  (Only the timing depends on this flag: a block that
        // does not fit writes out at once.)  The batch kernels, whose jobs
        // are small and dense, write out on their own.
        if constexpr (!TAG) {
            const int fa =
                __hip_atomic_load(&sm.flush_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            stage_records<RB, CB, PN_RECCAP>(
                acc, s.lo, sm.val[c.wave], sm.pos[c.wave], s.n_rec, gi0, c.t * c.bn + c.r32,
                [&] {
                    if (__builtin_amdgcn_readfirstlane(fa) == s.step && s.n_rec)
                        flush(p, sm, s, c);
                },
                [&] { flush(p, sm, s, c); });
            if (s.n_rec > kWriteOutAt)
                __hip_atomic_store(&sm.flush_at, s.step + 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            ++s.step;
        } else {
            stage_records<RB, CB, PN_RECCAP>(acc, s.lo, sm.val[c.wave], sm.pos[c.wave], s.n_rec,
                                             gi0, c.t * c.bn + c.r32, [] {},
                                             [&] { flush(p, sm, s, c); });
        }
    }

    __device__ static __forceinline__ void finish(const Params& p, Smem& sm, State& s, const TileCtx& c) {
        if (s.n_rec) flush(p, sm, s, c);
    }
};

// ---------------------------------------------------------------------------
// top-k candidate epilogue: every (i, j) with approximate score >= floor goes
// to slot cnt[i]++ of row i (slots past Kc are counted, not written)
// ---------------------------------------------------------------------------
// the single-join form (untagged band entries)
template <int NW>
using ThresholdEpi = ThresholdEpiT<NW, false, false>;


struct CandParams {
    const unsigned long long* hdr;  // floor as float bits in H_TOPK_F
    int* cnt;                       // per R row, number of candidates seen
    int2* cand;                     // per R row, Kc slots of (j, score bits)
    int Kc;
};

template <int NW>
struct CandEpi {
    typedef CandParams Params;
    struct Smem {
        int cnt[NW][64];              // per wave, its (up to 64) rows
        float4 val[NW][PN_CANDCAP];   // staged records (see stage_records)
        int2 pos[NW][PN_CANDCAP];
    };
    struct State {
        int n_rec;  // staged records of this wave (wave-uniform)
        float floor;
    };

    __device__ static __forceinline__ void init(const Params& p, Smem& sm, State& s, const TileCtx& c) {
        s.n_rec = 0;
        s.floor = __uint_as_float((uint32_t)p.hdr[H_TOPK_F]);
        sm.cnt[c.wave][c.lane] = 0;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }

    // Write the staged records out, one per lane: every score >= floor of a
    // row inside R and a column inside S takes the next slot of its row (an
    // LDS atomic on the row's counter; slots past Kc are counted, not
    // written).  The order of a row's slots carries no meaning.
    __device__ static __forceinline__ void flush(const Params& p, Smem& sm, State& s,
                                                 const TileCtx& c) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        for (int e0 = 0; e0 < s.n_rec; e0 += 64) {
            const int e = e0 + c.lane;
            const bool have = e < s.n_rec;
            const float4 a4 = sm.val[c.wave][have ? e : 0];
            const int2 rc = sm.pos[c.wave][have ? e : 0];
            const float a[4] = {a4.x, a4.y, a4.z, a4.w};
            const bool col = have && rc.y < c.nS;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int gi = rc.x + k;
                if (col && gi < c.nR && a[k] >= s.floor) {
                    const int slot = atomicAdd(&sm.cnt[c.wave][gi - c.r0], 1);
                    if (slot < p.Kc)
                        p.cand[(int64_t)gi * p.Kc + slot] = make_int2(rc.y, __float_as_int(a[k]));
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        s.n_rec = 0;
    }

    template <int RB, int CB>
    __device__ static __forceinline__ void tile(const Params& p, Smem& sm, State& s,
                                                v16f (&acc)[RB][CB], const TileCtx& c) {
        int gi0 = c.r0 + 4 * c.h;
        __asm__ volatile("" : "+v"(gi0));
        stage_records<RB, CB, PN_CANDCAP>(acc, s.floor, sm.val[c.wave], sm.pos[c.wave], s.n_rec,
                                          gi0, c.t * c.bn + c.r32, [] {},
                                          [&] { flush(p, sm, s, c); });
    }

    __device__ static __forceinline__ void finish(const Params& p, Smem& sm, State& s, const TileCtx& c) {
        if (s.n_rec) flush(p, sm, s, c);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (c.lane < c.rows) p.cnt[c.r0 + c.lane] = sm.cnt[c.wave][c.lane];
    }
};

// ---------------------------------------------------------------------------
// the panel kernel
// ---------------------------------------------------------------------------
// Exponent of a positive normal power of two (the FP8 row multipliers).
__device__ __forceinline__ int pow2_exponent(float x) {
    return (int)((__float_as_uint(x) >> 23) & 0xffu) - 127;
}

// Direct-load fill of one ring slot with one K slice of an S tile (`src`: the
// slice's first byte, the same for the whole wave).  A slice is PN_BN rows of
// 128 bytes, i.e. PN_BN / 8 blocks of 1 KB; instruction i of wave w fills
// block b = NW i + w (rows 8 b .. 8 b + 7), lane l writing the 16 bytes at
// l * 16 of the block, so the lane loads the chunk that the XOR swizzle of
// lds_off places there: row r = 8 b + l / 8, chunk (l % 8) ^ ((r / 2) % 8).
// With NW even, r / 2 mod 8 does not depend on i, so the source offset of
// instruction i is that of i = 0 (ring_lane_offset) plus 8 NW i rows.
template <int KPB, int NW, int NCH>
__device__ __forceinline__ void ring_fill(char* dst, const char* src, uint32_t loff, int wave) {
#pragma unroll
    for (int i = 0; i < NCH; ++i)
        lds_fill16(src + loff + i * 8 * NW * KPB, dst + (NW * i + wave) * 1024);
}

template <int KPB>
__device__ __forceinline__ uint32_t ring_lane_offset(int wave, int lane) {
    const int row = wave * 8 + (lane >> 3);
    return (uint32_t)(row * KPB + (((lane & 7) ^ ((row >> 1) & 7)) << 4));
}

// One K slice of MFMAs: B fragments of slice `sl` from LDS against the
// resident A fragments of K slice ks.  The fragments of k-group g + 1 are read
// before the MFMAs of group g are issued, so the LDS latency of one group is
// hidden behind the matrix-core work of the previous one.
template <int PREC, int KS, int RB, int CB>
__device__ __forceinline__ void slice_mma(const char* sl, int ks,
                                          const typename Mma<PREC>::Frag (&af)[RB][KS * Mma<PREC>::GROUPS],
                                          v16f (&acc)[RB][CB], const int (&sa)[RB],
                                          const int (&sb)[CB], int h, int r32) {
    typedef Mma<PREC> M;
    constexpr int G = M::GROUPS;
    typename M::Frag fb[2][CB];
    auto read = [&](int g, typename M::Frag (&f)[CB]) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int row = cb * 32 + r32;
#pragma unroll
            for (int c = 0; c < M::CPL; ++c) {
                v4i v = *(const v4i*)(sl + lds_off(row, M::chunk(g, h, c)));
#pragma unroll
                for (int e = 0; e < 4; ++e) f[cb][c * 4 + e] = v[e];
            }
        }
    };
    read(0, fb[0]);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (g + 1 < G) read(g + 1, fb[(g + 1) & 1]);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
                M::mma(af[rb][ks * G + g], fb[g & 1][cb], acc[rb][cb], sa[rb], sb[cb]);
    }
    // schedule: the reads of group 0, then each MFMA of group g followed by
    // one read of group g + 1
    __builtin_amdgcn_sched_group_barrier(0x100, CB * M::CPL, 0);
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int i = 0; i < RB * CB; ++i) {
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            if (g + 1 < G && i < CB * M::CPL) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        }
}

// Template parameters: RB 32-row blocks per wave, CB 32-column blocks per S
// tile, KS 128-byte K slices per row, NW waves per workgroup, OCC workgroups
// per CU, NSLOT ring slots of direct loads (0: the register-staged two-slot
// ring).  With direct loads, slice q of the sweep sits in slot q % NSLOT and
// is filled NSLOT - 1 slices ahead; KS is a multiple of NSLOT, so the slot of
// every slice is known at compile time.  The slots are separate LDS arrays,
// which lets the compiler see that the fills in flight never touch the slot
// being read and keeps it from waiting for them before the LDS reads (the
// waits for the fills are the explicit vmcnt waits).
// The sweep of one R panel over S tiles [t0, t1): resident R fragments,
// S slices through the LDS ring `slots` (see panel_kernel), one epilogue per
// S tile.  All threads of the workgroup call this; it ends with every fill
// landed and the epilogue's staging flushed.
template <int PREC, int KS, int RB, int CB, int NW, int NSLOT, class EPI, bool MASK = false>
__device__ __forceinline__ void panel_sweep(char* const (&slots)[6], typename EPI::Smem& esm,
                                            const char* __restrict__ A,
                                            const char* __restrict__ B,
                                            const RowInfo* __restrict__ info_r,
                                            const RowInfo* __restrict__ info_s, int64_t nR,
                                            int64_t nS, int panel, int t0, int t1,
                                            const typename EPI::Params& ep, uint64_t mask = 0) {
    typedef Mma<PREC> M;
    constexpr int G = M::GROUPS;
    constexpr int NF = KS * G;        // A fragments per 32-row block
    constexpr int KPB = KS * 128;     // bytes per operand row
    constexpr int PN_BN = 32 * CB;
    constexpr int PN_ROWS = 32 * RB * NW;
    constexpr int NT = 64 * NW;       // threads
    constexpr int SLOT = PN_BN * 128;
    constexpr bool DMA = NSLOT > 0;
    constexpr int NS = DMA ? NSLOT : 2;
    constexpr int NCH = PN_BN * 8 / NT;  // 16-byte chunks per thread per S slice
    static_assert(NCH >= 1 && NCH * NT == PN_BN * 8, "slice chunks must spread evenly");
    static_assert(NW % 2 == 0, "the fill offsets assume an even wave count");
    static_assert(!DMA || (NSLOT >= 2 && NSLOT <= 6 && KS % NSLOT == 0),
                  "direct loads need a static ring slot per slice");
    static_assert(!MASK || (DMA && NSLOT <= KS), "masked sweeps run on the direct-load ring");
    constexpr int D = NS - 1;  // fill distance of the direct-load ring
    // MASK: the sweep visits only S tiles t0 + b for the set bits b of
    // `mask` (at least one, all below t1 - t0 <= 64), in increasing order
    auto next_tile = [&](int t) -> int {
        if constexpr (MASK) {
            const uint64_t above =
                t - t0 >= 63 ? 0ull : mask & ~((2ull << (t - t0)) - 1ull);
            return above ? t0 + __builtin_ctzll(above) : t1;
        } else {
            return t + 1;
        }
    };
    const int tfirst = MASK ? t0 + __builtin_ctzll(mask) : t0;

    char* const sL0 = slots[0];
    char* const sL1 = slots[1];
    TileCtx ctx;
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    ctx.lane = tid & 63;
    ctx.wave = tid >> 6;
    ctx.h = ctx.lane >> 5;
    ctx.r32 = ctx.lane & 31;
    ctx.r0 = panel * PN_ROWS + ctx.wave * 32 * RB;
    ctx.rows = 32 * RB;
    ctx.bn = PN_BN;
    ctx.nR = nR;
    ctx.nS = nS;
    ctx.t = tfirst;
    ctx.edge = false;
    const int h = ctx.h, r32 = ctx.r32, r0 = ctx.r0;

    // ---- R fragments, resident for the whole sweep ----
    typename M::Frag af[RB][NF];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const char* ar = A + (int64_t)(r0 + rb * 32 + r32) * KPB;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int c = 0; c < M::CPL; ++c) {
                    v4i v = *(const v4i*)(ar + ks * 128 + M::chunk(g, h, c) * 16);
#pragma unroll
                    for (int e = 0; e < 4; ++e) af[rb][ks * G + g][c * 4 + e] = v[e];
                }
    }
    int sa[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
        sa[rb] = PREC == P_FP8 ? 127 - pow2_exponent(info_r[r0 + rb * 32 + r32].qscale) : 127;

    v16f acc[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    typename EPI::State est;
    EPI::init(ep, esm, est, ctx);
    const bool redge = (int64_t)panel * PN_ROWS + PN_ROWS > nR;

    // register-staged ring: slice q + 1 goes through registers into slot
    // (q + 1) % 2 while slice q is multiplied
    const int nq = (t1 - t0) * KS;
    v4i rbuf[NCH];
    auto gload = [&](int q) {
        const int t = t0 + q / KS, ks = q - (q / KS) * KS;
        const char* base = B + (int64_t)t * PN_BN * KPB + ks * 128;
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int qq = tid + i * NT;
            rbuf[i] = *(const v4i*)(base + (int64_t)(qq >> 3) * KPB + (qq & 7) * 16);
        }
    };
    auto lstore = [&](char* slot) {
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int qq = tid + i * NT;
            *(v4i*)(slot + lds_off(qq >> 3, qq & 7)) = rbuf[i];
        }
    };

    // the wave index as a wave-uniform (scalar) value: the LDS address of a
    // direct load goes through m0
    const int wave_u = __builtin_amdgcn_readfirstlane(ctx.wave);
    const uint32_t loff = ring_lane_offset<KPB>(wave_u, ctx.lane);
    if constexpr (DMA) {
        // slices 0 .. D - 1 (the sweep has at least KS >= NSLOT > D slices)
#pragma unroll
        for (int j = 0; j < D; ++j)
            ring_fill<KPB, NW, NCH>(slots[j], B + (int64_t)tfirst * PN_BN * KPB + j * 128, loff,
                                    wave_u);
    } else {
        gload(0);
        lstore(sL0);
        __syncthreads();
    }
    // per-column FP8 scale exponents, read one S tile ahead
    auto col_scales = [&](int t, int (&e)[CB]) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
            e[cb] = PREC == P_FP8
                        ? 127 - pow2_exponent(info_s[(int64_t)t * PN_BN + cb * 32 + r32].qscale)
                        : 127;
    };
    int sb_next[CB];
    col_scales(tfirst, sb_next);
    for (int t = tfirst; t < t1;) {
        const int tn = next_tile(t);
        int sb[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) sb[cb] = sb_next[cb];
        if (tn < t1) col_scales(tn, sb_next);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            if constexpr (DMA) {
                // slice q has landed once at most the D - 1 later slices'
                // loads are in flight; the barrier then publishes every
                // wave's part and retires all reads of slice q - 1, whose
                // slot slice q + D takes.  The ring always runs D fills
                // ahead: past the end of the sweep the fills reload the last
                // tile (never read), which keeps every wait count static.
                wait_vmcnt_lgkm0<(D - 1) * NCH>();
                bare_barrier();
                const int t2 = MASK ? ((ks + D) / KS && tn < t1 ? tn : t)
                                    : min(t + (ks + D) / KS, t1 - 1);
                const int k2 = (ks + D) % KS;
                ring_fill<KPB, NW, NCH>(slots[(ks + D) % NS], B + (int64_t)t2 * PN_BN * KPB + k2 * 128,
                                        loff, wave_u);
                slice_mma<PREC, KS, RB, CB>(slots[ks % NS], ks, af, acc, sa, sb, h, r32);
            } else {
                const int q = (t - t0) * KS + ks;
                const bool more = q + 1 < nq;
                if (more) gload(q + 1);
                slice_mma<PREC, KS, RB, CB>((q & 1) ? sL1 : sL0, ks, af, acc, sa, sb, h, r32);
                if (more) lstore(((q + 1) & 1) ? sL1 : sL0);
                __syncthreads();
            }
        }

        ctx.t = t;
        ctx.edge = redge || (int64_t)(t + 1) * PN_BN > nS;
        EPI::template tile<RB, CB>(ep, esm, est, acc, ctx);
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[rb][cb][e] = 0.0f;
        t = tn;
    }
    // the fills past the end land before the workgroup's LDS is released
    if constexpr (DMA) wait_vmcnt_lgkm0<0>();
    EPI::finish(ep, esm, est, ctx);
}

template <int PREC, int KS, int RB, int CB, int NW, int OCC, int NSLOT, class EPI>
__global__ __launch_bounds__(64 * NW, OCC) void panel_kernel(
    const char* __restrict__ A, const char* __restrict__ B, const RowInfo* __restrict__ info_r,
    const RowInfo* __restrict__ info_s, int64_t nR, int64_t nS, int n_panels, int n_items,
    int tiles_per_chunk, int n_stiles, const unsigned long long* __restrict__ flags, int grid_x,
    typename EPI::Params ep) {
    constexpr int PN_BN = 32 * CB;
    constexpr int SLOT = PN_BN * 128;
    constexpr bool DMA = NSLOT > 0;
    constexpr int NS = DMA ? NSLOT : 2;
    __shared__ __attribute__((aligned(16))) char sL0[SLOT];
    __shared__ __attribute__((aligned(16))) char sL1[SLOT];
    __shared__ __attribute__((aligned(16))) char sL2[NS > 2 ? SLOT : 16];
    __shared__ __attribute__((aligned(16))) char sL3[NS > 3 ? SLOT : 16];
    __shared__ __attribute__((aligned(16))) char sL4[NS > 4 ? SLOT : 16];
    __shared__ __attribute__((aligned(16))) char sL5[NS > 5 ? SLOT : 16];
    __shared__ typename EPI::Smem esm;
    char* const slots[6] = {sL0, sL1, sL2, sL3, sL4, sL5};
    // OCC workgroups must fit the CU's 160 KB of LDS together
    constexpr size_t kLds = 2 * SLOT + (NS > 2 ? SLOT : 16) + (NS > 3 ? SLOT : 16) +
                            (NS > 4 ? SLOT : 16) + (NS > 5 ? SLOT : 16) + sizeof(typename EPI::Smem);
    static_assert(OCC * kLds <= 160 * 1024, "LDS of OCC workgroups exceeds the CU's 160 KB");

    // (hardware ids through the builtins: with the kernel's size the inliner
    // leaves library helpers as calls, which would put the ids in vector
    // registers and hide their uniformity)
    const int item =
        (int)(__builtin_amdgcn_workgroup_id_y() * grid_x + __builtin_amdgcn_workgroup_id_x());
    if (item >= n_items) return;
    if (flags[H_FLAGS] != 0) return;
    const int chunk = item / n_panels;
    const int panel = item - chunk * n_panels;
    const int t0 = chunk * tiles_per_chunk;
    const int t1 = min(t0 + tiles_per_chunk, n_stiles);
    if (t0 >= t1) return;

    panel_sweep<PREC, KS, RB, CB, NW, NSLOT, EPI>(slots, esm, A, B, info_r, info_s, nR, nS, panel,
                                                  t0, t1, ep);
}

// ---------------------------------------------------------------------------
// batched threshold joins on deep register panels (BF16, 8 / 9 / 10 / 12 K
// slices per row)
// ---------------------------------------------------------------------------
// One persistent launch for all jobs, as the tile form (batch.hip) but with
// panel work items: job j owns items [tile_base_j, tile_base_j + tiles_m_j *
// ceil(tiles_n_j / chunk_tiles_j)), tiles_m = 128-row R panels, tiles_n =
// 128-column S tiles; an item is one panel's sweep over chunk_tiles S tiles
// (panel index fastest, so the items running together share their S chunk).
// In prefilter mode the items come from the work list instead, each with the
// mask of the chunk's S tiles that survived the bounds; the sweep visits only
// those.  The K depth of each job selects the sweep; band entries carry the
// job.
constexpr int BP_SLOT = 128 * 128;

template <int KS, bool WL>
__device__ __forceinline__ void batch_panel_item(char* const (&slots)[6],
                                                 typename ThresholdEpiT<4, true, WL>::Smem& esm,
                                                 const BatchJob& J, int panel, int t0, int t1,
                                                 uint32_t mask, const ThresholdParams& ep) {
    constexpr int NSLOT = KS == 8 ? 4 : KS == 9 ? 3 : KS == 10 ? 5 : 6;
    panel_sweep<P_BF16, KS, 1, 4, 4, NSLOT, ThresholdEpiT<4, true, WL>, WL>(
        slots, esm, J.A, J.B, J.info_r, J.info_s, J.nR, J.nS, panel, t0, t1, ep, mask);
}

// WL: prefilter mode (masked work-list items, rows in the prefilter order);
// else every (panel, chunk) item in full.
template <bool WL>
__global__ __launch_bounds__(256, 1) void batch_panel(const BatchHead* __restrict__ head,
                                                      const BatchJob* __restrict__ jobs,
                                                      unsigned long long* __restrict__ bctr) {
    __shared__ __attribute__((aligned(16))) char sL0[BP_SLOT];
    __shared__ __attribute__((aligned(16))) char sL1[BP_SLOT];
    __shared__ __attribute__((aligned(16))) char sL2[BP_SLOT];
    __shared__ __attribute__((aligned(16))) char sL3[BP_SLOT];
    __shared__ __attribute__((aligned(16))) char sL4[BP_SLOT];
    __shared__ __attribute__((aligned(16))) char sL5[BP_SLOT];
    __shared__ typename ThresholdEpiT<4, true, WL>::Smem esm;
    __shared__ int64_t s_item;
    __shared__ int s_job, s_panel, s_t0;
    __shared__ uint32_t s_mask;
    char* const slots[6] = {sL0, sL1, sL2, sL3, sL4, sL5};
    const int64_t* work = head->work;
    const int64_t total = WL ? (int64_t)*head->n_work : head->n_tiles;
    const int n_jobs = head->n_jobs;
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    for (;;) {
        if (tid == 0) {
            const int64_t item = (int64_t)atomicAdd(bctr + B_ITEM, 1ull);
            int job = 0, panel = 0, t0 = 0;
            uint32_t mask = 0;
            if (item < total) {
                if constexpr (WL) {
                    const int64_t w = work[item];
                    job = (int)(w >> 48);
                    panel = (int)((w >> 24) & 0xFFFFFF);
                    t0 = (int)(w & 0xFFFFFF);
                    mask = head->work_mask[item];
                } else {
                    // last job whose first item is <= item
                    int lo = 0, hi = n_jobs - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (jobs[mid].tile_base <= item) lo = mid;
                        else hi = mid - 1;
                    }
                    job = lo;
                    const BatchJob& J = jobs[lo];
                    const int64_t local = item - J.tile_base;
                    panel = (int)(local % J.tiles_m);
                    t0 = (int)(local / J.tiles_m) * J.chunk_tiles;
                }
            }
            s_item = item;
            s_job = job;
            s_panel = panel;
            s_t0 = t0;
            s_mask = mask;
        }
        // (also: every wave is done with the previous item's ring slots)
        __syncthreads();
        const int64_t item = s_item;
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        const int panel = __builtin_amdgcn_readfirstlane(s_panel);
        const int t0 = __builtin_amdgcn_readfirstlane(s_t0);
        const uint32_t mask = WL ? __builtin_amdgcn_readfirstlane(s_mask) : 0u;
        __syncthreads();  // the shared slots are rewritten by the next iteration
        if (item >= total) break;
        const BatchJob& J = jobs[job];
        if (J.hdr[H_FLAGS] != 0) continue;  // bad input rows in this job
        const int t1 = min(t0 + J.chunk_tiles, J.tiles_n);
        ThresholdParams ep;
        ep.lo = J.lo;
        ep.hi = J.hi;
        ep.lohi = nullptr;
        ep.out = J.out;
        ep.capacity = J.capacity;
        ep.out_ctr = J.hdr + H_OUT;
        ep.band = head->band;
        ep.band_cap = head->band_cap;
        ep.band_ctr = bctr + B_BAND;
        ep.job = job;
        ep.perm_r = J.perm_r;
        ep.perm_s = J.perm_s;
        switch (J.Kp_bytes) {  // uniform
            case 8 * 128: batch_panel_item<8, WL>(slots, esm, J, panel, t0, t1, mask, ep); break;
            case 9 * 128: batch_panel_item<9, WL>(slots, esm, J, panel, t0, t1, mask, ep); break;
            case 10 * 128: batch_panel_item<10, WL>(slots, esm, J, panel, t0, t1, mask, ep); break;
            default: batch_panel_item<12, WL>(slots, esm, J, panel, t0, t1, mask, ep); break;
        }
    }
}

// Two workgroups per CU for a dense batch (tile 22): 32-column S tiles keep
// the R fragments of up to 12 K slices and the rest of a wave within 256
// registers, and six 4 KB ring slots plus the staging leave LDS for two
// workgroups, so that one workgroup's epilogue runs beside the other's
// matrix work.  Items are those of the one-workgroup form (one 128-row
// panel over 16 x 128 S columns), swept as 64 tiles of 32 columns.
constexpr int BP2_SLOT = 32 * 128;

template <int KS, bool WL>
__device__ __forceinline__ void batch_panel2_item(char* const (&slots)[6],
                                                  typename ThresholdEpiT<4, true, WL>::Smem& esm,
                                                  const BatchJob& J, int panel, int t0, int t1,
                                                  uint64_t mask, const ThresholdParams& ep) {
    constexpr int NSLOT = KS == 8 ? 4 : KS == 9 ? 3 : KS == 10 ? 5 : 6;
    panel_sweep<P_BF16, KS, 1, 1, 4, NSLOT, ThresholdEpiT<4, true, WL>, WL>(
        slots, esm, J.A, J.B, J.info_r, J.info_s, J.nR, J.nS, panel, t0, t1, ep, mask);
}

// WL: prefilter mode (work-list items; each kept 128-column tile of the
// item's mask becomes four kept 32-column tiles; rows in the prefilter order)
template <bool WL>
__global__ __launch_bounds__(256, 2) void batch_panel2(const BatchHead* __restrict__ head,
                                                       const BatchJob* __restrict__ jobs,
                                                       unsigned long long* __restrict__ bctr) {
    __shared__ __attribute__((aligned(16))) char sL0[BP2_SLOT];
    __shared__ __attribute__((aligned(16))) char sL1[BP2_SLOT];
    __shared__ __attribute__((aligned(16))) char sL2[BP2_SLOT];
    __shared__ __attribute__((aligned(16))) char sL3[BP2_SLOT];
    __shared__ __attribute__((aligned(16))) char sL4[BP2_SLOT];
    __shared__ __attribute__((aligned(16))) char sL5[BP2_SLOT];
    __shared__ typename ThresholdEpiT<4, true, WL>::Smem esm;
    __shared__ int64_t s_item;
    __shared__ int s_job, s_panel, s_t0;
    __shared__ uint64_t s_mask;
    char* const slots[6] = {sL0, sL1, sL2, sL3, sL4, sL5};
    constexpr int SUB = 128 / 32;  // 32-column tiles per 128-column tile
    const int64_t* work = head->work;
    const int64_t total = WL ? (int64_t)*head->n_work : head->n_tiles;
    const int n_jobs = head->n_jobs;
    const int tid = (int)__builtin_amdgcn_workitem_id_x();
    for (;;) {
        if (tid == 0) {
            const int64_t item = (int64_t)atomicAdd(bctr + B_ITEM, 1ull);
            int job = 0, panel = 0, t0 = 0;
            uint64_t mask = 0;
            if (item < total) {
                if constexpr (WL) {
                    const int64_t w = work[item];
                    job = (int)(w >> 48);
                    panel = (int)((w >> 24) & 0xFFFFFF);
                    t0 = (int)(w & 0xFFFFFF) * SUB;
                    const uint32_t m16 = head->work_mask[item];
                    static_assert(SUB == 4, "one 32-column tile per mask bit per quarter");
                    for (int b = 0; b < kPanelChunkTiles; ++b)
                        if ((m16 >> b) & 1u) mask |= 0xFull << (SUB * b);
                } else {
                    // last job whose first item is <= item
                    int lo = 0, hi = n_jobs - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (jobs[mid].tile_base <= item) lo = mid;
                        else hi = mid - 1;
                    }
                    job = lo;
                    const int64_t local = item - jobs[lo].tile_base;
                    panel = (int)(local % jobs[lo].tiles_m);
                    t0 = (int)(local / jobs[lo].tiles_m) * jobs[lo].chunk_tiles * SUB;
                }
            }
            s_item = item;
            s_job = job;
            s_panel = panel;
            s_t0 = t0;
            s_mask = mask;
        }
        // (also: every wave is done with the previous item's ring slots)
        __syncthreads();
        const int64_t item = s_item;
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        const int panel = __builtin_amdgcn_readfirstlane(s_panel);
        const int t0 = __builtin_amdgcn_readfirstlane(s_t0);
        uint64_t mask = 0;
        if constexpr (WL) {
            const uint64_t m = s_mask;
            mask = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(m >> 32))
                    << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)m);
        }
        __syncthreads();  // the shared slots are rewritten by the next iteration
        if (item >= total) break;
        const BatchJob& J = jobs[job];
        if (J.hdr[H_FLAGS] != 0) continue;  // bad input rows in this job
        const int t1 = min(t0 + J.chunk_tiles * SUB, (int)((J.nS + 31) / 32));
        ThresholdParams ep;
        ep.lo = J.lo;
        ep.hi = J.hi;
        ep.lohi = nullptr;
        ep.out = J.out;
        ep.capacity = J.capacity;
        ep.out_ctr = J.hdr + H_OUT;
        ep.band = head->band;
        ep.band_cap = head->band_cap;
        ep.band_ctr = bctr + B_BAND;
        ep.job = job;
        ep.perm_r = J.perm_r;
        ep.perm_s = J.perm_s;
        switch (J.Kp_bytes) {  // uniform
            case 8 * 128: batch_panel2_item<8, WL>(slots, esm, J, panel, t0, t1, mask, ep); break;
            case 9 * 128: batch_panel2_item<9, WL>(slots, esm, J, panel, t0, t1, mask, ep); break;
            case 10 * 128: batch_panel2_item<10, WL>(slots, esm, J, panel, t0, t1, mask, ep); break;
            default: batch_panel2_item<12, WL>(slots, esm, J, panel, t0, t1, mask, ep); break;
        }
    }
}

int batch_panel2_occupancy() {
    int n = 0, m = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_panel2<false>, 256, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, batch_panel2<true>, 256, 0) != hipSuccess)
        return 0;
    return n < m ? n : m;
}

hipError_t launch_batch_panel2(const BatchHead* head, const BatchJob* jobs,
                               unsigned long long* bctr, int grid, bool worklist, hipStream_t st) {
    if (worklist)
        hipLaunchKernelGGL(batch_panel2<true>, dim3((unsigned)grid), dim3(256), 0, st, head, jobs,
                           bctr);
    else
        hipLaunchKernelGGL(batch_panel2<false>, dim3((unsigned)grid), dim3(256), 0, st, head, jobs,
                           bctr);
    return hipGetLastError();
}

// K bytes per row the batch panel form takes
bool batch_panel_depth(int kpb) {
    return kpb == 8 * 128 || kpb == 9 * 128 || kpb == 10 * 128 || kpb == 12 * 128;
}

int batch_panel_occupancy() {
    int n = 0;
    int m = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_panel<false>, 256, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&m, batch_panel<true>, 256, 0) != hipSuccess)
        return 0;
    return n < m ? n : m;
}

hipError_t launch_batch_panel(const BatchHead* head, const BatchJob* jobs,
                              unsigned long long* bctr, int grid, bool worklist, hipStream_t st) {
    if (worklist)
        hipLaunchKernelGGL(batch_panel<true>, dim3((unsigned)grid), dim3(256), 0, st, head, jobs,
                           bctr);
    else
        hipLaunchKernelGGL(batch_panel<false>, dim3((unsigned)grid), dim3(256), 0, st, head, jobs,
                           bctr);
    return hipGetLastError();
}

// S chunks per panel: the threshold sweep is split so that there are enough
// workgroups to balance the 256 CUs (about 32 per CU); the top-k sweep must
// see all of S in one workgroup (one chunk).
template <int PREC, int KS, int RB, int CB, int NW, int OCC, int NSLOT, class EPI>
static hipError_t run_panel(const void* A, const void* B, const RowInfo* info_r,
                            const RowInfo* info_s, int64_t nR, int64_t nS, bool split_s,
                            const unsigned long long* hdr, const typename EPI::Params& ep,
                            hipStream_t st, PanelQuery* q = nullptr) {
    if (q) {  // the instantiation's designed and actual workgroups per CU; no launch
        q->designed = OCC;
        q->waves = NW;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &q->resident, panel_kernel<PREC, KS, RB, CB, NW, OCC, NSLOT, EPI>, 64 * NW, 0);
    }
    constexpr int PN_BN = 32 * CB;
    constexpr int PN_ROWS = 32 * RB * NW;
    const int64_t n_panels = (nR + PN_ROWS - 1) / PN_ROWS;
    const int64_t n_stiles = (nS + PN_BN - 1) / PN_BN;
    if (n_panels == 0 || n_stiles == 0) return hipSuccess;
    int64_t n_chunks = 1;
    if (split_s) {
        n_chunks = (8192 + n_panels - 1) / n_panels;
        if (n_chunks > n_stiles) n_chunks = n_stiles;
    }
    const int64_t tpc = (n_stiles + n_chunks - 1) / n_chunks;
    n_chunks = (n_stiles + tpc - 1) / tpc;
    const int64_t items = n_panels * n_chunks;
    if (items > 0x7fffffffLL) return hipErrorInvalidValue;
    const int64_t gx = items < 65536 ? items : 65536;
    const int64_t gy = (items + gx - 1) / gx;
    hipLaunchKernelGGL((panel_kernel<PREC, KS, RB, CB, NW, OCC, NSLOT, EPI>),
                       dim3((unsigned)gx, (unsigned)gy), dim3(64 * NW), 0, st, (const char*)A,
                       (const char*)B, info_r, info_s, nR, nS, (int)n_panels, (int)items, (int)tpc,
                       (int)n_stiles, hdr, (int)gx, ep);
    return hipGetLastError();
}

// Kp * element size must be KS * 128 bytes with KS in 1..6 (BF16 one
// workgroup per CU: also 8, 9, 10, 12).
//  * two_waves: one 32-row block per wave, two workgroups of four waves per
//    CU (the epilogue of one overlaps the MFMAs of the other); BF16 K slices
//    on a direct-load ring from three slices on (64-column S tiles where the
//    ring or the R fragments would not fit otherwise);
//  * otherwise one workgroup per CU: for KS 3 .. 6 eight waves with one row
//    block each, four 32-column blocks per tile and a direct-load ring of one
//    slot per K slice (three for KS = 3); else four waves with two row blocks
//    each.
template <int PREC, template <int> class EPI>
static hipError_t dispatch_panel(int ks, int form, const void* A, const void* B,
                                 const RowInfo* ir, const RowInfo* is, int64_t nR, int64_t nS,
                                 bool split_s, const unsigned long long* hdr,
                                 const typename EPI<4>::Params& ep, hipStream_t st,
                                 PanelQuery* q = nullptr) {
#define EJ_RUN(KS_, RB_, CB_, NW_, OCC_, NSLOT_)                                          \
    return run_panel<PREC, KS_, RB_, CB_, NW_, OCC_, NSLOT_, EPI<NW_>>(A, B, ir, is, nR, nS, \
                                                                       split_s, hdr, ep, st, q)
    if (form == 2) {
        // two 32-row blocks per wave, one wave per SIMD: every B fragment read
        // from LDS feeds two MFMAs (half the LDS traffic per flop of the
        // one-block forms); R fragments and accumulators take up to 352 of
        // the 512 registers a lone wave has
        if constexpr (PREC != P_FP32) {
            switch (ks) {
                case 3: EJ_RUN(3, 2, 4, 4, 1, 3);
                case 4: EJ_RUN(4, 2, 4, 4, 1, 4);
                case 5: EJ_RUN(5, 2, 4, 4, 1, 5);
                case 6: EJ_RUN(6, 2, 4, 4, 1, 6);
            }
        }
        return hipErrorInvalidValue;
    }
    const bool two_waves = form == 1;
    if (two_waves) {
        if constexpr (PREC == P_FP32) {
            // two workgroups per CU, each with its own ring, so that one
            // workgroup's epilogue runs beside the other's matrix work; deeper
            // rows take 64- (32-) column S tiles to stay within 256 registers
            switch (ks) {
                case 1: EJ_RUN(1, 1, 4, 4, 2, 0);
                case 2: EJ_RUN(2, 1, 4, 4, 2, 0);
                case 3: EJ_RUN(3, 1, 4, 4, 2, 3);
                case 4: EJ_RUN(4, 1, 4, 4, 2, 2);
                case 5: EJ_RUN(5, 1, 2, 4, 2, 5);
                case 6: EJ_RUN(6, 1, 2, 4, 2, 3);
                case 8: EJ_RUN(8, 1, 2, 4, 2, 4);
                case 9: EJ_RUN(9, 1, 2, 4, 2, 3);
                case 10: EJ_RUN(10, 1, 2, 4, 2, 5);
                case 12: EJ_RUN(12, 1, 1, 4, 2, 6);
            }
        } else if constexpr (PREC == P_BF16) {
            switch (ks) {
                case 1: EJ_RUN(1, 1, 4, 4, 2, 0);
                case 2: EJ_RUN(2, 1, 4, 4, 2, 0);
                case 3: EJ_RUN(3, 1, 4, 4, 2, 3);
                case 4: EJ_RUN(4, 1, 4, 4, 2, 2);
                case 5: EJ_RUN(5, 1, 2, 4, 2, 5);
                case 6: EJ_RUN(6, 1, 4, 4, 2, 3);
                // deep rows: 64-column S tiles keep a wave within 256
                // registers; at 12 slices 32-column tiles (with a few spills
                // outside the matrix loop: 56.5 ms against 59.1 ms for the
                // one-workgroup panel on a 200k x 200k 768-d join)
                case 8: EJ_RUN(8, 1, 2, 4, 2, 4);
                case 9: EJ_RUN(9, 1, 2, 4, 2, 3);
                case 10: EJ_RUN(10, 1, 2, 4, 2, 5);
                case 12: EJ_RUN(12, 1, 1, 4, 2, 6);
            }
        } else {
            // FP8 fragments are twice as wide: one S block per tile keeps the
            // deep panels within the register file at two workgroups per CU
            switch (ks) {
                case 1: EJ_RUN(1, 1, 4, 4, 2, 0);
                case 2: EJ_RUN(2, 1, 2, 4, 2, 0);
                case 3: EJ_RUN(3, 1, 1, 4, 2, 3);
                case 4: EJ_RUN(4, 1, 1, 4, 2, 0);
                case 5: EJ_RUN(5, 1, 1, 4, 2, 0);
                case 6: EJ_RUN(6, 1, 1, 4, 2, 3);
            }
        }
        return hipErrorInvalidValue;
    }
    if constexpr (PREC == P_BF16) {
        switch (ks) {
            case 1: EJ_RUN(1, 2, 4, 4, 1, 0);
            case 2: EJ_RUN(2, 2, 4, 4, 1, 0);
            case 3: EJ_RUN(3, 1, 4, 8, 1, 3);
            case 4: EJ_RUN(4, 1, 4, 8, 1, 4);
            case 5: EJ_RUN(5, 1, 4, 8, 1, 5);
            case 6: EJ_RUN(6, 1, 4, 8, 1, 6);
            // deeper rows: the resident fragments of one 32-row block fill
            // most of a 512-register wave, so four waves (one per SIMD)
            case 8: EJ_RUN(8, 1, 4, 4, 1, 4);
            case 9: EJ_RUN(9, 1, 4, 4, 1, 3);
            case 10: EJ_RUN(10, 1, 4, 4, 1, 5);
            case 12: EJ_RUN(12, 1, 4, 4, 1, 6);
        }
    } else if constexpr (PREC == P_FP32) {
        // FP32 fragments take the same registers per K slice as BF16 (16 per
        // 32-row block), with four times the matrix-core steps per slice
        switch (ks) {
            case 1: EJ_RUN(1, 2, 4, 4, 1, 0);
            case 2: EJ_RUN(2, 2, 4, 4, 1, 0);
            case 3: EJ_RUN(3, 1, 4, 8, 1, 3);
            case 4: EJ_RUN(4, 1, 4, 8, 1, 4);
            case 5: EJ_RUN(5, 1, 4, 8, 1, 5);
            case 6: EJ_RUN(6, 1, 4, 8, 1, 6);
            case 8: EJ_RUN(8, 1, 4, 4, 1, 4);
            case 9: EJ_RUN(9, 1, 4, 4, 1, 3);
            case 10: EJ_RUN(10, 1, 4, 4, 1, 5);
            case 12: EJ_RUN(12, 1, 4, 4, 1, 6);
        }
    } else {
        // FP8 fragments are twice as wide per MFMA
        switch (ks) {
            case 1: EJ_RUN(1, 2, 4, 4, 1, 0);
            case 2: EJ_RUN(2, 2, 4, 4, 1, 0);
            case 3: EJ_RUN(3, 1, 4, 8, 1, 3);
            case 4: EJ_RUN(4, 1, 4, 8, 1, 4);
            case 5: EJ_RUN(5, 1, 4, 8, 1, 5);
            case 6: EJ_RUN(6, 1, 4, 8, 1, 6);
        }
    }
#undef EJ_RUN
    return hipErrorInvalidValue;
}

static int row_bytes(int prec, int Kp) { return Kp * (prec == P_FP32 ? 4 : prec == P_BF16 ? 2 : 1); }
static int slices(int prec, int Kp) { return row_bytes(prec, Kp) / 128; }

hipError_t launch_threshold_panel(int prec, int form, const ThresholdArgs& a,
                                  hipStream_t st) {
    const int kpb = row_bytes(prec, a.Kp);
    if (kpb % 128 != 0) return hipErrorInvalidValue;
    ThresholdParams ep;
    ep.lo = a.lo;
    ep.hi = a.hi;
    ep.lohi = a.lohi;
    ep.out = a.out;
    ep.capacity = a.capacity;
    ep.out_ctr = a.hdr + H_OUT;
    ep.band = a.band;
    ep.band_cap = a.band_cap;
    ep.band_ctr = a.hdr + H_BAND;
    ep.job = 0;
    ep.perm_r = nullptr;
    ep.perm_s = nullptr;
    const int ks = slices(prec, a.Kp);
    if (prec == P_BF16)
        return dispatch_panel<P_BF16, ThresholdEpi>(ks, form, a.A, a.B, a.info_r, a.info_s,
                                                    a.nR, a.nS, true, a.hdr, ep, st);
    if (prec == P_FP8)
        return dispatch_panel<P_FP8, ThresholdEpi>(ks, form, a.A, a.B, a.info_r, a.info_s,
                                                   a.nR, a.nS, true, a.hdr, ep, st);
    if (prec == P_FP32)
        return dispatch_panel<P_FP32, ThresholdEpi>(ks, form, a.A, a.B, a.info_r, a.info_s,
                                                    a.nR, a.nS, true, a.hdr, ep, st);
    return hipErrorInvalidValue;
}

// Row depths (bytes of K) that the top-k candidate sweep runs on register
// panels: up to six K slices in every format; BF16 and FP32 also eight,
// nine, ten or twelve.
hipError_t panel_query(int prec, int form, int Kp, PanelQuery* q) {
    const int kpb = row_bytes(prec, Kp);
    if (kpb % 128 != 0 || !q) return hipErrorInvalidValue;
    const int ks = slices(prec, Kp);
    ThresholdParams ep = {};
    if (prec == P_BF16)
        return dispatch_panel<P_BF16, ThresholdEpi>(ks, form, nullptr, nullptr, nullptr, nullptr,
                                                    0, 0, true, nullptr, ep, nullptr, q);
    if (prec == P_FP8)
        return dispatch_panel<P_FP8, ThresholdEpi>(ks, form, nullptr, nullptr, nullptr, nullptr,
                                                   0, 0, true, nullptr, ep, nullptr, q);
    if (prec == P_FP32)
        return dispatch_panel<P_FP32, ThresholdEpi>(ks, form, nullptr, nullptr, nullptr, nullptr,
                                                    0, 0, true, nullptr, ep, nullptr, q);
    return hipErrorInvalidValue;
}

bool topk_panel_depth(int prec, int kpb) {
    if (kpb % 128 != 0 || kpb <= 0) return false;
    const int ks = kpb / 128;
    if (ks <= 6) return true;
    return prec != P_FP8 && (ks == 8 || ks == 9 || ks == 10 || ks == 12);
}

// Top-k candidate sweep.  Every workgroup sweeps all of S for its rows.  The
// counter table holds 64 rows per wave, which covers both layouts.
hipError_t launch_topk_candidates(int prec, const CandArgs& a, hipStream_t st) {
    const int kpb = row_bytes(prec, a.Kp);
    if (!topk_panel_depth(prec, kpb)) return hipErrorInvalidValue;
    CandParams ep;
    ep.hdr = a.hdr;
    ep.cnt = a.cnt;
    ep.cand = a.cand;
    ep.Kc = a.Kc;
    const int ks = slices(prec, a.Kp);
#define EJ_RUN(P_, KS_, RB_, CB_, NW_, OCC_, NSLOT_)                                           \
    return run_panel<P_, KS_, RB_, CB_, NW_, OCC_, NSLOT_, CandEpi<NW_>>(                       \
        a.A, a.B, a.info_r, a.info_s, a.nR, a.nS, false, a.hdr, ep, st)
    // K of three slices or more: eight waves (one row block each), 128-column
    // S tiles and a direct-load ring of one slot per slice (FP8 at 768-d fits
    // 255 registers with 128-column tiles: 235 against 247 ms on the 2M x 200k
    // top-10 sweep with 64-column ones)
    if (prec == P_BF16) {
        switch (ks) {
            case 3: EJ_RUN(P_BF16, 3, 1, 4, 8, 1, 3);
            case 4: EJ_RUN(P_BF16, 4, 1, 4, 8, 1, 4);
            case 5: EJ_RUN(P_BF16, 5, 1, 4, 8, 1, 5);
            case 6: EJ_RUN(P_BF16, 6, 1, 4, 8, 1, 6);
        }
        return dispatch_panel<P_BF16, CandEpi>(ks, 1, a.A, a.B, a.info_r, a.info_s, a.nR,
                                               a.nS, false, a.hdr, ep, st);
    }
    if (prec == P_FP8) {
        switch (ks) {
            case 3: EJ_RUN(P_FP8, 3, 1, 4, 8, 1, 3);
            case 4: EJ_RUN(P_FP8, 4, 1, 4, 8, 1, 4);
            case 5: EJ_RUN(P_FP8, 5, 1, 4, 8, 1, 5);
            case 6: EJ_RUN(P_FP8, 6, 1, 4, 8, 1, 6);
        }
        return dispatch_panel<P_FP8, CandEpi>(ks, 1, a.A, a.B, a.info_r, a.info_s, a.nR,
                                              a.nS, false, a.hdr, ep, st);
    }
    if (prec == P_FP32)  // two workgroups per CU (the FP32 threshold default)
        return dispatch_panel<P_FP32, CandEpi>(ks, 1, a.A, a.B, a.info_r, a.info_s, a.nR,
                                               a.nS, false, a.hdr, ep, st);
#undef EJ_RUN
    return hipErrorInvalidValue;
}

}  // namespace ej
