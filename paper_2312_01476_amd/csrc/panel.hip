// panel.hip -- register-resident R panels for the narrow-format contraction.
//
// The tensor join's cache argument (Section IV.C: a block of vectors stays in
// cache and is reused across many products) is taken here to the register
// file.  A workgroup owns a panel of 256 R rows (64 per wave); each wave loads
// its rows' BF16 or FP8 MFMA operand fragments into VGPRs once and keeps them
// while the workgroup sweeps a range of S tiles (128 columns each).  S slices
// (128 bytes of K per row) stream through a double-buffered LDS ring shared by
// the four waves, so per MFMA only the S operand is read from LDS and only S
// traffic reaches L2.  With K short (a few hundred), this removes the
// per-output-tile prologue that a classic tile kernel pays for every block of
// D (Section V.B's mini-batch slowdown, at tile scale).
//
// Epilogue (single pass): each accumulator is compared with the band edges;
// the rare hits are appended to a per-wave staging list in LDS (ballot +
// mbcnt, no atomics) and the list is flushed to the global output with one
// atomicAdd per flush, i.e. per few hundred pairs.
#include "common.hpp"
#include "launch.hpp"
#include "mma.hpp"

namespace ej {

constexpr int PN_OUTCAP = 512;  // staged certain pairs per wave
constexpr int PN_BANDCAP = 512; // staged band pairs per wave

// Append the staged entries of one wave to a global list: one atomicAdd on
// the list counter, then a coalesced copy.  Entries past `cap` are dropped
// (the counter still counts them, so the caller learns the true size).
template <typename T>
__device__ __forceinline__ void flush_stage(T* stage, int& n, T* __restrict__ dst, int64_t cap,
                                            unsigned long long* ctr, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(ctr, (unsigned long long)n);
    const uint32_t blo = __shfl((uint32_t)base, 0, 64);
    const uint32_t bhi = __shfl((uint32_t)(base >> 32), 0, 64);
    const unsigned long long b = ((unsigned long long)bhi << 32) | blo;
    for (int e = lane; e < n; e += 64)
        if ((int64_t)(b + e) < cap) dst[b + e] = stage[e];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    n = 0;
}

// RB 32-row blocks per wave (4 waves), CB 32-column blocks per S tile, KS
// 128-byte K slices per row.
template <int PREC, int KS, int RB, int CB, int OCC>
__global__ __launch_bounds__(256, OCC) void threshold_panel(
    const char* __restrict__ A, const char* __restrict__ B, const RowInfo* __restrict__ info_r,
    const RowInfo* __restrict__ info_s, int64_t nR, int64_t nS, int n_panels, int n_items,
    int tiles_per_chunk, int n_stiles, float lo, float hi, Pair* __restrict__ out,
    int64_t capacity, int2* __restrict__ band, int64_t band_cap,
    unsigned long long* __restrict__ hdr) {
    typedef Mma<PREC> M;
    constexpr int G = M::GROUPS;
    constexpr int NF = KS * G;       // A fragments per 32-row block
    constexpr int KPB = KS * 128;    // bytes per operand row
    constexpr int PN_BN = 32 * CB;
    constexpr int PN_ROWS = 128 * RB;
    constexpr int NCH = PN_BN * 8 / 256;  // 16-byte chunks per thread per S slice

    __shared__ __attribute__((aligned(16))) char sB[2][PN_BN * 128];
    __shared__ Pair sOut[4][PN_OUTCAP];
    __shared__ int2 sBand[4][PN_BANDCAP];

    const int item = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    if (item >= n_items) return;
    if (hdr[H_FLAGS] != 0) return;
    const int chunk = item / n_panels;
    const int panel = item - chunk * n_panels;
    const int t0 = chunk * tiles_per_chunk;
    const int t1 = min(t0 + tiles_per_chunk, n_stiles);
    if (t0 >= t1) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int h = lane >> 5, r32 = lane & 31;
    const int r0 = panel * PN_ROWS + wave * 32 * RB;  // first R row of this wave

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
        sa[rb] = PREC == P_FP8 ? 127 - ilogbf(info_r[r0 + rb * 32 + r32].qscale) : 127;

    v16f acc[RB][CB];
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < CB; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    const int nq = (t1 - t0) * KS;
    v4i rbuf[NCH];
    auto gload = [&](int q) {
        const int t = t0 + q / KS, ks = q - (q / KS) * KS;
        const char* base = B + (int64_t)t * PN_BN * KPB + ks * 128;
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int qq = tid + i * 256;
            rbuf[i] = *(const v4i*)(base + (int64_t)(qq >> 3) * KPB + (qq & 7) * 16);
        }
    };
    auto lstore = [&](int slot) {
#pragma unroll
        for (int i = 0; i < NCH; ++i) {
            const int qq = tid + i * 256;
            *(v4i*)(&sB[slot][lds_off(qq >> 3, qq & 7)]) = rbuf[i];
        }
    };

    int n_out = 0, n_band = 0;  // staged entries of this wave (wave-uniform)
    const bool redge = (int64_t)panel * PN_ROWS + PN_ROWS > nR;

    gload(0);
    lstore(0);
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        int sb[CB];
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
            sb[cb] = PREC == P_FP8
                         ? 127 - ilogbf(info_s[(int64_t)t * PN_BN + cb * 32 + r32].qscale)
                         : 127;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int q = (t - t0) * KS + ks;
            const bool more = q + 1 < nq;
            if (more) gload(q + 1);
            const char* sl = sB[q & 1];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                typename M::Frag fb[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const int row = cb * 32 + r32;
#pragma unroll
                    for (int c = 0; c < M::CPL; ++c) {
                        v4i v = *(const v4i*)(sl + lds_off(row, M::chunk(g, h, c)));
#pragma unroll
                        for (int e = 0; e < 4; ++e) fb[cb][c * 4 + e] = v[e];
                    }
                }
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        M::mma(af[rb][ks * G + g], fb[cb], acc[rb][cb], sa[rb], sb[cb]);
            }
            if (more) lstore((q + 1) & 1);
            __syncthreads();
        }

        // ---- epilogue of S tile t ----
        // Phase 1 (no branches): one wave mask per group of four
        // accumulators (four rows of one column per lane), from a compare of
        // their maximum.  Phase 2: only groups with a possible hit are split
        // per register; interior tiles skip the bounds test.
        const bool edge = redge || (int64_t)(t + 1) * PN_BN > nS;
        const int gi0 = r0 + 4 * h;               // + rb*32 + 8*(e/4) + e%4
        const int gj0 = t * PN_BN + r32;          // + cb*32
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
                    gmask[rb][cb][q4] = __ballot(m4 >= lo);
                }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int q4 = 0; q4 < 4; ++q4) {
                    const int e4 = 4 * q4;
                    if (gmask[rb][cb][q4]) {
                        // room for the at most 4 x 64 hits of this group
                        if (n_out > PN_OUTCAP - 256)
                            flush_stage(sOut[wave], n_out, out, capacity, hdr + H_OUT, lane);
                        if (n_band > PN_BANDCAP - 256)
                            flush_stage(sBand[wave], n_band, band, band_cap, hdr + H_BAND, lane);
                        const int gj = gj0 + cb * 32;
                        const bool vj = !edge || gj < nS;
                        uint64_t ml[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int gi = gi0 + rb * 32 + 8 * q4 + k;
                            const bool v = vj && (!edge || gi < nR);
                            ml[k] = __ballot(v && acc[rb][cb][e4 + k] >= lo);
                        }
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if (!ml[k]) continue;
                            const float a = acc[rb][cb][e4 + k];
                            const int gi = gi0 + rb * 32 + 8 * q4 + k;
                            const bool in_lo = (ml[k] >> lane) & 1ull;
                            const bool in_hi = in_lo && a >= hi;
                            const uint64_t mhi = __ballot(in_hi);
                            const uint64_t mb = ml[k] & ~mhi;
                            if (in_hi) {
                                Pair pr;
                                pr.r = gi;
                                pr.s = gj;
                                pr.score = a;
                                sOut[wave][n_out + lanes_below(mhi)] = pr;
                            } else if (in_lo) {
                                sBand[wave][n_band + lanes_below(mb)] = make_int2(gi, gj);
                            }
                            n_out += __popcll(mhi);
                            n_band += __popcll(mb);
                        }
                    }
                }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
#pragma unroll
                for (int e = 0; e < 16; ++e) acc[rb][cb][e] = 0.0f;
    }
    if (n_out) flush_stage(sOut[wave], n_out, out, capacity, hdr + H_OUT, lane);
    if (n_band) flush_stage(sBand[wave], n_band, band, band_cap, hdr + H_BAND, lane);
}

template <int PREC, int KS, int RB, int CB, int OCC = 1>
static hipError_t run_panel(const ThresholdArgs& a, hipStream_t st) {
    constexpr int PN_BN = 32 * CB;
    constexpr int PN_ROWS = 128 * RB;
    const int64_t n_panels = (a.nR + PN_ROWS - 1) / PN_ROWS;
    const int64_t n_stiles = (a.nS + PN_BN - 1) / PN_BN;
    if (n_panels == 0 || n_stiles == 0) return hipSuccess;
    // split the S sweep so that there are enough workgroups to balance the
    // 256 CUs (about 32 per CU), keeping whole S tiles per chunk
    int64_t n_chunks = (8192 + n_panels - 1) / n_panels;
    if (n_chunks > n_stiles) n_chunks = n_stiles;
    const int64_t tpc = (n_stiles + n_chunks - 1) / n_chunks;
    n_chunks = (n_stiles + tpc - 1) / tpc;
    const int64_t items = n_panels * n_chunks;
    if (items > 0x7fffffffLL) return hipErrorInvalidValue;
    const int64_t gx = items < 65536 ? items : 65536;
    const int64_t gy = (items + gx - 1) / gx;
    hipLaunchKernelGGL((threshold_panel<PREC, KS, RB, CB, OCC>), dim3((unsigned)gx, (unsigned)gy), dim3(256),
                       0, st, (const char*)a.A, (const char*)a.B, a.info_r, a.info_s, a.nR, a.nS,
                       (int)n_panels, (int)items, (int)tpc, (int)n_stiles, a.lo, a.hi, a.out,
                       a.capacity, a.band, a.band_cap, a.hdr);
    return hipGetLastError();
}

// Kp * element size must be KS * 128 bytes with KS in 1..6.  Two 32-row
// blocks per wave while the resident fragments fit the register file (up to
// 512 bytes of K per row), one beyond.
template <int PREC>
static hipError_t dispatch_panel(int ks, bool two_waves, const ThresholdArgs& a, hipStream_t st) {
    if (two_waves) {
        // one 32-row block per wave, 128-column S tiles, two workgroups per CU
        switch (ks) {
            case 1: return run_panel<PREC, 1, 1, 4, 2>(a, st);
            case 2: return run_panel<PREC, 2, 1, 4, 2>(a, st);
            case 3: return run_panel<PREC, 3, 1, 4, 2>(a, st);
            case 4: return run_panel<PREC, 4, 1, 4, 2>(a, st);
            case 5: return run_panel<PREC, 5, 1, 4, 2>(a, st);
            case 6: return run_panel<PREC, 6, 1, 4, 2>(a, st);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (PREC == P_BF16) {
        switch (ks) {
            case 1: return run_panel<PREC, 1, 2, 4>(a, st);
            case 2: return run_panel<PREC, 2, 2, 4>(a, st);
            case 3: return run_panel<PREC, 3, 2, 4>(a, st);
            case 4: return run_panel<PREC, 4, 2, 4>(a, st);
            case 5: return run_panel<PREC, 5, 1, 8>(a, st);
            case 6: return run_panel<PREC, 6, 1, 8>(a, st);
        }
    } else {
        // FP8 fragments are twice as wide per MFMA: one row block beyond 256 B
        switch (ks) {
            case 1: return run_panel<PREC, 1, 2, 4>(a, st);
            case 2: return run_panel<PREC, 2, 2, 4>(a, st);
            case 3: return run_panel<PREC, 3, 1, 4>(a, st);
            case 4: return run_panel<PREC, 4, 1, 4>(a, st);
            case 5: return run_panel<PREC, 5, 1, 2>(a, st);
            case 6: return run_panel<PREC, 6, 1, 2>(a, st);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_threshold_panel(int prec, bool two_waves, const ThresholdArgs& a,
                                  hipStream_t st) {
    const int kpb = a.Kp * (prec == P_BF16 ? 2 : 1);
    if (kpb % 128 != 0) return hipErrorInvalidValue;
    if (prec == P_BF16) return dispatch_panel<P_BF16>(kpb / 128, two_waves, a, st);
    if (prec == P_FP8) return dispatch_panel<P_FP8>(kpb / 128, two_waves, a, st);
    return hipErrorInvalidValue;
}

}  // namespace ej
