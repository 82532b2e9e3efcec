// epi_stage.hpp -- single-pass threshold epilogue with per-wave staging in
// LDS, for tiles whose accumulators fill the register file.
//
// Screening goes four accumulators at a time: one wave ballot of the
// maximum of a group of four registers tells whether any of them can reach
// the band; only groups with a possible hit are split per register.  Hits are
// appended to per-wave LDS lists (certain pairs and band pairs) and each
// list is flushed to its global list with one atomicAdd when it runs full
// and once at the end, so the global counters see one atomic per few hundred
// pairs instead of one per tile and wave.
#pragma once

#include "common.hpp"

namespace ej {

constexpr int ST_OUT = 512;   // staged certain pairs per wave
constexpr int ST_BAND = 512;  // staged band pairs per wave

template <bool TAG>
struct BandEntryT {
    typedef int2 type;
};
template <>
struct BandEntryT<true> {
    typedef int4 type;
};

// Append a wave's staged entries to a global list (one atomicAdd on its
// counter, then a coalesced copy); entries past `cap` are dropped but
// counted, so the caller learns the true size.
// (kept out of line: it runs rarely, and a small caller body lets the
// compiler unroll the epilogue completely, keeping the accumulators in
// registers)
template <typename T>
__device__ __noinline__ int stage_flush(T* stage, int n, T* __restrict__ dst, int64_t cap,
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
    return 0;
}

// Threshold epilogue of one wave's FM x FN blocks of 32 x 32 accumulators.
// Element e of block (i, j) of a lane is row i0 + 32 i + 8 (e/4) + 4 h + e%4
// and column j0 + 32 j + r32 (h = lane / 32, r32 = lane % 32).  st_out and
// st_band are this wave's LDS staging lists (ST_OUT and ST_BAND entries).
template <int FM, int FN, bool TAG>
__device__ __forceinline__ void stage_epilogue(
    v16f (&acc)[FM][FN], int64_t i0, int64_t j0, bool edge, int64_t nR, int64_t nS, float lo,
    float hi, Pair* __restrict__ out, int64_t capacity, unsigned long long* __restrict__ out_ctr,
    void* __restrict__ band, int64_t band_cap, unsigned long long* __restrict__ band_ctr,
    int job, const int32_t* __restrict__ perm_r, const int32_t* __restrict__ perm_s,
    Pair* st_out, typename BandEntryT<TAG>::type* st_band) {
    typedef typename BandEntryT<TAG>::type BE;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5, r32 = lane & 31;
    int n_out = 0, n_band = 0;  // wave-uniform
#pragma clang loop unroll(full)
    for (int i = 0; i < FM; ++i)
#pragma clang loop unroll(full)
        for (int j = 0; j < FN; ++j)
#pragma clang loop unroll(full)
            for (int q4 = 0; q4 < 4; ++q4) {
                const int e4 = 4 * q4;
                const float m4 =
                    __builtin_fmaxf(__builtin_fmaxf(acc[i][j][e4], acc[i][j][e4 + 1]),
                                    __builtin_fmaxf(acc[i][j][e4 + 2], acc[i][j][e4 + 3]));
                if (!__ballot(m4 >= lo)) continue;
                // room for the at most 4 x 64 hits of this group
                if (n_out > ST_OUT - 256)
                    n_out = stage_flush(st_out, n_out, out, capacity, out_ctr, lane);
                if (n_band > ST_BAND - 256)
                    n_band = stage_flush(st_band, n_band, (BE*)band, band_cap, band_ctr, lane);
                const int64_t gj = j0 + j * 32 + r32;
                const bool vj = !edge || gj < nS;
#pragma clang loop unroll(full)
                for (int k = 0; k < 4; ++k) {
                    const float a = acc[i][j][e4 + k];
                    const int64_t gi = i0 + i * 32 + 8 * q4 + 4 * h + k;
                    const bool in_lo = vj && (!edge || gi < nR) && a >= lo;
                    const uint64_t mlo = __ballot(in_lo);
                    if (!mlo) continue;
                    const bool in_hi = in_lo && a >= hi;
                    const uint64_t mhi = __ballot(in_hi);
                    const uint64_t mb = mlo & ~mhi;
                    int32_t ri = (int32_t)gi, si = (int32_t)gj;
                    if (in_lo && perm_r) {
                        ri = perm_r[gi];
                        si = perm_s[gj];
                    }
                    if (in_hi) {
                        Pair pr;
                        pr.r = ri;
                        pr.s = si;
                        pr.score = a;
                        st_out[n_out + lanes_below(mhi)] = pr;
                    } else if (in_lo) {
                        BE be;
                        if constexpr (TAG)
                            be = make_int4(ri, si, job, 0);
                        else
                            be = make_int2(ri, si);
                        st_band[n_band + lanes_below(mb)] = be;
                    }
                    n_out += __popcll(mhi);
                    n_band += __popcll(mb);
                }
            }
    if (n_out) stage_flush(st_out, n_out, out, capacity, out_ctr, lane);
    if (n_band) stage_flush(st_band, n_band, (BE*)band, band_cap, band_ctr, lane);
}

}  // namespace ej
