// nlj.hip -- the nested-loop join as a GPU comparator for the tensor join.
//
// Section V.A of the paper contrasts the tensor formulation with a
// data-parallel nested-loop join: every pair's similarity is computed on its
// own, vectorised over the embedding dimension, with no blocking of the
// relations.  Here one wavefront computes one pair at a time: its 64 lanes
// split the dimension, the R row stays in registers while the wave streams
// the S rows of its chunk (each read with coalesced loads and reduced across
// the wave), and there is no tiling, no LDS and no matrix-core work.  The
// pairs go through the same rigorous band and FP64 rescore as the tensor
// join, so the result set is the same exact one; only the cost differs.
#include "common.hpp"
#include "launch.hpp"

namespace ej {

constexpr int kNljMaxNV = 16;   // FP32 values per lane: rows of up to 1024 elements
constexpr int kNljChunk = 1024;  // S rows per work item (about 1.3 MB at 320 floats)

__global__ __launch_bounds__(256) void nlj_threshold(const float* __restrict__ A,
                                                     const float* __restrict__ B, int Kp,
                                                     int64_t nR, int64_t nS, float lo, float hi,
                                                     Pair* __restrict__ out, int64_t capacity,
                                                     int2* __restrict__ band, int64_t band_cap,
                                                     unsigned long long* __restrict__ hdr) {
    if (hdr[H_FLAGS] != 0) return;
    const int lane = threadIdx.x & 63;
    const int nv = (Kp + 63) / 64;
    const int64_t nch = (nS + kNljChunk - 1) / kNljChunk;
    const int64_t items = nR * nch;
    // item -> (R row fastest, S chunk): the waves running together share a chunk
    for (int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); item < items;
         item += (int64_t)gridDim.x * 4) {
        const int64_t i = item % nR;
        const int64_t j0 = (item / nR) * kNljChunk;
        const int64_t j1 = min(nS, j0 + kNljChunk);
        float r[kNljMaxNV];
#pragma unroll
        for (int v = 0; v < kNljMaxNV; ++v) {
            const int k = lane + 64 * v;
            r[v] = (v < nv && k < Kp) ? A[i * Kp + k] : 0.0f;
        }
        for (int64_t jb = j0; jb < j1; jb += 64) {
            const int n = (int)min((int64_t)64, j1 - jb);
            float mine = 0.0f;  // lane l ends with the score of pair (i, jb + l)
            for (int jj = 0; jj < n; ++jj) {
                const float* s = B + (jb + jj) * Kp;
                float p = 0.0f;
#pragma unroll
                for (int v = 0; v < kNljMaxNV; ++v) {
                    const int k = lane + 64 * v;
                    if (v < nv && k < Kp) p = fmaf(r[v], s[k], p);
                }
                p = wave_sum(p);
                if (lane == jj) mine = p;
            }
            const bool in_lo = lane < n && mine >= lo;
            const bool in_hi = in_lo && mine >= hi;
            const uint64_t mh = __ballot(in_hi);
            const uint64_t mb = __ballot(in_lo && !in_hi);
            if (mh) {
                unsigned long long b = 0;
                if (lane == 0) b = atomicAdd(hdr + H_OUT, (unsigned long long)__popcll(mh));
                b = __shfl(b, 0, 64);
                const unsigned long long q = b + lanes_below(mh);
                if (in_hi && (int64_t)q < capacity) {
                    Pair pr;
                    pr.r = (int32_t)i;
                    pr.s = (int32_t)(jb + lane);
                    pr.score = mine;
                    out[q] = pr;
                }
            }
            if (mb) {
                unsigned long long b = 0;
                if (lane == 0) b = atomicAdd(hdr + H_BAND, (unsigned long long)__popcll(mb));
                b = __shfl(b, 0, 64);
                const unsigned long long q = b + lanes_below(mb);
                if (in_lo && !in_hi && (int64_t)q < band_cap)
                    band[q] = make_int2((int)i, (int)(jb + lane));
            }
        }
    }
}

hipError_t launch_threshold_nlj(const ThresholdArgs& a, hipStream_t st) {
    if (a.Kp > 64 * kNljMaxNV) return hipErrorInvalidValue;
    if (a.nR == 0 || a.nS == 0) return hipSuccess;
    hipLaunchKernelGGL(nlj_threshold, dim3(8192), dim3(256), 0, st, (const float*)a.A,
                       (const float*)a.B, a.Kp, a.nR, a.nS, a.lo, a.hi, a.out, a.capacity, a.band,
                       a.band_cap, a.hdr);
    return hipGetLastError();
}

}  // namespace ej
