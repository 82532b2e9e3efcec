// batch.hip -- the persistent contraction kernel of the batched threshold
// join, and the small bookkeeping kernels around it.
//
// Many joins of uneven |R|, |S| and theta are served by ONE launch: the
// output tiles of all jobs form a flat work list (job j owns items
// [tile_base_j, tile_base_j + tiles_m_j * tiles_n_j)), and a grid sized to
// fill the GPU once pulls items from an atomic counter until the list is
// exhausted.  Jobs are stored largest first, so the last items handed out
// are small and the tail of the launch stays short.  Each item runs the same
// tile body as the single-join kernel with its job's operands, band edges,
// output buffer and counters; band pairs of all jobs go to one shared list
// tagged with the job index.
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "mma.hpp"
#include "tile_body.hpp"

namespace ej {

template <int PREC, int BM, int BN, int WM, int WN, bool BIG = false>
__global__ __launch_bounds__(WM* WN * 64, (BM * BN <= 128 * 128) ? 2 : 1) void batch_tile(const BatchHead* __restrict__ head,
                                                          const BatchJob* __restrict__ jobs,
                                                          unsigned long long* __restrict__ bctr) {
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    __shared__ int64_t s_item;
    __shared__ int s_job;
    // dense mode: every tile of every job; prefilter mode: the work list
    const int64_t* work = head->work;
    const int64_t total = work ? (int64_t)*head->n_work : head->n_tiles;
    const int n_jobs = head->n_jobs;
    int4* band = head->band;
    const int64_t band_cap = head->band_cap;
    __shared__ int s_tm, s_tn;
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t item = (int64_t)atomicAdd(bctr + B_ITEM, 1ull);
            int job = 0, tm = 0, tn = 0;
            if (item < total) {
                if (work) {
                    const int64_t w = work[item];
                    job = (int)(w >> 48);
                    tm = (int)((w >> 24) & 0xFFFFFF);
                    tn = (int)(w & 0xFFFFFF);
                } else {
                    // last job whose first item is <= item
                    int lo = 0, hi = n_jobs - 1;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (jobs[mid].tile_base <= item) lo = mid;
                        else hi = mid - 1;
                    }
                    job = lo;
                    raster_tile((int)(item - jobs[lo].tile_base), jobs[lo].tiles_m,
                                jobs[lo].tiles_n, tm, tn);
                }
            }
            s_item = item;
            s_job = job;
            s_tm = tm;
            s_tn = tn;
        }
        __syncthreads();
        const int64_t item = s_item;
        const int job = __builtin_amdgcn_readfirstlane(s_job);
        const int tm = __builtin_amdgcn_readfirstlane(s_tm);
        const int tn = __builtin_amdgcn_readfirstlane(s_tn);
        __syncthreads();  // the shared slots are rewritten by the next iteration
        if (item >= total) break;
        const BatchJob& J = jobs[job];
        if (J.hdr[H_FLAGS] != 0) continue;  // bad input rows in this job
        if constexpr (BIG)
            big_tile_body<PREC, true>(sm, J.A, J.B, J.info_r, J.info_s, J.Kp_bytes, J.nR, J.nS, tm,
                                      tn, J.lo, J.hi, J.out, J.capacity, J.hdr + H_OUT, band,
                                      band_cap, bctr + B_BAND, job, J.perm_r, J.perm_s,
                                      J.kg_last);
        else
            tile_body<PREC, BM, BN, WM, WN, true>(sm, J.A, J.B, J.info_r, J.info_s, J.Kp_bytes,
                                                  J.nR, J.nS, tm, tn, J.lo, J.hi, J.out,
                                                  J.capacity, J.hdr + H_OUT, band, band_cap,
                                                  bctr + B_BAND, job, J.perm_r, J.perm_s,
                                                  J.kg_last);
    }
}

// Zero the pass counters and every job's counters (a kernel, not a memset,
// so that a captured graph of the pass replays correctly).
__global__ void batch_zero(const BatchHead* __restrict__ head, unsigned long long* bctr) {
    const int64_t n = (int64_t)head->n_jobs * H_COUNT;
    unsigned long long* hdrs = head->hdrs;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 < B_COUNT) bctr[i0] = 0ull;
    for (int64_t i = i0; i < n; i += (int64_t)gridDim.x * blockDim.x) hdrs[i] = 0ull;
}

// Per-job match counts to the caller's device array (asynchronous mode):
// the count, or minus the status code of a failure found on the device
// (the band list is shared, so its overflow fails every job).
__global__ void batch_counts(const BatchHead* __restrict__ head, const BatchJob* __restrict__ jobs,
                             const unsigned long long* __restrict__ bctr) {
    int64_t* n_out = head->n_out;
    if (n_out == nullptr) return;
    const bool band_over = (int64_t)bctr[B_BAND] > head->band_cap;
    for (int j = threadIdx.x; j < head->n_jobs; j += blockDim.x) {
        const unsigned long long* h = jobs[j].hdr;
        int64_t v = (int64_t)h[H_OUT];
        if (h[H_FLAGS] & F_NONFINITE) v = -4;      // EJOIN_E_NONFINITE
        else if (h[H_FLAGS] & F_RANGE) v = -7;     // EJOIN_E_RANGE
        else if (band_over) v = -3;                // EJOIN_E_WORKSPACE
        n_out[jobs[j].user] = v;
    }
}

template <int PREC, int BM, int BN, int WM, int WN, bool BIG = false>
static hipError_t run_batch(const BatchHead* head, const BatchJob* jobs, unsigned long long* bctr,
                            int grid, hipStream_t st) {
    hipLaunchKernelGGL((batch_tile<PREC, BM, BN, WM, WN, BIG>), dim3((unsigned)grid),
                       dim3(WM * WN * 64), 0, st, head, jobs, bctr);
    return hipGetLastError();
}

template <int PREC, int BM, int BN, int WM, int WN, bool BIG = false>
static int occ_of() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_tile<PREC, BM, BN, WM, WN, BIG>,
                                                     WM * WN * 64, 0) != hipSuccess)
        return 0;
    return n;
}

bool batch_has_tile(int tile_id) {
    switch (tile_id) {
        case 1: case 2: case 3: case 4: case 5: case 6: case 8: case 10: case 11: case 16:
        case 17: case 18: case 19: case 22:
            return true;
        default: return false;
    }
}

// Workgroups per CU the persistent kernel of a tile keeps resident (0: the
// tile has no batch form).
int batch_occupancy(int tile_id) {
    switch (tile_id) {
        case 1: return occ_of<P_FP32, 128, 128, 2, 2>();
        case 2: return occ_of<P_FP32, 64, 64, 2, 2>();
        case 3: return occ_of<P_BF16, 128, 128, 2, 2>();
        case 4: return occ_of<P_BF16, 256, 128, 2, 2>();
        case 5: return occ_of<P_FP8, 128, 128, 2, 2>();
        case 6: return occ_of<P_FP8, 256, 128, 2, 2>();
        case 8: return occ_of<P_BF16, 256, 256, 2, 4>();
        case 10: return occ_of<P_FP8, 256, 256, 2, 4>();
        case 11: return occ_of<P_FP32, 256, 128, 2, 2>();
        case 16: return occ_of<P_BF16, 256, 256, 2, 2, true>();
        case 17: return occ_of<P_FP8, 256, 256, 2, 2, true>();
        case 18: return occ_of<P_FP32, 256, 256, 2, 2, true>();
        case 19: return batch_panel_occupancy();
        case 22: return batch_panel2_occupancy();
        default: return 0;
    }
}

hipError_t launch_batch_tile(int tile_id, const BatchHead* head, const BatchJob* jobs,
                             unsigned long long* bctr, int grid, hipStream_t st, bool worklist) {
    switch (tile_id) {
        case 1: return run_batch<P_FP32, 128, 128, 2, 2>(head, jobs, bctr, grid, st);
        case 2: return run_batch<P_FP32, 64, 64, 2, 2>(head, jobs, bctr, grid, st);
        case 3: return run_batch<P_BF16, 128, 128, 2, 2>(head, jobs, bctr, grid, st);
        case 4: return run_batch<P_BF16, 256, 128, 2, 2>(head, jobs, bctr, grid, st);
        case 5: return run_batch<P_FP8, 128, 128, 2, 2>(head, jobs, bctr, grid, st);
        case 6: return run_batch<P_FP8, 256, 128, 2, 2>(head, jobs, bctr, grid, st);
        case 8: return run_batch<P_BF16, 256, 256, 2, 4>(head, jobs, bctr, grid, st);
        case 10: return run_batch<P_FP8, 256, 256, 2, 4>(head, jobs, bctr, grid, st);
        case 11: return run_batch<P_FP32, 256, 128, 2, 2>(head, jobs, bctr, grid, st);
        case 16: return run_batch<P_BF16, 256, 256, 2, 2, true>(head, jobs, bctr, grid, st);
        case 17: return run_batch<P_FP8, 256, 256, 2, 2, true>(head, jobs, bctr, grid, st);
        case 18: return run_batch<P_FP32, 256, 256, 2, 2, true>(head, jobs, bctr, grid, st);
        case 19: return launch_batch_panel(head, jobs, bctr, grid, worklist, st);
        case 22: return launch_batch_panel2(head, jobs, bctr, grid, worklist, st);
        default: return hipErrorInvalidValue;
    }
}

// Per job with a measured band: the band edges from the largest error norms
// its prep found (the bound of the single join's band_edges), written into
// the job table that the contraction kernels read.
__global__ void batch_band_edges(const BatchHead* __restrict__ head, BatchJob* __restrict__ jobs) {
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < head->n_jobs;
         j += gridDim.x * blockDim.x) {
        BatchJob& J = jobs[j];
        if (!J.measured) continue;
        const unsigned long long* h = J.hdr;
        const double er = (double)__uint_as_float((uint32_t)h[H_ENORM_R]) * 1.001 + 1e-7;
        const double es =
            (double)__uint_as_float((uint32_t)h[J.alias ? H_ENORM_R : H_ENORM_S]) * 1.001 + 1e-7;
        const double f = J.band_f;
        double d = er * (1.0 + es) + es + f * (1.0 + er) * (1.0 + es);
        if (!(d <= J.band_rig)) d = J.band_rig;
        const double lo = J.theta - d, hi = J.theta + d;
        float flo = (float)lo, fhi = (float)hi;
        if ((double)flo > lo) flo = nextafterf(flo, -INFINITY);
        if ((double)fhi < hi) fhi = nextafterf(fhi, INFINITY);
        if (J.all64) fhi = INFINITY;
        J.lo = flo;
        J.hi = fhi;
    }
}

hipError_t launch_batch_band_edges(const BatchHead* head, BatchJob* jobs, hipStream_t st) {
    hipLaunchKernelGGL(batch_band_edges, dim3(4), dim3(256), 0, st, head, jobs);
    return hipGetLastError();
}

hipError_t launch_batch_zero(const BatchHead* head, unsigned long long* bctr, hipStream_t st) {
    hipLaunchKernelGGL(batch_zero, dim3(64), dim3(256), 0, st, head, bctr);
    return hipGetLastError();
}

hipError_t launch_batch_counts(const BatchHead* head, const BatchJob* jobs,
                               const unsigned long long* bctr, hipStream_t st) {
    hipLaunchKernelGGL(batch_counts, dim3(1), dim3(256), 0, st, head, jobs, bctr);
    return hipGetLastError();
}

}  // namespace ej
