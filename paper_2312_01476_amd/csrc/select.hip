// select.hip -- a relational selection evaluated on the device, for pushing
// it below the join.
//
// The paper's scan-versus-probe study (Section VI.E) runs the join after a
// relational pre-filter on another attribute of the relation, at
// selectivities from 1% to 100%: the scan-based (tensor) join only
// contracts the tuples that pass.  This kernel turns a range predicate
// lo <= col[i] < hi on a float attribute column into the strictly ascending
// list of the passing row ids that the join entry points take as a
// selection.  Three launches: hits per block (fixed grid), one exclusive scan
// of the block counts (which also writes the total), and a stable write in
// which each block walks its contiguous part of the column in order.
#include "common.hpp"
#include "launch.hpp"

namespace ej {

constexpr int kSelBlocks = 1024;

size_t select_range_workspace() { return 2 * kSelBlocks * sizeof(int64_t); }

__device__ __forceinline__ bool sel_hit(const float* __restrict__ col, int64_t i, int64_t end,
                                        float lo, float hi) {
    if (i >= end) return false;
    const float v = col[i];
    return lo <= v && v < hi;  // NaN passes neither
}

__global__ __launch_bounds__(256) void select_count(const float* __restrict__ col, int64_t n,
                                                    float lo, float hi,
                                                    int64_t* __restrict__ blk_cnt) {
    __shared__ int64_t s_c[4];
    const int64_t per = (n + kSelBlocks - 1) / kSelBlocks;
    const int64_t c0 = (int64_t)blockIdx.x * per, c1 = min(n, c0 + per);
    int64_t c = 0;
    for (int64_t i = c0 + threadIdx.x; i < c1; i += blockDim.x)
        c += sel_hit(col, i, c1, lo, hi) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) blk_cnt[blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
}

// exclusive scan of the kSelBlocks counts (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void select_scan(const int64_t* __restrict__ blk_cnt,
                                                    int64_t* __restrict__ blk_off,
                                                    int64_t* __restrict__ n_sel) {
    __shared__ int64_t s[kSelBlocks];
    const int t = threadIdx.x;
    s[t] = blk_cnt[t];
    __syncthreads();
    for (int d = 1; d < kSelBlocks; d <<= 1) {  // Hillis-Steele inclusive scan
        const int64_t v = t >= d ? s[t - d] : 0;
        __syncthreads();
        s[t] += v;
        __syncthreads();
    }
    blk_off[t] = s[t] - blk_cnt[t];
    if (t == kSelBlocks - 1) *n_sel = s[t];
}

__global__ __launch_bounds__(256) void select_write(const float* __restrict__ col, int64_t n,
                                                    float lo, float hi,
                                                    const int64_t* __restrict__ blk_off,
                                                    int32_t* __restrict__ ids) {
    __shared__ int s_w[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t per = (n + kSelBlocks - 1) / kSelBlocks;
    const int64_t c0 = (int64_t)blockIdx.x * per, c1 = min(n, c0 + per);
    int64_t off = blk_off[blockIdx.x];
    for (int64_t base = c0; base < c1; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const bool hit = sel_hit(col, i, c1, lo, hi);
        const uint64_t m = __ballot(hit);
        if (lane == 0) s_w[wave] = __popcll(m);
        __syncthreads();
        int before = 0;
        for (int w = 0; w < wave; ++w) before += s_w[w];
        const int total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (hit) ids[off + before + lanes_below(m)] = (int32_t)i;
        off += total;
        __syncthreads();  // s_w is rewritten by the next round
    }
}

hipError_t launch_select_range(const float* col, int64_t n, float lo, float hi, int32_t* ids,
                               int64_t* n_sel, void* ws, hipStream_t st) {
    int64_t* blk_cnt = (int64_t*)ws;
    int64_t* blk_off = blk_cnt + kSelBlocks;
    hipLaunchKernelGGL(select_count, dim3(kSelBlocks), dim3(256), 0, st, col, n, lo, hi, blk_cnt);
    hipLaunchKernelGGL(select_scan, dim3(1), dim3(kSelBlocks), 0, st, (const int64_t*)blk_cnt,
                       blk_off, n_sel);
    hipLaunchKernelGGL(select_write, dim3(kSelBlocks), dim3(256), 0, st, col, n, lo, hi,
                       (const int64_t*)blk_off, ids);
    return hipGetLastError();
}

}  // namespace ej
