// mlp.hip -- the learned prefilter's network: training (forward, backward,
// Adam) and inference kernels.
//
// The network maps a normalised embedding row x (d values) to a unit code:
// h = ReLU(x W1 + b1) (256), z = h W2 + b2 (64), u = z / ||z||.  The
// predicted similarity of a pair is u_r . u_s.  Weights are kept as FP32
// masters with BF16 copies; every product uses the BF16 values and
// accumulates in FP32.
//
// Training runs on small batches (a few thousand pairs) with plain SIMT
// kernels: a strided FP32 GEMM covers every product of the forward and
// backward passes, a per-pair kernel does the loss and the backward step
// through the pair product and the normalisation, and Adam updates the
// masters and refreshes the BF16 copies.  Inference codes millions of rows
// and runs on the matrix cores with the tile mainloop of the join (BF16
// operands, FP32 accumulate), the hidden layer stored in BF16.
#include "common.hpp"
#include "launch.hpp"
#include "mlp.hpp"
#include "mma.hpp"
#include "tile_body.hpp"

namespace ej {

__device__ __forceinline__ float bf16r(float x) { return bf16_to_f32(f32_to_bf16_rne(x)); }

template <typename T>
__device__ __forceinline__ float ldf(const T* p, int64_t i);
template <>
__device__ __forceinline__ float ldf<float>(const float* p, int64_t i) {
    return p[i];
}
template <>
__device__ __forceinline__ float ldf<uint16_t>(const uint16_t* p, int64_t i) {
    return bf16_to_f32(p[i]);
}

// ---------------------------------------------------------------------------
// strided SIMT GEMM: C[i][j] = sum_k A(i,k) B(k,j) (+ bias[j]) (* (mask>0))
// A(i,k) = A[i*sai + k*sak] (optionally ReLU-ed), B(k,j) = B[k*sbk + j*sbj].
// 64x64 output tile per 256 threads, 4x4 per thread, K in steps of 16
// through LDS.  The bias is rounded to BF16 (it is a weight).
// ---------------------------------------------------------------------------
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void gemm_simt(int M, int N, int K, const TA* __restrict__ A,
                                                 int64_t sai, int64_t sak, bool reluA,
                                                 const TB* __restrict__ B, int64_t sbk,
                                                 int64_t sbj, float* __restrict__ C, int64_t ldc,
                                                 const float* __restrict__ bias,
                                                 const float* __restrict__ mask) {
    __shared__ float sA[16][64 + 1];
    __shared__ float sB[16][64 + 1];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int ti = (tid >> 4) * 4, tj = (tid & 15) * 4;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += 16) {
        // 64x16 of A and 16x64 of B: 1024 values each, 4 per thread
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            const int r = e & 63, c = e >> 6;  // A: row r, k c
            float va = 0.0f;
            if (i0 + r < M && k0 + c < K) {
                va = ldf(A, (int64_t)(i0 + r) * sai + (int64_t)(k0 + c) * sak);
                if (reluA) va = fmaxf(va, 0.0f);
            }
            sA[c][r] = va;
            float vb = 0.0f;  // B: k c, col r
            if (j0 + r < N && k0 + c < K) vb = ldf(B, (int64_t)(k0 + c) * sbk + (int64_t)(j0 + r) * sbj);
            sB[c][r] = vb;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            float a[4], b[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
                a[x] = sA[k][ti + x];
                b[x] = sB[k][tj + x];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = fmaf(a[x], b[y], acc[x][y]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int i = i0 + ti + x, j = j0 + tj + y;
            if (i >= M || j >= N) continue;
            float v = acc[x][y];
            if (bias) v += bf16r(bias[j]);
            if (mask && !(mask[(int64_t)i * ldc + j] > 0.0f)) v = 0.0f;
            C[(int64_t)i * ldc + j] = v;
        }
}

template <typename TA, typename TB>
static hipError_t gemm(int M, int N, int K, const TA* A, int64_t sai, int64_t sak, bool reluA,
                       const TB* B, int64_t sbk, int64_t sbj, float* C, int64_t ldc,
                       const float* bias, const float* mask, hipStream_t st) {
    if (M <= 0 || N <= 0) return hipSuccess;
    dim3 g((unsigned)((N + 63) / 64), (unsigned)((M + 63) / 64));
    hipLaunchKernelGGL((gemm_simt<TA, TB>), g, dim3(256), 0, st, M, N, K, A, sai, sak, reluA, B,
                       sbk, sbj, C, ldc, bias, mask);
    return hipGetLastError();
}

// gather the rows of the pair batch: slot i < B is row pr[i], slot B + i is
// row ps[i]; BF16 rows of X (ldx elements apart) to FP32 rows of Dp values
// (zero beyond dim)
__global__ void mlp_gather(const uint16_t* __restrict__ X, int64_t ldx, int64_t rows, int dim,
                           int Dp, const int32_t* __restrict__ pr,
                           const int32_t* __restrict__ ps, int B, float* __restrict__ Xb) {
    const int slot = blockIdx.x;
    const int64_t row = slot < B ? pr[slot] : ps[slot - B];
    const bool ok = row >= 0 && row < rows;  // an index out of range reads as zeros
    for (int k = threadIdx.x; k < Dp; k += blockDim.x)
        Xb[(int64_t)slot * Dp + k] = (ok && k < dim) ? bf16_to_f32(X[row * ldx + k]) : 0.0f;
}

// loss and backward through p = u_r . u_s and u = z / ||z||: one wave per
// pair, lane o holds coordinate o of both codes
__global__ __launch_bounds__(256) void mlp_pair_loss(const float* __restrict__ Z,
                                                     const float* __restrict__ t, int B,
                                                     float lam, float theta_lo,
                                                     float* __restrict__ dZ,
                                                     float* __restrict__ loss) {
    const int lane = threadIdx.x & 63;
    const int pair = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (pair >= B) return;
    const float zr = Z[(int64_t)pair * MLP_OUT + lane];
    const float zs = Z[(int64_t)(B + pair) * MLP_OUT + lane];
    const float nr = sqrtf(wave_sum(zr * zr));
    const float ns = sqrtf(wave_sum(zs * zs));
    const float ur = zr / nr, us = zs / ns;
    const float p = wave_sum(ur * us);
    const float tt = t[pair];
    const float under = tt >= theta_lo ? fmaxf(0.0f, tt - p) : 0.0f;
    const float dp = (2.0f / (float)B) * ((p - tt) - lam * under);
    const float dur = dp * us, dus = dp * ur;
    const float pr_ = wave_sum(ur * dur), ps_ = wave_sum(us * dus);
    dZ[(int64_t)pair * MLP_OUT + lane] = (dur - ur * pr_) / nr;
    dZ[(int64_t)(B + pair) * MLP_OUT + lane] = (dus - us * ps_) / ns;
    if (lane == 0) atomicAdd(loss, ((p - tt) * (p - tt) + lam * under * under) / (float)B);
}

// column sums of an M x N matrix (bias gradients): a workgroup per 64
// columns, each of its 16 waves sums every 16th row (lane = column), then the
// 16 partial sums are added in wave order (deterministic)
constexpr int kColsumWaves = 16;
__global__ __launch_bounds__(64 * kColsumWaves) void mlp_colsum(const float* __restrict__ G, int M,
                                                                int N, float* __restrict__ out) {
    __shared__ float s_part[kColsumWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int j = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (j < N)
        for (int i = w; i < M; i += kColsumWaves) s += G[(int64_t)i * N + j];
    s_part[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < N) {
        float t = 0.0f;
        for (int q = 0; q < kColsumWaves; ++q) t += s_part[q][lane];
        out[j] = t;
    }
}

// Adam on the flat parameter vector; the step counter lives in the state
__global__ void mlp_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ Mv,
                         float* __restrict__ Vv, int64_t n, const int64_t* __restrict__ step,
                         float lr, float b1, float b2, float eps) {
    const double t = (double)(*step + 1);
    const float c1 = (float)(1.0 - pow((double)b1, t));
    const float c2 = (float)(1.0 - pow((double)b2, t));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float g = G[i];
        const float m = b1 * Mv[i] + (1.0f - b1) * g;
        const float v = b2 * Vv[i] + (1.0f - b2) * g * g;
        Mv[i] = m;
        Vv[i] = v;
        P[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    }
}

__global__ void mlp_step_inc(int64_t* step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += 1;
}

// BF16 copies of the weights, transposed so that both layers read
// K-contiguous rows: W1t[j][k] = W1[k][j] (zero for k >= dim), W2t[o][h] = W2[h][o]
__global__ void mlp_refresh(const float* __restrict__ P, int dim, int Dp,
                            uint16_t* __restrict__ W1t, uint16_t* __restrict__ W2t) {
    const int64_t n1 = (int64_t)MLP_HIDDEN * Dp;
    const int64_t n2 = (int64_t)MLP_OUT * MLP_HIDDEN;
    const float* W1 = P;
    const float* W2 = P + (int64_t)dim * MLP_HIDDEN + MLP_HIDDEN;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n1 + n2;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < n1) {
            const int j = (int)(e / Dp), k = (int)(e % Dp);
            W1t[e] = k < dim ? f32_to_bf16_rne(W1[(int64_t)k * MLP_HIDDEN + j]) : (uint16_t)0;
        } else {
            const int64_t f = e - n1;
            const int o = (int)(f / MLP_HIDDEN), hh = (int)(f % MLP_HIDDEN);
            W2t[f] = f32_to_bf16_rne(W2[(int64_t)hh * MLP_OUT + o]);
        }
    }
}

__global__ void mlp_copy(float* __restrict__ dst, const float* __restrict__ src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src ? src[i] : 0.0f;
}

__global__ void mlp_zero_i64(int64_t* p) {
    if (threadIdx.x == 0) *p = 0;
}

hipError_t launch_mlp_init(const MlpDev& m, const float* params, hipStream_t st) {
    hipLaunchKernelGGL(mlp_copy, dim3(256), dim3(256), 0, st, m.P, params, m.np);
    hipLaunchKernelGGL(mlp_copy, dim3(256), dim3(256), 0, st, m.G, (const float*)nullptr, m.np);
    hipLaunchKernelGGL(mlp_copy, dim3(256), dim3(256), 0, st, m.M, (const float*)nullptr, m.np);
    hipLaunchKernelGGL(mlp_copy, dim3(256), dim3(256), 0, st, m.V, (const float*)nullptr, m.np);
    hipLaunchKernelGGL(mlp_zero_i64, dim3(1), dim3(64), 0, st, m.step);
    hipLaunchKernelGGL(mlp_refresh, dim3(256), dim3(256), 0, st, m.P, m.dim, m.Dp, m.W1t, m.W2t);
    return hipGetLastError();
}

hipError_t launch_mlp_restored(const MlpDev& m, hipStream_t st) {
    hipLaunchKernelGGL(mlp_copy, dim3(256), dim3(256), 0, st, m.G, (const float*)nullptr, m.np);
    hipLaunchKernelGGL(mlp_refresh, dim3(256), dim3(256), 0, st, m.P, m.dim, m.Dp, m.W1t, m.W2t);
    return hipGetLastError();
}

hipError_t launch_mlp_train_step(const MlpDev& m, const uint16_t* X, int64_t ldx, int64_t rows,
                                 const int32_t* pr, const int32_t* ps, const float* t, int B,
                                 const MlpHyper& hp, const MlpTrainWs& w, float* loss,
                                 hipStream_t st) {
    const int R2 = 2 * B;
    const int D = m.dim, Dp = m.Dp, H = MLP_HIDDEN, O = MLP_OUT;
    hipError_t e;
    float* gW1 = m.G;
    float* gb1 = m.G + (int64_t)D * H;
    float* gW2 = gb1 + H;
    float* gb2 = gW2 + (int64_t)H * O;
    const float* b1 = m.P + (int64_t)D * H;
    const float* b2 = b1 + H + (int64_t)H * O;
    hipLaunchKernelGGL(mlp_copy, dim3(1), dim3(64), 0, st, loss, (const float*)nullptr,
                       (int64_t)1);
    hipLaunchKernelGGL(mlp_gather, dim3(R2), dim3(256), 0, st, X, ldx, rows, D, Dp, pr, ps, B,
                       w.Xb);
    // forward: A1 = Xb W1 + b1 ; Z = ReLU(A1) W2 + b2
    if ((e = gemm<float, uint16_t>(R2, H, Dp, w.Xb, Dp, 1, false, m.W1t, 1, Dp, w.A1, H, b1,
                                   nullptr, st)) != hipSuccess)
        return e;
    if ((e = gemm<float, uint16_t>(R2, O, H, w.A1, H, 1, true, m.W2t, 1, H, w.Z, O, b2, nullptr,
                                   st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(mlp_pair_loss, dim3((B + 3) / 4), dim3(256), 0, st, w.Z, t, B, hp.lambda,
                       hp.theta_lo, w.dZ, loss);
    // backward: gW2 = ReLU(A1)^T dZ, gb2 = sum dZ, dA1 = (dZ W2^T) * (A1 > 0)
    if ((e = gemm<float, float>(H, O, R2, w.A1, 1, H, true, w.dZ, O, 1, gW2, O, nullptr, nullptr,
                                st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(mlp_colsum, dim3((O + 63) / 64), dim3(64 * kColsumWaves), 0, st, w.dZ, R2, O,
                       gb2);
    if ((e = gemm<float, uint16_t>(R2, H, O, w.dZ, O, 1, false, m.W2t, H, 1, w.dA1, H, nullptr,
                                   w.A1, st)) != hipSuccess)
        return e;
    // gW1 = Xb^T dA1 (rows k < dim), gb1 = sum dA1
    if ((e = gemm<float, float>(D, H, R2, w.Xb, 1, Dp, false, w.dA1, H, 1, gW1, H, nullptr,
                                nullptr, st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(mlp_colsum, dim3((H + 63) / 64), dim3(64 * kColsumWaves), 0, st, w.dA1, R2,
                       H, gb1);
    if (hp.grad_only) return hipGetLastError();
    hipLaunchKernelGGL(mlp_adam, dim3(512), dim3(256), 0, st, m.P, m.G, m.M, m.V, m.np, m.step,
                       hp.lr, hp.beta1, hp.beta2, hp.eps);
    hipLaunchKernelGGL(mlp_step_inc, dim3(1), dim3(64), 0, st, m.step);
    hipLaunchKernelGGL(mlp_refresh, dim3(256), dim3(256), 0, st, m.P, m.dim, m.Dp, m.W1t, m.W2t);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// inference on the matrix cores
// ---------------------------------------------------------------------------

// layer 1: H = BF16(ReLU(X W1 + b1)), X the prepared rows (Dp BF16 values
// per row, rows up to a multiple of 128 readable)
__global__ __launch_bounds__(256) void mlp_l1(const uint16_t* __restrict__ X, int Dp,
                                              const uint16_t* __restrict__ W1t,
                                              const float* __restrict__ b1,
                                              uint16_t* __restrict__ Hb) {
    constexpr int BM = 128, BN = 128, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    const int tm = blockIdx.y, tn = blockIdx.x;
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)X, (const char*)W1t, nullptr, nullptr,
                                          Dp * 2, tm, tn, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
#pragma unroll
    for (int j = 0; j < TG::FN; ++j) {
        const int col = tn * BN + wn * TG::WTN + j * 32 + r32;
        const float bias = bf16r(b1[col]);
#pragma unroll
        for (int i = 0; i < TG::FM; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t row = (int64_t)tm * BM + wm * TG::WTM + i * 32 + 8 * (e >> 2) +
                                    4 * h + (e & 3);
                Hb[row * MLP_HIDDEN + col] = f32_to_bf16_rne(fmaxf(acc[i][j][e] + bias, 0.0f));
            }
    }
}

// layer 2: Z = H W2 + b2 (FP32)
__global__ __launch_bounds__(256) void mlp_l2(const uint16_t* __restrict__ Hb,
                                              const uint16_t* __restrict__ W2t,
                                              const float* __restrict__ b2,
                                              float* __restrict__ Z) {
    constexpr int BM = 128, BN = 64, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    const int tm = blockIdx.x;
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)Hb, (const char*)W2t, nullptr, nullptr,
                                          MLP_HIDDEN * 2, tm, 0, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
#pragma unroll
    for (int j = 0; j < TG::FN; ++j) {
        const int col = wn * TG::WTN + j * 32 + r32;
        const float bias = bf16r(b2[col]);
#pragma unroll
        for (int i = 0; i < TG::FM; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int64_t row = (int64_t)tm * BM + wm * TG::WTM + i * 32 + 8 * (e >> 2) +
                                    4 * h + (e & 3);
                Z[row * MLP_OUT + col] = acc[i][j][e] + bias;
            }
    }
}

// u = z / ||z|| for rows < n, one wave per row
__global__ __launch_bounds__(256) void mlp_normalise(const float* __restrict__ Z, int64_t n,
                                                     float* __restrict__ U) {
    const int lane = threadIdx.x & 63;
    for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < n;
         row += (int64_t)gridDim.x * 4) {
        const float z = Z[row * MLP_OUT + lane];
        const float nz = sqrtf(wave_sum(z * z));
        U[row * MLP_OUT + lane] = z / nz;
    }
}

hipError_t launch_mlp_forward(const MlpDev& m, const uint16_t* X, int64_t n, uint16_t* Hb,
                              float* Z, float* U, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + 127) / 128;
    if (tiles > 65535 * 64) return hipErrorInvalidValue;
    const float* b1 = m.P + (int64_t)m.dim * MLP_HIDDEN;
    const float* b2 = b1 + MLP_HIDDEN + (int64_t)MLP_HIDDEN * MLP_OUT;
    // grid.y carries the row tiles (up to 65535), grid.x the two column tiles
    for (int64_t t0 = 0; t0 < tiles; t0 += 65535) {
        const int64_t nt = std::min<int64_t>(65535, tiles - t0);
        hipLaunchKernelGGL(mlp_l1, dim3(MLP_HIDDEN / 128, (unsigned)nt), dim3(256), 0, st,
                           X + t0 * 128 * m.Dp, m.Dp, m.W1t, b1, Hb + t0 * 128 * MLP_HIDDEN);
    }
    hipLaunchKernelGGL(mlp_l2, dim3((unsigned)tiles), dim3(256), 0, st, Hb, m.W2t, b2, Z);
    int64_t blocks = std::min<int64_t>((n + 3) / 4, 8192);
    hipLaunchKernelGGL(mlp_normalise, dim3((unsigned)blocks), dim3(256), 0, st, Z, n, U);
    return hipGetLastError();
}

}  // namespace ej
