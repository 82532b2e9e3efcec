// prune.hip -- exact pruning of tile pairs for the batched join.
//
// The certified counterpart of the learned prefilter: every relation of the
// batch is put in an order that keeps similar rows together, cut into tiles
// of 128 rows, and a tile pair (T, U) is skipped only when a rigorous upper
// bound of the cosine of every one of its pairs, taken in the original
// embedding space, lies below theta.  The skipped pairs then all have
// sim64 < theta and the result is the exact join.
//
//  * Order: the input rows are coded by a fixed random +-1 projection to
//    64 dimensions (no training), normalised; the anchor keys and the stable
//    per-relation sort of the prefilter follow (prefilter.hip).  The order
//    only decides how tight the tiles are, never what is returned.
//  * Per tile T of prepared rows x_r (BF16, in tile order): the direction d_T
//    of the rows' mean and the angular radius A_T, an upper bound of the
//    angle between d_T and every exact unit row r / |r| of T: the largest
//    angle measured on the prepared rows, plus the angle their rounding can
//    hide (|x_r - r/|r|| <= e_r, the row's quantisation error norm plus the
//    FP32 normalisation error), plus slack for the FP32 evaluation.
//  * Tile to rows (on the matrix cores): M1 = max over the rows s of U of
//    d_T . x_s, M2 = max over the rows r of T of d_U . x_r.  Raised by the
//    BF16 rounding of d and the rows' error norms, m1 bounds d_T . s/|s| for
//    every s of U; the angle between r and s is then at least
//    acos(m1) - A_T (triangle inequality for angles), so
//        cos(r, s) <= cos(max(0, acos(m1) - A_T))
//    and the same with (M2, A_U).  The pair of tiles is kept when the smaller
//    bound reaches theta (minus slack for the FP32 cos).
#include "batch.hpp"
#include "common.hpp"
#include "launch.hpp"
#include "mma.hpp"
#include "prefilter.hpp"
#include "tile_body.hpp"

namespace ej {

namespace {

__device__ __forceinline__ int xp_seg_of(const PrepSeg* __restrict__ segs, int nseg,
                                         int64_t row) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (segs[mid].row_base <= row) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int xp_job_of(const BatchJob* __restrict__ jobs, int n_jobs,
                                         int64_t item, bool side) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if ((side ? jobs[mid].side_base : jobs[mid].tile_base) <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace

// The projection: P[o][k] = +-1/8 for k < dim (sign from a SplitMix64-style
// mix of the index), 0 beyond; BF16, 64 x Dp.
__global__ void xp_proj(int dim, int Dp, uint16_t* __restrict__ P) {
    const int64_t n = (int64_t)MLP_OUT * Dp;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(q % Dp);
        uint64_t z = (uint64_t)q * 0x9E3779B97F4A7C15ull + 0x5EEDull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        const float v = k < dim ? ((z & 1ull) ? 0.125f : -0.125f) : 0.0f;
        P[q] = f32_to_bf16_rne(v);
    }
}

// LDS written by some lanes of a wave and read by others: order the
// accesses (LDS operations of one wave complete in issue order)
__device__ __forceinline__ void wave_lds_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Totals over the wave of 16 per-lane values (transposed butterfly: half of
// the values cross at each step); lane l returns the total of value
// (l >> 2) & 15.
template <int H, int M>
__device__ __forceinline__ void xp_fold(float (&v)[16], int lane) {
    const bool up = lane & M;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const float send = up ? v[i] : v[i + H];
        const float keep = up ? v[i + H] : v[i];
        v[i] = keep + __shfl_xor(send, M, 64);
    }
}
__device__ __forceinline__ float xp_wave_sum16(float (&v)[16]) {
    const int lane = threadIdx.x & 63;
    xp_fold<8, 32>(v, lane);
    xp_fold<4, 16>(v, lane);
    xp_fold<2, 8>(v, lane);
    xp_fold<1, 4>(v, lane);
    float s = v[0];
    s += __shfl_xor(s, 2, 64);
    s += __shfl_xor(s, 1, 64);
    return s;
}

// Codes u = z / |z|, z = X P^T, straight from the caller's FP32 rows (row
// order of the input, before any preparation): 32 rows per wave, four waves
// per 128-row tile, the 64 code columns as two 32-column matrix-core blocks.
// The rows go through LDS in chunks of 64 elements: sixteen lanes read 256
// contiguous bytes of a row (four rows per load), round them to BF16 and
// store them as swizzled 128-byte rows, from which every lane takes the
// fragment of its row for each of the chunk's four BF16 steps.  P's
// fragments come from memory (64 x Dp, held in the caches).  The
// normalisation makes the rows' own norms drop out; elements past dim, and
// padding rows, are zero.
template <bool VEC>
__device__ __forceinline__ void xp_load4(const float* __restrict__ x, int k, int dim, float (&v)[4]) {
    typedef __attribute__((address_space(1))) const float* gf_ptr;
    if (VEC && k + 4 <= dim) {
        typedef float v4f __attribute__((ext_vector_type(4)));
        const v4f a = *(__attribute__((address_space(1))) const v4f*)(x + k);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = a[j];
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = k + j < dim ? *(gf_ptr)(x + k + j) : 0.0f;
    }
}

template <bool VEC>
__device__ __forceinline__ void xp_codes_rows(const PrepSeg& g, int64_t l0,
                                              const uint16_t* __restrict__ P, int Dp,
                                              float* __restrict__ U, uint16_t* __restrict__ Ub,
                                              int64_t zrow0, char* __restrict__ sx) {
    const int lane = threadIdx.x & 63, rr = lane & 31, kh = lane >> 5;
    // loader view: row 4 i + lane / 16 of the wave's 32, elements 4 (lane % 16) .. + 4
    const int lr = lane >> 4, lc = lane & 15;
    const float* xrow[8];
    bool live[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t r = l0 + 4 * i + lr;
        live[i] = r < g.rows;  // padding rows read row 0 and drop it
        xrow[i] = g.X + (live[i] ? r : 0) * g.ld;
    }
    typedef __attribute__((address_space(1))) const v4i* gv4_ptr;
    const uint16_t* p0 = P + (int64_t)rr * Dp + 8 * kh;
    const uint16_t* p1 = P + (int64_t)(32 + rr) * Dp + 8 * kh;
    v16f acc0, acc1;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        acc0[e] = 0.0f;
        acc1[e] = 0.0f;
    }
    const int nch = (g.dim + 63) / 64;
    for (int c = 0; c < nch; ++c) {
        float v[8][4];
#pragma unroll
        for (int i = 0; i < 8; ++i) xp_load4<VEC>(xrow[i], 64 * c + 4 * lc, g.dim, v[i]);
        v4i b0[4], b1[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            b0[t] = *(gv4_ptr)(p0 + 64 * c + 16 * t);
            b1[t] = *(gv4_ptr)(p1 + 64 * c + 16 * t);
        }
        wave_lds_fence();  // the previous chunk's fragments have been read
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            uint2 w;
            w.x = (uint32_t)f32_to_bf16_rne(live[i] ? v[i][0] : 0.0f) |
                  ((uint32_t)f32_to_bf16_rne(live[i] ? v[i][1] : 0.0f) << 16);
            w.y = (uint32_t)f32_to_bf16_rne(live[i] ? v[i][2] : 0.0f) |
                  ((uint32_t)f32_to_bf16_rne(live[i] ? v[i][3] : 0.0f) << 16);
            *(uint2*)(sx + lds_off(4 * i + lr, lc >> 1) + 8 * (lc & 1)) = w;
        }
        wave_lds_fence();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const v4i a = *(const v4i*)(sx + lds_off(rr, 2 * t + kh));
            Mma<P_BF16>::mma(a, b0[t], acc0, 0, 0);
            Mma<P_BF16>::mma(a, b1[t], acc1, 0, 0);
        }
    }
    // u = z / |z| per row (zero for zero, padding and non-finite rows), FP32
    // and BF16.  Lane (rr, kh) holds column rr (and 32 + rr) of rows
    // 8 (e / 4) + 4 kh + e % 4: the squares are totalled over the 32 lanes of
    // each half, row e's total landing in lane 2 e of the half.
    float q[16];
#pragma unroll
    for (int e = 0; e < 16; ++e) q[e] = acc0[e] * acc0[e] + acc1[e] * acc1[e];
    xp_fold<8, 16>(q, lane);
    xp_fold<4, 8>(q, lane);
    xp_fold<2, 4>(q, lane);
    xp_fold<1, 2>(q, lane);
    const float qt = q[0] + __shfl_xor(q[0], 1, 64);
#pragma unroll
    for (int e = 0; e < 16; ++e) {
        const float nz = sqrtf(__shfl(qt, 32 * kh + 2 * e, 64));
        const float u0 = nz > 0.0f ? acc0[e] / nz : 0.0f;
        const float u1 = nz > 0.0f ? acc1[e] / nz : 0.0f;
        const int64_t row = zrow0 + 8 * (e >> 2) + 4 * kh + (e & 3);
        U[row * MLP_OUT + rr] = u0;
        U[row * MLP_OUT + 32 + rr] = u1;
        Ub[row * MLP_OUT + rr] = f32_to_bf16_rne(u0);
        Ub[row * MLP_OUT + 32 + rr] = f32_to_bf16_rne(u1);
    }
}

__global__ __launch_bounds__(256) void xp_codes_raw(const BatchHead* __restrict__ head,
                                                    const PrepSeg* __restrict__ segs,
                                                    const uint16_t* __restrict__ P, int Dp,
                                                    float* __restrict__ U,
                                                    uint16_t* __restrict__ Ub) {
    const int64_t tile = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    const int64_t row0 = tile * 128 + 32 * (threadIdx.x >> 6);
    if (row0 >= head->n_rows) return;
    __shared__ __attribute__((aligned(16))) char s_x[4][32 * 128];
    const PrepSeg& g = segs[xp_seg_of(segs, head->n_segs, row0)];
    const int64_t l0 = row0 - g.row_base;
    char* sx = s_x[threadIdx.x >> 6];
    // 16-byte loads where every row of the relation starts on 16 bytes
    if (((uintptr_t)g.X & 15) == 0 && (g.ld & 3) == 0)
        xp_codes_rows<true>(g, l0, P, Dp, U, Ub, row0, sx);
    else
        xp_codes_rows<false>(g, l0, P, Dp, U, Ub, row0, sx);
}

// One workgroup of eight waves per 128-row tile of the ordered prepared rows
// (each wave holds 16 rows in registers, lane l elements 4 (l + 64 v) .. +3,
// so the tile is read from memory once): direction d_T (BF16 into Dir, zero
// for an empty or directionless tile), the angular radius A_T with its
// margins (alpha; 4 for a directionless tile: the bound is void; -1 for an
// empty tile) and the largest row error e_T (err).
//
// The angle between a prepared row x and d is taken from the chord,
// 2 asin(|x/|x| - d| / 2), which FP32 evaluates to within ~1e-4 for every
// angle up to 2 pi / 3 (an arccos of the cosine loses up to the square root
// of the cosine's error next to angle 0, where tight tiles live); a larger
// radius is taken as pi.
template <int NV>
__global__ __launch_bounds__(512) void xp_tile_stats(const BatchHead* __restrict__ head,
                                                     const PrepSeg* __restrict__ segs, int Dp,
                                                     uint16_t* __restrict__ Dir,
                                                     float* __restrict__ alpha,
                                                     float* __restrict__ err) {
    constexpr int RW = 16;  // rows per wave
    __shared__ float4 s_c[8][NV * 64];
    __shared__ float s_e[8], s_a[8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t row0 = tile * 128;
    if (row0 >= head->n_rows) return;
    const PrepSeg& g = segs[xp_seg_of(segs, head->n_segs, row0)];
    const int64_t l0 = row0 - g.row_base;
    const int cnt = (int)max<int64_t>(0, min<int64_t>(128, g.rows - l0));
    const int rb = wave * RW;
    const int nr = max(0, min(RW, cnt - rb));
    const int nu = Dp >> 2;  // 8-byte units per row
    // every tile lies inside one relation's prepared copy, padded with zero
    // rows to whole tiles: the wave reads its 16 rows whatever the count
    // (a uniform row address plus a 32-bit lane offset per load)
    typedef __attribute__((address_space(1))) const char* gbyte_ptr;
    const gbyte_ptr X = (gbyte_ptr)((const uint16_t*)g.Xq + (l0 + rb) * Dp);
    uint2 x[RW][NV];
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        const gbyte_ptr xr = X + (size_t)i * (size_t)(2 * Dp);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            // lanes past the row's end read its last unit and drop it
            const uint32_t u = (uint32_t)(lane + 64 * v);
            const uint32_t uc = min(u, (uint32_t)nu - 1u);
            uint64_t w = *(__attribute__((address_space(1))) const uint64_t*)(xr + (uc << 3));
            if (u >= (uint32_t)nu) w = 0ull;
            x[i][v] = make_uint2((uint32_t)w, (uint32_t)(w >> 32));
        }
    }
    // three unpackings of the BF16 pairs: shifts and masks for the column
    // sums, byte permutes for the squares and other byte permutes for the
    // chords; the compiler does not merge them, so every unpacked value dies
    // at once and the rows stay packed
    auto lo = [](uint32_t w) { return __uint_as_float(w << 16); };
    auto hi = [](uint32_t w) { return __uint_as_float(w & 0xffff0000u); };
    auto lo2 = [](uint32_t w) { return __uint_as_float(__builtin_amdgcn_perm(w, 0u, 0x05040c0cu)); };
    auto hi2 = [](uint32_t w) { return __uint_as_float(__builtin_amdgcn_perm(w, 0u, 0x07060c0cu)); };
    // (the chord pass takes its low bytes from the zero operand instead)
    auto lo3 = [](uint32_t w) { return __uint_as_float(__builtin_amdgcn_perm(w, 0u, 0x05040100u)); };
    auto hi3 = [](uint32_t w) { return __uint_as_float(__builtin_amdgcn_perm(w, 0u, 0x07060100u)); };
    // column sums of the wave's rows and the rows' squared norms
    float4 c[NV];
    float nn[RW];
#pragma unroll
    for (int v = 0; v < NV; ++v) c[v] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int i = 0; i < RW; ++i) {
        float s = 0.0f;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            c[v].x += lo(x[i][v].x);
            c[v].y += hi(x[i][v].x);
            c[v].z += lo(x[i][v].y);
            c[v].w += hi(x[i][v].y);
            const float a = lo2(x[i][v].x), b = hi2(x[i][v].x);
            const float e = lo2(x[i][v].y), f = hi2(x[i][v].y);
            s = fmaf(a, a, s);
            s = fmaf(b, b, s);
            s = fmaf(e, e, s);
            s = fmaf(f, f, s);
        }
        nn[i] = s;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) s_c[wave][lane + 64 * v] = c[v];
    const float en = lane < nr ? g.info[l0 + rb + lane].enorm : 0.0f;
    const float ew = wave_max(en);
    if (lane == 0) s_e[wave] = ew;
    __syncthreads();
    // the tile's column sums, added in wave order (every wave gets the same)
    float cc = 0.0f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        float4 t = s_c[0][lane + 64 * v];
#pragma unroll
        for (int w = 1; w < 8; ++w) {
            const float4 q = s_c[w][lane + 64 * v];
            t.x += q.x;
            t.y += q.y;
            t.z += q.z;
            t.w += q.w;
        }
        c[v] = t;
        cc += t.x * t.x + t.y * t.y + t.z * t.z + t.w * t.w;
    }
    const float cn = sqrtf(wave_sum(cc));
    const bool dir = cnt > 0 && cn > 1e-3f * (float)cnt;
    const float ic = dir ? 1.0f / cn : 0.0f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        c[v].x *= ic;
        c[v].y *= ic;
        c[v].z *= ic;
        c[v].w *= ic;
    }
    // largest angle between a prepared row of the wave and the direction
    float amax = 0.0f;
    if (dir) {
        const float nt = xp_wave_sum16(nn);  // lane l: row (l >> 2) & 15
        float ch[RW];
#pragma unroll
        for (int i = 0; i < RW; ++i) {
            const float n_i = __shfl(nt, 4 * i, 64);
            const float inv = n_i > 0.0f ? rsqrtf(n_i) : 0.0f;
            float s = 0.0f;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const float a = fmaf(lo3(x[i][v].x), inv, -c[v].x);
                const float b = fmaf(hi3(x[i][v].x), inv, -c[v].y);
                const float e = fmaf(lo3(x[i][v].y), inv, -c[v].z);
                const float f = fmaf(hi3(x[i][v].y), inv, -c[v].w);
                s = fmaf(a, a, s);
                s = fmaf(b, b, s);
                s = fmaf(e, e, s);
                s = fmaf(f, f, s);
            }
            ch[i] = s;
        }
        const float ct = xp_wave_sum16(ch);
        const int i = (lane >> 2) & 15;
        // zero rows (similarity 0 with every row) and rows past the tile's
        // end do not count
        if (i < nr && nt > 0.0f) {
            const float chord = sqrtf(ct);
            amax = chord <= 1.7320508f ? 2.0f * asinf(0.5f * chord) : 3.14159274f;
        }
        amax = wave_max(amax);
    }
    if (lane == 0) s_a[wave] = amax;
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int u = lane + 64 * v;
            if (u < nu) {
                uint2 b;
                b.x = (uint32_t)f32_to_bf16_rne(c[v].x) | ((uint32_t)f32_to_bf16_rne(c[v].y) << 16);
                b.y = (uint32_t)f32_to_bf16_rne(c[v].z) | ((uint32_t)f32_to_bf16_rne(c[v].w) << 16);
                ((uint2*)(Dir + tile * Dp))[u] = b;
            }
        }
        if (lane == 0) {
            float em = 0.0f, am = 0.0f;
            for (int w = 0; w < 8; ++w) {
                em = fmaxf(em, s_e[w]);
                am = fmaxf(am, s_a[w]);
            }
            // rows are the exact unit rows up to e: quantisation error norm
            // plus the FP32 normalisation (relative (d + 8) 2^-24, counted
            // 1.5 times)
            const float e = em + 1.5f * (float)(g.dim + 8) * 5.9604645e-8f + 1e-6f;
            err[tile] = e;
            float a;
            if (cnt == 0) a = -1.0f;
            else if (!dir) a = 4.0f;
            else a = am + 1.1f * e + 1e-3f;
            alpha[tile] = a;
        }
    }
}

// Tile-to-rows maxima (as the prefilter's pf_sidemax, in the original
// space): one item multiplies the directions of 128 tiles of one side by
// the 128 prepared rows of one tile of the other side (K = Dp) and keeps
// the row maxima.
__global__ __launch_bounds__(256) void xp_sidemax(const BatchHead* __restrict__ head,
                                                  const BatchJob* __restrict__ jobs, int Dp,
                                                  const uint16_t* __restrict__ Dir,
                                                  float* __restrict__ M1,
                                                  float* __restrict__ M2) {
    constexpr int BM = 128, BN = 128, WM = 2, WN = 2;
    typedef TileGeom<BM, BN, WM, WN> TG;
    EJ_TILE_SMEM(BM, BN, WM * WN, sm);
    __shared__ float s_v[WN][BM];
    const int64_t item = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    if (item >= head->n_side) return;
    const int jb = xp_job_of(jobs, head->n_jobs, item, true);
    const BatchJob& J = jobs[jb];
    int64_t local = item - J.side_base;
    const int64_t n0 = (int64_t)((J.tiles_m + 127) / 128) * J.tiles_n;
    const bool side0 = local < n0;
    int ag, b;
    int64_t a_first, n_a;
    const char* rows;
    if (side0) {  // R tile directions x S tile rows
        ag = (int)(local / J.tiles_n);
        b = (int)(local % J.tiles_n);
        a_first = J.rtile0 + (int64_t)ag * 128;
        n_a = J.tiles_m;
        rows = J.B;
    } else {      // S tile directions x R tile rows
        local -= n0;
        ag = (int)(local / J.tiles_m);
        b = (int)(local % J.tiles_m);
        a_first = J.stile0 + (int64_t)ag * 128;
        n_a = J.tiles_n;
        rows = J.A;
    }
    v16f acc[TG::FM][TG::FN];
    tile_mainloop<P_BF16, BM, BN, WM, WN>(sm, (const char*)(Dir + a_first * Dp), rows, nullptr,
                                          nullptr, Dp * 2, 0, b, acc);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / WN, wn = wave % WN, h = lane >> 5, r32 = lane & 31;
    // rows past the end of the relation are zero rows of the padded copy:
    // a product 0 never raises a maximum above the real rows' only when some
    // real row is larger, so they are left out explicitly
    const int64_t n_rows_b = side0 ? J.nS : J.nR;
#pragma unroll
    for (int i = 0; i < TG::FM; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            float v = -2.0f;
#pragma unroll
            for (int j = 0; j < TG::FN; ++j) {
                const int64_t col = (int64_t)b * BN + wn * TG::WTN + j * 32 + r32;
                if (col < n_rows_b) v = fmaxf(v, acc[i][j][e]);
            }
#pragma unroll
            for (int o = 16; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
            if (r32 == 0) s_v[wn][wm * TG::WTM + i * 32 + 8 * (e >> 2) + 4 * h + (e & 3)] = v;
        }
    __syncthreads();
    if (threadIdx.x < BM) {
        const int t = threadIdx.x;
        const int64_t a = (int64_t)ag * 128 + t;
        if (a < n_a) {
            const float v = fmaxf(s_v[0][t], s_v[1][t]);
            if (side0) M1[J.tile_base + a * J.tiles_n + b] = v;
            else M2[J.tile_base + (int64_t)b * J.tiles_n + a] = v;
        }
    }
}

__device__ __forceinline__ float xp_rows_bound(float m, float e_other, float a) {
    // m: the computed maximum of d . x over the other tile's rows; raised by
    // the BF16 rounding of d (2^-9, counted twice), the rows' error norm and
    // the FP32 accumulation, it bounds d . s/|s| for every exact row s
    const float mu = fminf(1.0f, m + 0.0078125f + 1.1f * e_other + 1e-4f);
    const float gap = acosf(fmaxf(-1.0f, mu)) - a - 1e-3f;
    return gap > 0.0f ? cosf(gap) + 1e-5f : 1.0f + 1e-5f;
}

// Every tile pair of every job: keep it unless the smaller tile-to-rows bound
// lies below theta.  Output as pf_bounds: a compacted work list, or a flag
// per tile pair for the panel form's chunks.
__global__ __launch_bounds__(256) void xp_bounds(const BatchHead* __restrict__ head,
                                                 const BatchJob* __restrict__ jobs,
                                                 const float* __restrict__ alpha,
                                                 const float* __restrict__ err,
                                                 const float* __restrict__ M1,
                                                 const float* __restrict__ M2,
                                                 int64_t* __restrict__ work,
                                                 unsigned long long* __restrict__ n_work,
                                                 uint8_t* __restrict__ keep_flags) {
    const int lane = threadIdx.x & 63;
    const int64_t total = head->n_tiles;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63); base < total;
         base += (int64_t)gridDim.x * blockDim.x) {
        const int64_t item = base + lane;
        bool keep = false;
        int64_t packed = 0;
        if (item < total) {
            const int jb = xp_job_of(jobs, head->n_jobs, item, false);
            const BatchJob& J = jobs[jb];
            const int64_t local = item - J.tile_base;
            const int tm = (int)(local / J.tiles_n), tn = (int)(local % J.tiles_n);
            const int64_t a = J.rtile0 + tm, b = J.stile0 + tn;
            const float aa = alpha[a], ab = alpha[b];
            if (aa >= 0.0f && ab >= 0.0f) {
                float bound = 1.0f + 1e-5f;
                if (aa < 3.5f) bound = fminf(bound, xp_rows_bound(M1[item], err[b], aa));
                if (ab < 3.5f) bound = fminf(bound, xp_rows_bound(M2[item], err[a], ab));
                // theta <= 0: a zero row's pairs (similarity 0) match, and
                // the bound does not cover them; such jobs are not pruned
                keep = J.theta <= 0.0 || (double)bound >= J.theta;
                packed = ((int64_t)jb << 48) | ((int64_t)tm << 24) | (int64_t)tn;
            }
        }
        if (keep_flags) {
            if (item < total) keep_flags[item] = keep ? 1 : 0;
            continue;
        }
        const uint64_t m = __ballot(keep);
        if (m) {
            const int leader = __ffsll((unsigned long long)m) - 1;
            unsigned long long b0 = 0;
            if (lane == leader) b0 = atomicAdd(n_work, (unsigned long long)__popcll(m));
            const uint32_t blo = __shfl((uint32_t)b0, leader, 64);
            const uint32_t bhi = __shfl((uint32_t)(b0 >> 32), leader, 64);
            const unsigned long long bb = ((unsigned long long)bhi << 32) | blo;
            if (keep) work[bb + lanes_below(m)] = packed;
        }
    }
}

hipError_t launch_xp_codes(const BatchHead* head, const PrepSeg* segs, int64_t n_rows, int dim,
                           int Dp, uint16_t* P, float* U, uint16_t* Ub, hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    if (Dp > 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xp_proj, dim3(64), dim3(256), 0, st, dim, Dp, P);
    const int64_t tiles = n_rows / 128;
    const int64_t gx = std::min<int64_t>(tiles, 65536), gy = (tiles + gx - 1) / gx;
    hipLaunchKernelGGL(xp_codes_raw, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, head,
                       segs, (const uint16_t*)P, Dp, U, Ub);
    return hipGetLastError();
}

hipError_t launch_xp_tiles(const BatchHead* head, const PrepSeg* segs, const BatchJob* jobs,
                           int64_t n_rows, int Dp, uint16_t* Dir, float* alpha, float* err,
                           float* M1, float* M2, int64_t n_side, int64_t* work,
                           unsigned long long* n_work, int64_t n_tiles, uint8_t* keep,
                           hipStream_t st) {
    if (n_rows <= 0) return hipSuccess;
    if (Dp > 1024 || (Dp & 3)) return hipErrorInvalidValue;
    const int64_t tiles = n_rows / 128;
    const dim3 tg((unsigned)tiles), tb(512);
    switch ((Dp + 255) / 256) {
        case 1: hipLaunchKernelGGL(xp_tile_stats<1>, tg, tb, 0, st, head, segs, Dp, Dir, alpha, err); break;
        case 2: hipLaunchKernelGGL(xp_tile_stats<2>, tg, tb, 0, st, head, segs, Dp, Dir, alpha, err); break;
        case 3: hipLaunchKernelGGL(xp_tile_stats<3>, tg, tb, 0, st, head, segs, Dp, Dir, alpha, err); break;
        default: hipLaunchKernelGGL(xp_tile_stats<4>, tg, tb, 0, st, head, segs, Dp, Dir, alpha, err); break;
    }
    if (n_side > 0) {
        const int64_t gx = std::min<int64_t>(n_side, 65536), gy = (n_side + gx - 1) / gx;
        hipLaunchKernelGGL(xp_sidemax, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, head,
                           jobs, Dp, (const uint16_t*)Dir, M1, M2);
    }
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n_tiles + 255) / 256, 8192));
    hipLaunchKernelGGL(xp_bounds, dim3((unsigned)blocks), dim3(256), 0, st, head, jobs,
                       (const float*)alpha, (const float*)err, (const float*)M1,
                       (const float*)M2, work, n_work, keep);
    return hipGetLastError();
}

}  // namespace ej
