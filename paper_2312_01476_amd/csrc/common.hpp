// common.hpp -- shared device-side definitions of the gfx950 E-join kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ej {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));

enum Prec : int { P_FP32 = 0, P_BF16 = 1, P_FP8 = 2 };

// Workspace header: int64 counters at the start of every workspace.
enum : int {
    H_OUT = 0,        // matching pairs emitted so far (certain + accepted band)
    H_BAND = 1,       // band pairs found (may exceed the band capacity)
    H_FLAGS = 2,      // OR of row flags (non-finite / range)
    H_CERT = 3,       // certain pairs (for the report)
    H_BAND_ACC = 4,   // band pairs accepted by the FP64 rescore
    H_ENORM_R = 5,    // max quantisation error norm over R rows (float bits)
    H_ENORM_S = 6,    // same for S
    H_MISC = 7,
    H_TOPK_F = 8,     // top-k candidate floor (float bits)
    H_TOPK_FB = 9,    // top-k rows sent to the exact fallback
    H_TOPK_EMAX = 10, // top-k: largest per-row error bound (float bits)
    H_LO = 11,        // threshold band edges from the measured error norms (float bits)
    H_HI = 12,
    H_BAND_W = 13,    // the band half-width they come from (double bits)
    H_COUNT = 32      // header size in int64 (256 bytes)
};

enum : uint32_t { F_NONFINITE = 1u, F_RANGE = 2u, F_BADSEL = 4u };  // F_BADSEL: a selection id
                                                                        // out of range or out of order

// Per-row information written by the prep kernel.
struct RowInfo {
    float inv;      // 1 / ||x|| in FP32 (0 for a zero row)
    float qscale;   // power-of-two multiplier applied before FP8 rounding (1 otherwise)
    float enorm;    // || dequantised row - fp32 normalised row ||_2 (0 for FP32)
    uint32_t flags; // F_* bits
};

// Result pair as laid out in the public header.
struct Pair {
    int32_t r;
    int32_t s;
    float score;
};

// ---------------------------------------------------------------------------
// direct-load ring helpers
// ---------------------------------------------------------------------------
// Wait until at most N global memory operations of this wave are in flight
// and all its LDS operations are done (gfx9 s_waitcnt encoding: vmcnt in bits
// 3:0 and 15:14, expcnt 6:4 left at its maximum, lgkmcnt 11:8 = 0).
template <int N>
__device__ __forceinline__ void wait_vmcnt_lgkm0() {
    static_assert(N >= 0 && N < 64, "vmcnt is six bits");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4));
}

// Workgroup barrier without a memory fence: the waits before it are the
// caller's, and direct-load fills in flight stay in flight across it.  The
// signal fences keep the compiler from moving memory accesses across.
__device__ __forceinline__ void bare_barrier() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_barrier();
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// One 16-byte direct global->LDS load per lane: lane l writes the 16 bytes at
// lds + 16 l (`lds` is the same for the whole wave).
__device__ __forceinline__ void lds_fill16(const void* src, char* lds) {
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// ---------------------------------------------------------------------------
// wave-level helpers (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` strictly below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------------------
// rounding to the narrow operand formats (software, round-to-nearest-even)
// ---------------------------------------------------------------------------

// float -> bfloat16 bits, RNE.  Inputs are finite here.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}

// OCP e4m3 (bias 7, 3 mantissa bits, max 448, no infinities): value of the
// nearest representable number (ties to even) for |x| <= 448.
__device__ __forceinline__ float e4m3_round(float x) {
    float a = fabsf(x);
    if (a == 0.0f) return x;
    // spacing of representable numbers around a: 2^(e-3) for normals
    // (e >= -6), 2^-9 in the subnormal range
    int e = ilogbf(a);
    if (e < -6) e = -6;
    float step = ldexpf(1.0f, e - 3);
    float q = rintf(a / step) * step;  // a/step exact (power-of-two divide)
    return copysignf(q, x);
}
// Encode a value already representable in e4m3 (|q| <= 448).
__device__ __forceinline__ uint8_t e4m3_bits(float q) {
    uint32_t sign = (__float_as_uint(q) >> 31) & 1u;
    float a = fabsf(q);
    uint32_t bits;
    if (a == 0.0f) {
        bits = 0;
    } else if (a < 0.015625f) {          // subnormal: a = m * 2^-9, m in 1..7
        bits = (uint32_t)(a * 512.0f);
    } else {
        int e = ilogbf(a);               // -6 .. 8
        uint32_t m = (uint32_t)(ldexpf(a, -e) * 8.0f) - 8u;   // 0..7
        bits = ((uint32_t)(e + 7) << 3) | m;
    }
    return (uint8_t)((sign << 7) | bits);
}

}  // namespace ej
