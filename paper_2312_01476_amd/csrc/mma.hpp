// mma.hpp -- one matrix-core step per operand precision, and the LDS slice
// layout shared by the contraction kernels.
#pragma once

#include "common.hpp"

namespace ej {

// ---------------------------------------------------------------------------
// matrix-core step per precision
//
// Every operand row is stored in LDS as 128-byte K slices made of eight
// 16-byte chunks.  For one MFMA a lane reads the chunk(s) of its row given by
// its lane half; the A and B operands are read with the same chunk schedule,
// so the pairing of k indices inside the instruction is consistent whatever
// order the hardware sums them in.
// ---------------------------------------------------------------------------
template <int PREC>
struct Mma;

template <>
struct Mma<P_FP32> {
    // v_mfma_f32_32x32x2_f32: per lane one float of A and of B.
    // A k-group is two chunks (half h reads chunk 2g+h) = 4 MFMAs.
    static constexpr int GROUPS = 4;     // k-groups per 128-byte slice
    static constexpr int CPL = 1;        // chunks per lane per group
    static constexpr int SUB = 4;        // matrix-core steps per fragment pair
    typedef v4i Frag;
    static __device__ __forceinline__ int chunk(int g, int h, int c) { return 2 * g + h; }
    static __device__ __forceinline__ void mma(const Frag& a, const Frag& b, v16f& acc, int, int) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__int_as_float(a[j]), __int_as_float(b[j]),
                                                       acc, 0, 0, 0);
    }
    // step j only: callers interleave the steps of independent accumulators
    static __device__ __forceinline__ void mma_sub(const Frag& a, const Frag& b, v16f& acc, int,
                                                   int, int j) {
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(__int_as_float(a[j]), __int_as_float(b[j]), acc,
                                                   0, 0, 0);
    }
};

template <>
struct Mma<P_BF16> {
    // v_mfma_f32_32x32x16_bf16: per lane 8 bf16 (one chunk) of A and of B.
    static constexpr int GROUPS = 4;
    static constexpr int CPL = 1;
    static constexpr int SUB = 1;
    typedef v4i Frag;
    static __device__ __forceinline__ int chunk(int g, int h, int c) { return 2 * g + h; }
    static __device__ __forceinline__ void mma(const Frag& a, const Frag& b, v16f& acc, int, int) {
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                      __builtin_bit_cast(v8bf, b), acc, 0, 0, 0);
    }
    static __device__ __forceinline__ void mma_sub(const Frag& a, const Frag& b, v16f& acc, int sa,
                                                   int sb, int) {
        mma(a, b, acc, sa, sb);
    }
};

template <>
struct Mma<P_FP8> {
    // v_mfma_scale_f32_32x32x64_f8f6f4 with e4m3 operands: per lane 32
    // bytes (two chunks) of A and of B, and one E8M0 scale per lane that
    // covers the lane's 32 k values.  The scale of a row is 2^-p, the
    // inverse of the power of two the prep kernel applied before rounding,
    // so the accumulator is the dot of the normalised rows directly.
    static constexpr int GROUPS = 2;
    static constexpr int CPL = 2;
    static constexpr int SUB = 1;
    typedef v8i Frag;
    static __device__ __forceinline__ int chunk(int g, int h, int c) { return 4 * g + 2 * h + c; }
    static __device__ __forceinline__ void mma(const Frag& a, const Frag& b, v16f& acc, int sa,
                                               int sb) {
        acc = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, acc, 0, 0, 0, sa, 0, sb);
    }
    static __device__ __forceinline__ void mma_sub(const Frag& a, const Frag& b, v16f& acc, int sa,
                                                   int sb, int) {
        mma(a, b, acc, sa, sb);
    }
};

// byte offset of 16-byte chunk c of LDS row `row`.  The LDS has 64 banks of
// 4 bytes, i.e. 16 groups of 16 bytes, and a 128-byte row covers 8 of them;
// XOR-ing the chunk index with (row / 2) mod 8 puts the same chunk of 16
// consecutive rows into 16 different bank groups, so a ds_read_b128 of 16
// lanes (16 rows, one chunk) is conflict free, and so are the row-wise writes.
__device__ __forceinline__ int lds_off(int row, int c) {
    return row * 128 + ((c ^ ((row >> 1) & 7)) << 4);
}

}  // namespace ej
