// plan.hpp -- host-side planning helpers shared by the C ABI sources:
// padded sizes, the rigorous band, outward rounding of the band edges,
// argument checks and the planner's default tile.
#pragma once

#include "../../include/ejoin.h"

#include <math.h>
#include <string.h>

#include <algorithm>

#include "common.hpp"
#include "launch.hpp"

namespace ej {
namespace plan {


constexpr double kU32 = 5.9604644775390625e-08;  // 2^-24, FP32 unit roundoff

inline int elem_bytes(int prec) { return prec == P_FP32 ? 4 : prec == P_BF16 ? 2 : 1; }

// contraction depth: dim rounded up to a whole 128-byte slice
inline int padded_k(int prec, int dim) {
    const int per = 128 / elem_bytes(prec);
    return ((dim + per - 1) / per) * per;
}

// k-groups (elements per matrix-core step group: FP32 8, BF16 16, FP8 64)
// of the last 128-byte K slice that hold data
inline int last_slice_groups(int prec, int dim) {
    const int per = 128 / elem_bytes(prec);
    const int gsz = prec == P_FP32 ? 8 : prec == P_BF16 ? 16 : 64;
    const int Kp = padded_k(prec, dim);
    const int rem = dim - (Kp - per);  // elements of the last slice, 1..per
    return (rem + gsz - 1) / gsz;
}

inline int64_t padded_rows(int64_t rows) { return ((rows + 255) / 256) * 256; }

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Rigorous bound on |approximate score - sim64| for unit-norm operands.
//  * normalisation in FP32 (norm, sqrt, divide, scale): relative error per
//    operand below gamma_d + 4u;
//  * FP32 accumulation over Kp terms: gamma_Kp times sum |r_k s_k| <= 1;
//  * BF16 rounding of both operands: 2 u_b + u_b^2 with u_b = 2^-8;
//  * FP8 e4m3: |e_r| + |e_s| + |e_r||e_s| from the quantisation error norms,
//    worst case |e| <= 2^-4 + sqrt(d) 2^-10 / 224 (power-of-two scale puts
//    the largest element in [224, 448]);
//  * 1e-5 of slack absorbs the FP64 rounding of sim64 itself (~1e-15) and
//    second-order terms.
// The FP32 terms are counted four times over to stay valid if the matrix
// cores round each step toward zero rather than to nearest.
inline double band_fp32_terms(int Kp) { return 1e-5 + 4.04 * (double)(Kp + 8) * kU32; }

inline double band_rigorous(int prec, int dim) {
    if (dim < 1) return -1.0;
    const int Kp = padded_k(prec, dim);
    const double f = band_fp32_terms(Kp);
    if (prec == P_FP32) return f;
    if (prec == P_BF16) return 0.0078125 + 1.52587890625e-05 + f;
    const double E = 0.0625 * 1.001 + sqrt((double)dim) * (1.0 / 1024.0) / 224.0 + 1e-7;
    return 2.0 * E + E * E + f * (1.0 + E) * (1.0 + E);
}

inline float round_down_f(double x) {
    float f = (float)x;
    if ((double)f > x) f = nextafterf(f, -INFINITY);
    return f;
}
inline float round_up_f(double x) {
    float f = (float)x;
    if ((double)f < x) f = nextafterf(f, INFINITY);
    return f;
}

inline bool rel_ok(const ejoin_rel* X) {
    if (!X) return false;
    if (X->rows < 0 || X->rows >= 0x7fffffffLL) return false;
    if (X->dim < 1 || X->ld < X->dim) return false;
    if (X->rows > 0 && X->data == nullptr) return false;
    return true;
}

// planner default: the register-resident panel kernel for narrow formats
// whose rows fit it (up to 768 bytes of K), else the LDS tile kernel
// Row depths (K bytes) a panel tile takes: up to 768; the one-workgroup BF16
// and the FP32 panels (tiles 12, 20, 21) also 1024, 1152, 1280 and 1536.
inline bool panel_fits(int tile, int kpb) {
    if (tile == 24 || tile == 25) return kpb >= 384 && kpb <= 768;  // 3 to 6 K slices
    if (kpb <= 768) return true;
    return (tile == 12 || tile == 14 || tile == 20 || tile == 21) &&
           (kpb == 1024 || kpb == 1152 || kpb == 1280 || kpb == 1536);
}

inline int default_tile(int prec, int Kp) {
    // FP32: register panels in two workgroups per CU for rows of 8, 9 or 10
    // K slices (225-320 dims), else the 128 x 128 tile
    if (prec == P_FP32) return (Kp == 256 || Kp == 288 || Kp == 320) ? 21 : 1;
    // register panels: BF16 rows of up to four K slices of 128 bytes in two
    // workgroups of four waves per CU, of five or six in one workgroup of
    // eight waves (both on direct-load rings where the slices divide evenly)
    if (Kp * elem_bytes(prec) <= 768)
        return prec == P_FP8 ? 13 : (Kp * elem_bytes(prec) >= 640 ? 12 : 14);
    // deeper BF16 rows (8, 9, 10 or 12 K slices): two workgroups per CU,
    // with 64-column S tiles (32-column at 12 slices)
    if (prec == P_BF16 && panel_fits(14, Kp * 2)) return 14;
    return prec == P_BF16 ? 3 : 5;
}

// Tile recorded by a tuner for (batch or single, prec, dim, |R| x |S|
// summed over jobs); 0 when it holds nothing for this precision and depth.
int tuner_pick(const ejoin_tuner* t, int batch, int prec, int dim, double pairs);

inline void opts_init(ejoin_opts* o) {
    memset(o, 0, sizeof(*o));
    o->prec = EJOIN_FP32;
    o->band = -1.0;
}

inline ejoin_opts opts_or_default(const ejoin_opts* o) {
    ejoin_opts d;
    opts_init(&d);
    return o ? *o : d;
}

}  // namespace plan
}  // namespace ej

#define HIP_TRY(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return EJOIN_E_HIP;  \
    } while (0)

