// prefilter.hpp -- launch wrappers of the approximate (prefiltered) batch
// mode (prefilter.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp.hpp"

namespace ej {

struct BatchHead;
struct BatchJob;
struct PrepSeg;

constexpr int32_t PF_PAD_KEY = 4095;        // ordering key of padding rows (sorts last)
constexpr int PF_MAX_ANCHORS = 4094;        // anchors of the ordering key (labels < 4095)

// codes U (flat rows x 64, and a BF16 copy Ub) of every prepared row
hipError_t launch_pf_codes(const BatchHead* head, const PrepSeg* segs, int64_t n_rows,
                           const MlpDev& m, uint16_t* Hb, float* U, uint16_t* Ub,
                           hipStream_t st);
// exact pruning (prune.hip): normalised codes (U, and the BF16 copy Ub) of
// the input rows under a fixed +-1 projection (P: 64 x Dp BF16 scratch),
// then per-tile directions / angular radii in the original space,
// tile-to-rows maxima and the kept tile pairs (outputs as launch_pf_tiles;
// err: tiles floats)
hipError_t launch_xp_codes(const BatchHead* head, const PrepSeg* segs, int64_t n_rows, int dim,
                           int Dp, uint16_t* P, float* U, uint16_t* Ub, hipStream_t st);
hipError_t launch_xp_tiles(const BatchHead* head, const PrepSeg* segs, const BatchJob* jobs,
                           int64_t n_rows, int Dp, uint16_t* Dir, float* alpha, float* err,
                           float* M1, float* M2, int64_t n_side, int64_t* work,
                           unsigned long long* n_work, int64_t n_tiles, uint8_t* keep,
                           hipStream_t st);
// ordering keys: K anchors = codes of the flat rows anchor_idx, leader
// labels at cosine tau, key = label of the nearest anchor
// 64-bit words per anchor row of the anchors' pair-test bit matrix (abits:
// K x pf_anchor_words(K) words)
inline int pf_anchor_words(int K) { return (K + 63) / 64; }
hipError_t launch_pf_keys(const BatchHead* head, const PrepSeg* segs, int64_t n_rows,
                          const float* U, const uint16_t* Ub, const int64_t* anchor_idx, int K,
                          float tau, float* Af, uint16_t* Ab, uint64_t* abits, int32_t* label,
                          int32_t* key, hipStream_t st);
// stable order of every relation's rows by key: perm_a[row_base + i] is the
// local row at ordered position i
hipError_t launch_pf_sort(const BatchHead* head, const PrepSeg* segs, int n_segs, int64_t n_rows,
                          const int32_t* key, int32_t* perm_a, int32_t* perm_b, int32_t* hist,
                          int32_t* offs, hipStream_t st);
// 128-row tile statistics of the ordered rows and the surviving tile pairs:
// a compacted (job, tm, tn) work list, or with `keep` one flag per tile pair
// (flat tile order) for launch_pf_chunks
hipError_t launch_pf_tiles(const BatchHead* head, const PrepSeg* segs, const BatchJob* jobs,
                           int64_t n_rows, const float* U, const int32_t* perm, float* C,
                           float* rho, float* cnorm, float* alpha, uint16_t* Up, uint16_t* Dir,
                           float* M1, float* M2, int64_t n_side, float eps, int64_t* work,
                           unsigned long long* n_work, int64_t n_tiles, uint8_t* keep,
                           hipStream_t st);
// panel form: the (job, panel, S chunk) items with at least one kept tile,
// packed job << 48 | tm << 24 | first tn, each with its mask of kept tiles;
// n_kept counts the kept tile pairs
hipError_t launch_pf_chunks(const BatchHead* head, const BatchJob* jobs, const uint8_t* keep,
                            int64_t* work, uint32_t* work_mask, unsigned long long* n_work,
                            unsigned long long* n_kept, int64_t n_chunks, hipStream_t st);

}  // namespace ej
