// launch.hpp -- host-side launch wrappers shared between the kernel files and
// the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ej {

struct RowInfo;
struct Pair;

// Tile shapes of the threshold kernel (ids are part of the ABI's tile names).
struct TileDesc {
    int id;
    int prec;   // Prec
    int bm, bn; // output tile
    int bk;     // elements per K step (128 bytes)
    const char* name;
};
int tile_count();                 // number of real tiles (ids 1..count)
const TileDesc* tile_get(int id); // nullptr if unknown

hipError_t launch_zero_header(unsigned long long* hdr, hipStream_t st);

// sel (may be null): output row i < rows is input row sel[i] of a relation
// of n_src rows (ids strictly ascending; violations raise F_BADSEL)
hipError_t launch_prep(int prec, const float* X, int64_t rows, int dim, int64_t ld, void* Xq,
                       int Kp, int64_t rows_pad, RowInfo* info, unsigned long long* hdr,
                       int enorm_slot, hipStream_t st, const int32_t* sel = nullptr,
                       int64_t n_src = 0);

struct ThresholdArgs {
    const void* A;   // normalised R copy, rows_pad_r x Kp
    const void* B;   // normalised S copy, rows_pad_s x Kp
    const RowInfo* info_r;
    const RowInfo* info_s;
    int Kp;
    int64_t nR, nS;
    float lo, hi;    // approximate-score band edges (rounded outward)
    // when set: the edges measured on the device (lohi[0], lohi[1] as float
    // bits, written by launch_band_edges after prep) replace lo, hi
    const unsigned long long* lohi = nullptr;
    Pair* out;
    int64_t capacity;
    int2* band;
    int64_t band_cap;
    unsigned long long* hdr;
    int kg_last;     // k-groups of the last K slice that hold data
};
hipError_t launch_threshold(int tile_id, const ThresholdArgs& a, hipStream_t st);
// the nested-loop comparator (FP32, rows of up to 1024 elements): one pair
// per wavefront, no tiling; never chosen by the planner or the tuner
constexpr int kTileNlj = 23;
hipError_t launch_threshold_nlj(const ThresholdArgs& a, hipStream_t st);
// form 0: one workgroup per CU, 1: two workgroups per CU, 2: two 32-row
// blocks per wave (BF16 / FP8 rows of 3 to 6 K slices)
// Designed and actual resident workgroups per CU of the panel kernel that a
// threshold join of this precision, form (0 one workgroup, 1 two workgroups,
// 2 two row blocks per wave) and padded depth Kp would launch; no launch.
struct PanelQuery {
    int designed, resident, waves;
};
hipError_t panel_query(int prec, int form, int Kp, PanelQuery* q);
hipError_t launch_threshold_panel(int prec, int form, const ThresholdArgs& a,
                                  hipStream_t st);

// top-k candidate sweep (panel kernel with the candidate epilogue)
struct CandArgs {
    const void* A;
    const void* B;
    const RowInfo* info_r;
    const RowInfo* info_s;
    int Kp;
    int64_t nR, nS;
    unsigned long long* hdr;  // floor read from H_TOPK_F
    int* cnt;                 // per padded R row
    int2* cand;               // per padded R row, Kc slots
    int Kc;
    // tile form only: A holds gathered rows, row gi standing for R row
    // row_map[gi] (its cnt / cand entries) swept with floor floors[gi]
    const int* row_map = nullptr;
    const float* floors = nullptr;
};
// register-panel form: returns hipErrorInvalidValue for row depths without
// a panel form (then the tile form below takes any depth; its per-row
// counters must be zero first)
hipError_t launch_topk_candidates(int prec, const CandArgs& a, hipStream_t st);
bool topk_panel_depth(int prec, int kpb);
hipError_t launch_topk_candidates_tile(int prec, const CandArgs& a, hipStream_t st);

// exact top-k: pilot + floor, per-row finalize and fallback
struct TopkArgs {
    const float* R;
    int64_t ldR;
    const float* S;
    int64_t ldS;
    int dim;
    int64_t nR, nS;
    const double* nr64;       // canonical FP64 squared norms
    const double* ns64;
    const RowInfo* info_r;
    const int* cnt;
    const int2* cand;
    int Kc;
    int k;
    double fp32_terms;        // FP32 part of the error bound
    unsigned long long* hdr;
    int* fb_rows;             // rows sent to the exact fallback
    int* pilot_rows;
    double* pilot_kth;
    int* keys;                // finalize order: best candidate per row
    int* counts;              // nS + 1 bucket counts / offsets
    int* order;               // rows grouped by best candidate
    double* part_v;           // per-range partial lists of the exact scans
    int* part_j;
    int part_rows;            // list entries one exact-scan batch holds
    int n_pilot;
    bool all_columns;         // |S| <= Kc: every column is a candidate
    int32_t* out_idx;
    float* out_score;
    double min_sim = -INFINITY;  // only columns with sim64 >= min_sim count
};
hipError_t launch_fill_int(int* p, int64_t n, int v, hipStream_t st);
hipError_t launch_norms64(const float* X, int64_t rows, int dim, int64_t ld, double* out,
                          hipStream_t st);
hipError_t launch_topk_pilot(const TopkArgs& a, hipStream_t st);
hipError_t launch_topk_finalize(const TopkArgs& a, hipStream_t st);
hipError_t launch_topk_fallback(const TopkArgs& a, int64_t n_fb, hipStream_t st);
// refinement of overflowed rows (rows[0 .. n): the first finalize's failures):
// per-row floors (+inf for rows that did not overflow) and counters reset
hipError_t launch_topk_refine_floor(const TopkArgs& a, const int* rows, int64_t n, float* floors,
                                    hipStream_t st);
hipError_t launch_topk_finalize_rows(const TopkArgs& a, const int* order, int64_t n,
                                     const float* floors, hipStream_t st);
hipError_t launch_gather_prepared(const void* X, int row_bytes, const int* rows, int64_t n,
                                  int64_t n_pad, void* dst, hipStream_t st);

// sel_r / sel_s (may be null): band entries hold selection positions; the
// FP64 rule reads the caller's rows sel[position]
hipError_t launch_rescore_band(const float* R, int64_t ldR, const float* S, int64_t ldS, int dim,
                               const int2* band, int64_t band_cap, double theta, Pair* out,
                               int64_t capacity, unsigned long long* hdr, hipStream_t st,
                               const int32_t* sel_r = nullptr, const int32_t* sel_s = nullptr);
// Rewrite the first min(count, capacity) emitted pairs from selection
// positions to the caller's row ids (a null selection keeps its side).
hipError_t launch_map_pairs(Pair* out, int64_t capacity, const unsigned long long* hdr,
                            const int32_t* sel_r, const int32_t* sel_s, hipStream_t st);
// Copy the selected rows (ids strictly ascending, in [0, n_src)) into a
// compact row-major buffer (ld = dim); violations raise F_BADSEL.
hipError_t launch_gather_rows(const float* X, int64_t ld, int dim, const int32_t* sel, int64_t n,
                              int64_t n_src, float* dst, unsigned long long* hdr, hipStream_t st);
// Top-k output indices from selection positions (n_sel of them) to the
// caller's S ids; skipped after a failed input check (flags in hdr).
hipError_t launch_map_topk(int32_t* idx, int64_t n, const int32_t* sel_s, int64_t n_sel,
                           const unsigned long long* hdr, hipStream_t st);
// sigma(lo <= col[i] < hi) as a strictly ascending id list: counts per
// block, a scan, then a stable write; n_sel is a device int64.
size_t select_range_workspace();
hipError_t launch_select_range(const float* col, int64_t n, float lo, float hi, int32_t* ids,
                               int64_t* n_sel, void* ws, hipStream_t st);

// Band edges from the measured quantisation error norms (hdr[H_ENORM_R/S]):
// delta = eR (1 + eS) + eS + f (1 + eR)(1 + eS), at most `rigorous`; writes
// round_down(theta - delta), round_up(theta + delta) to hdr[H_LO], hdr[H_HI]
// and delta to hdr[H_BAND_W]; all64: the upper edge is +inf (every candidate
// is rescored).
hipError_t launch_band_edges(unsigned long long* hdr, double theta, double fp32_terms,
                             double rigorous, bool alias, bool all64, hipStream_t st);
hipError_t launch_copy_count(const unsigned long long* hdr, int64_t band_cap, int64_t* dst,
                             hipStream_t st);

}  // namespace ej

// ---- batched threshold join (batch.hpp holds the table layout) ----
namespace ej {
struct BatchHead;
struct BatchJob;
struct PrepSeg;
bool batch_has_tile(int tile_id);  // the tile has a persistent batch form
// batch form on BF16 register panels (tile 19): the K depths it takes, its
// resident workgroups per CU, its launch
bool batch_panel_depth(int kpb);
int batch_panel_occupancy();
hipError_t launch_batch_panel(const BatchHead* head, const BatchJob* jobs,
                              unsigned long long* bctr, int grid, bool worklist, hipStream_t st);
// the same form in two workgroups per CU (tile 22)
int batch_panel2_occupancy();
hipError_t launch_batch_panel2(const BatchHead* head, const BatchJob* jobs,
                               unsigned long long* bctr, int grid, bool worklist, hipStream_t st);
int batch_occupancy(int tile_id);  // resident workgroups per CU, 0: no batch form
hipError_t launch_batch_zero(const BatchHead* head, unsigned long long* bctr, hipStream_t st);
// after prep: measured band edges of the jobs that use one (job table on the device)
hipError_t launch_batch_band_edges(const BatchHead* head, BatchJob* jobs, hipStream_t st);
// kp_max: the deepest padded row of the batch (sizes the per-lane registers;
// deeper rows still take the unregistered form); the grid is the device's
// resident workgroups of the kernel
hipError_t launch_batch_prep(int prec, int kp_max, const BatchHead* head, const PrepSeg* segs,
                             bool ordered, hipStream_t st);
// the grid launch_batch_prep uses (its device query runs once per kernel:
// call this before a stream capture so that none runs inside it)
int batch_prep_query(int prec, int kp_max);
// worklist: the items come from the prefilter's work list (head->work)
hipError_t launch_batch_tile(int tile_id, const BatchHead* head, const BatchJob* jobs,
                             unsigned long long* bctr, int grid, hipStream_t st,
                             bool worklist = false);
hipError_t launch_batch_rescore(const BatchHead* head, const BatchJob* jobs,
                                const unsigned long long* bctr, int grid, hipStream_t st);
hipError_t launch_batch_counts(const BatchHead* head, const BatchJob* jobs,
                               const unsigned long long* bctr, hipStream_t st);

// prefilter training data
struct TrainJob;
hipError_t launch_train_rows(const TrainJob* jobs, const int4* samples, int B, int Dp,
                             uint16_t* pool, RowInfo* info, unsigned long long* hdr,
                             hipStream_t st);
hipError_t launch_train_targets(const TrainJob* jobs, const int4* samples, int B, float* t,
                                hipStream_t st);
}  // namespace ej
