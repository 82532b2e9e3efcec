// batch.hpp -- device-side job table of the batched threshold join.
//
// A batch is a list of independent threshold joins (each its own R, S,
// theta, output buffer and capacity), run as one pass of four launches:
// batched prep, one persistent contraction kernel whose workgroups pull
// (job, tile) work items from an atomic counter, a batched FP64 rescore of
// the band pairs of every job, and a count copy.  Every launch reads its
// work from this table in device memory and uses a grid size that does not
// depend on the jobs, so a captured graph of the pass can be replayed for
// another batch after only the table has been rewritten.
#pragma once

#include "common.hpp"

namespace ej {

// Panel form of the batch (tiles 19 and 22): S tiles of 128 columns per
// work item.  The prefilter's kept-tile mask of an item is one bit per tile
// (32 bits), and the two-workgroup form widens it to four 32-column tiles per
// bit in a 64-bit mask, so at most 16 tiles per item.
constexpr int kPanelChunkTiles = 16;
static_assert(kPanelChunkTiles * 4 <= 64, "the widened kept-tile mask holds 64 32-column tiles");

// One join of the batch.  Jobs are stored largest first (by tile count), so
// the work items handed out last are the small tiles of small jobs.
struct BatchJob {
    const char* A;             // prepared R rows (padded K)
    const char* B;             // prepared S rows
    const RowInfo* info_r;
    const RowInfo* info_s;
    const float* R;            // caller's float32 rows (FP64 rescore)
    const float* S;
    Pair* out;
    unsigned long long* hdr;   // per-job counters (H_OUT, H_FLAGS, H_BAND_ACC)
    int64_t ldR, ldS;
    int64_t nR, nS;
    int64_t capacity;
    int64_t tile_base;         // first flat work item of this job
    double theta;
    float lo, hi;              // approximate-score band edges
    int32_t tiles_m, tiles_n;
    int32_t Kp_bytes, dim;
    int32_t user;              // index of the job in the caller's array
    int32_t kg_last;           // k-groups of the last K slice that hold data
    int32_t chunk_tiles;       // panel form: S tiles per work item
    // prefilter mode: the prepared rows are in code order; perm maps a
    // prepared row back to the caller's row, rtile0 / stile0 are the flat
    // indices of the first 128-row tiles of R and S
    const int32_t* perm_r;
    const int32_t* perm_s;
    int64_t rtile0, stile0;
    int64_t side_base;         // first item of this job's tile-to-rows bound pass
    int64_t chunk_base;        // prefilter panel form: first (panel, S chunk) item
    // measured band (BF16 / FP8 with the default band): after prep, lo and hi
    // are narrowed on the device from the largest quantisation error norms
    // of the job's rows (hdr[H_ENORM_R / S]); band_f: the FP32 part of the
    // bound, band_rig: the worst case it never exceeds; all64: hi stays +inf
    // (EJOIN_FP64_SCORES: every candidate is rescored)
    double band_f, band_rig;
    int32_t measured, alias, all64, pad2_;
};

// One relation to prepare (R or S of a job; an aliased self-join has one).
struct PrepSeg {
    const float* X;
    void* Xq;
    RowInfo* info;
    unsigned long long* hdr;   // flags go to the owning job's counters
    const int32_t* perm;       // prefilter ordering: prepared row r is input row perm[r] (or null)
    int64_t rows, rows_pad, ld;
    int64_t row_base;          // first flat prep row of this segment
    int32_t dim, Kp;
    int32_t enorm_slot;        // hdr slot of the largest error norm (H_ENORM_R or _S)
    int32_t pad_;
};

struct BatchHead {
    int64_t n_tiles;           // flat work items over all jobs
    int64_t n_rows;            // flat prep rows over all segments
    int64_t band_cap;          // entries of the shared band list
    int4* band;                // {r, s, job, 0}
    int64_t* n_out;            // per caller job (device), or null
    unsigned long long* hdrs;  // n_jobs x H_COUNT counters, contiguous
    int32_t n_jobs, n_segs;
    int32_t pad_[2];
    // prefilter mode: the surviving (job, tm, tn) work items, packed as
    // job << 48 | tm << 24 | tn, and their count (null in the plain mode)
    const int64_t* work;
    const unsigned long long* n_work;
    int64_t n_side;            // items of the tile-to-rows bound pass
    // prefilter panel form: work items are (job, panel, first S tile of a
    // chunk); work_mask[i] has bit b set when S tile tn + b of item i is kept
    const uint32_t* work_mask;
    int64_t n_chunks;          // (panel, S chunk) items over all jobs
};

// Global counters of a batch pass.
enum : int {
    B_ITEM = 0,     // next work item of the persistent kernel
    B_BAND = 1,     // band entries found (may exceed band_cap)
    B_WORK = 2,     // prefilter: surviving work items
    B_KEPT = 3,     // prefilter panel form: surviving tile pairs
    B_COUNT = 32
};

// Prefilter training: the relations and exact outputs of one job, and one
// drawn pair {job, kind, a, b}: kind 1 is output pair a of the job, kind 0
// the pair (row a of R, row b of S).
struct TrainJob {
    const float* R;
    const float* S;
    const Pair* out;
    int64_t ldR, ldS, nR, nS;
    int32_t dim, pad_;
};

// Table image: head, then jobs[max_jobs], then segs[2 * max_jobs].
struct BatchTable {
    const BatchHead* head;
    const BatchJob* jobs;
    const PrepSeg* segs;
};

}  // namespace ej
