/*
 * ejoin.h -- C ABI of the MI355X (gfx950) context-enhanced similarity join.
 *
 * The operator is the E-theta-join of the paper (Section III.C): two relations
 * of embedding vectors R and S are joined on the cosine similarity of their
 * rows (Section III.A, the "Cosine Similarity" equation).  It is evaluated in
 * the tensor-join form of Section IV.C: the |R| x |S| similarity matrix
 * D = R_hat S_hat^T of the L2-normalised rows (cosine = dot of normalised
 * vectors) is computed block by block (the block-matrix decomposition
 * equation) and the predicate is applied to each block as it is produced; D
 * is never materialised, which is the bounded-buffer scheme of Section V.B
 * taken to the size of one MFMA tile.  The result is a list of tuple-offset
 * pairs (Section IV.C, "late materialisation").
 *
 * Conventions for every entry point
 * ---------------------------------
 *  - Pointers are DEVICE pointers unless a comment says "(host)".  The caller
 *    owns every buffer: inputs, outputs and the workspace.  The library never
 *    allocates device memory inside a join call.
 *  - Inputs are row-major float32, ejoin_rel.ld elements between rows
 *    (ld >= dim); only the first dim columns are read.  They must stay valid
 *    until the stream work is complete.
 *  - Canonical similarity.  The exact result is defined with the FP64 rule
 *        sim64(r,s) = dot(r,s) / sqrt(dot(r,r) * dot(s,s))   (0 for a zero row)
 *    with every dot summed sequentially over k = 0..dim-1 in FP64 from the
 *    float32 inputs, one rounding per product and per sum, correctly rounded
 *    sqrt and divide.  A pair matches iff sim64 >= theta.
 *  - Exactness.  The bulk contraction runs in FP32, BF16 or FP8 e4m3 on the
 *    matrix cores; every pair whose approximate score lies within a rigorous
 *    error band of theta is rescored on the GPU with the rule above, so the
 *    returned set is exactly { (i,j) : sim64(r_i,s_j) >= theta } in every
 *    precision.
 *  - Errors are returned, never printed or aborted on.  No global mutable
 *    state (except the scratch array of ejoin_threshold_noalloc): calls with
 *    distinct workspaces may run concurrently.
 *  - Rows with a non-finite element give EJOIN_E_NONFINITE; rows whose L2 norm
 *    is non-zero but outside [2^-100, 2^100] give EJOIN_E_RANGE (rescale such
 *    input; zero rows are fine and have similarity 0 with everything).
 *  - Offsets in results are int32, so |R| and |S| must be < 2^31.
 */
#ifndef EJOIN_H
#define EJOIN_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EJOIN_OK = 0,
    EJOIN_E_INVAL = 1,       /* bad argument (null pointer, dim mismatch, theta not finite, ...) */
    EJOIN_E_OVERFLOW = 2,    /* output capacity too small: *n_out holds the true count */
    EJOIN_E_WORKSPACE = 3,   /* workspace too small: see ejoin_stats.ws_needed / band_needed */
    EJOIN_E_NONFINITE = 4,   /* an input row holds NaN or Inf */
    EJOIN_E_HIP = 5,         /* a HIP runtime call failed */
    EJOIN_E_UNSUPPORTED = 6, /* combination not supported (e.g. dimension too large) */
    EJOIN_E_RANGE = 7        /* a row norm outside [2^-100, 2^100] (and not zero) */
} ejoin_status;

/* Precision of the bulk contraction (the FP64 rescore is always FP64). */
typedef enum {
    EJOIN_FP32 = 0,     /* float32 operands, FP32 MFMA */
    EJOIN_BF16 = 1,     /* bfloat16 operands (RNE), FP32 accumulate */
    EJOIN_FP8_E4M3 = 2  /* OCP e4m3 operands, per-row power-of-two scale, FP32 accumulate */
} ejoin_prec;

/* One relation: rows x dim embedding matrix, row-major, ld elements per row. */
typedef struct {
    const float *data;  /* device */
    int64_t rows;
    int32_t dim;
    int64_t ld;
} ejoin_rel;

/* One result pair: offsets into R and S, and the score (float32 of the FP64
 * rescored value for pairs inside the band, the accumulator otherwise). */
typedef struct {
    int32_t r;
    int32_t s;
    float score;
} ejoin_pair;

/* flags */
#define EJOIN_NO_SYNC   0x1u  /* do not synchronise; n_out is a DEVICE int64 and the status
                                 only covers argument and launch errors.  The device count
                                 is the match count, or minus a status code when the call
                                 failed on the device: -EJOIN_E_WORKSPACE (band list too
                                 small), -EJOIN_E_NONFINITE, -EJOIN_E_RANGE */
#define EJOIN_TIMING    0x2u  /* record per-phase times in ejoin_stats (adds event syncs) */
#define EJOIN_APPROX_PREFILTER 0x4u  /* ejoin_batch: skip the 128 x 128 tile pairs that the
                                        learned prefilter (opts->prefilter) bounds below
                                        theta - opts->prefilter_eps.  Approximate: the result
                                        of each job is a SUBSET of its exact join (every pair
                                        returned is exact); see ejoin_batch. */
#define EJOIN_EXACT_PRUNE 0x10u  /* ejoin_batch: skip the 128 x 128 tile pairs whose every pair is
                                    certified below theta (exact; see ejoin_batch) */
#define EJOIN_TOPK_MIN_SIM 0x8u  /* top-k: only S rows with sim64 >= opts->topk_min_sim count
                                    (the range predicate combined with the top-k condition);
                                    rows with fewer passing S rows are padded */
#define EJOIN_FP64_SCORES 0x20u  /* threshold joins (single, selection, batch): no pair is
                                    accepted on its approximate score; every pair at or above
                                    the band's lower edge goes to the FP64 rescore, so every
                                    returned score is float(sim64).  The band list must then
                                    hold all those pairs (opts->band_capacity; the
                                    EJOIN_E_WORKSPACE retry reports band_needed).  Top-k
                                    scores are always float(sim64) and ignore the flag. */

/* Autotuned tile choices (opaque; see ejoin_tuner_create). */
typedef struct ejoin_tuner ejoin_tuner;

typedef struct {
    int32_t prec;           /* ejoin_prec */
    int32_t tile;           /* 0: planner's choice; otherwise a tile id from ejoin_tile_name */
    double band;            /* < 0: the default: the rigorous bound for prec and dim, which
                               BF16 / FP8 single threshold joins narrow on the device with
                               the largest quantisation error norm measured on each side
                               (stats->band reports it); otherwise the band half-width (must
                               be >= the rigorous bound, else EJOIN_E_INVAL) */
    int64_t band_capacity;  /* <= 0: default; number of band pairs the workspace can hold */
    uint32_t flags;         /* EJOIN_* flags */
    int32_t topk_cand;      /* top-k: per-row candidate capacity (<= 0: default) */
    const ejoin_tuner *tuner; /* (host, may be NULL) consulted when tile == 0 */
    const void *prefilter;  /* EJOIN_APPROX_PREFILTER: device state block of a prefilter
                               network (ejoin_mlp_*) for the jobs' dim */
    float prefilter_eps;    /* EJOIN_APPROX_PREFILTER: margin below theta */
    double topk_min_sim;    /* EJOIN_TOPK_MIN_SIM: the range bound (finite) */
} ejoin_opts;

/* Optional per-call report (host struct, may be NULL). */
typedef struct {
    int64_t n_pairs;        /* total matches (may exceed capacity) */
    int64_t n_certain;      /* pairs accepted straight from the approximate score */
    int64_t n_band;         /* pairs rescored in FP64 */
    int64_t n_band_accepted;
    int64_t band_needed;    /* band capacity that would have been enough */
    size_t ws_needed;       /* workspace bytes this call needs */
    double band;            /* band half-width used */
    int32_t tile;           /* tile id used */
    int32_t n_fallback;     /* top-k: rows recomputed by the exact row scan */
    float ms_prep, ms_main, ms_rescore, ms_total;  /* with EJOIN_TIMING */
    double topk_floor;      /* top-k: candidate floor used by the sweep */
    int32_t topk_slots;     /* top-k: candidate slots per row */
    int64_t tiles_total;    /* batch: tile pairs of all jobs */
    int64_t tiles_kept;     /* batch: tile pairs contracted (all of them unless prefiltered) */
    int64_t topk_refined;   /* top-k: rows swept again with a floor of their own */
} ejoin_stats;

/* Library version string (static storage). */
const char *ejoin_version(void);

/* Human-readable text for a status code (static storage). */
const char *ejoin_strerror(ejoin_status s);

/* Default options: FP32, planner tile, rigorous band, default capacities. */
void ejoin_opts_default(ejoin_opts *opts /* host */);

/* Rigorous band half-width for a precision and dimension: the bound on
 * |approximate score - sim64| derived in the design notes (FP32 and BF16:
 * a global bound; FP8: the worst case of the per-pair bound). */
double ejoin_band_default(int32_t prec, int32_t dim);

/*
 * Workspace bytes needed by ejoin_threshold for these relations and options
 * (the band list size follows opts->band_capacity).  R, S, opts are host
 * pointers; only rows/dim are read from R and S.  Returns 0 on bad arguments.
 */
size_t ejoin_threshold_workspace(const ejoin_rel *R, const ejoin_rel *S,
                                 const ejoin_opts *opts);

/*
 * Threshold E-join (Sections III.C, IV.C): every (i, j) with
 * sim64(R_i, S_j) >= theta.
 *   R, S      (host structs) relations; R->dim == S->dim.  R and S may alias.
 *   theta     finite threshold.
 *   opts      (host, may be NULL = defaults).  opts->tile: 0 or a tile id of
 *             opts->prec (ejoin_tile_name); the register-panel tiles (12 BF16,
 *             13 FP8, 14 / 15 BF16 / FP8 in two workgroups per CU, 20 / 21
 *             FP32 in one / two) take rows of at most 768 bytes of padded K,
 *             tiles 12, 14, 20 and 21 also of 1024, 1152, 1280 or 1536 bytes;
 *             other depths give EJOIN_E_INVAL; 19 and 22 are batch-only.
 *             Tile 23 (FP32, dim <= 1024) is the nested-loop comparator of
 *             Section V.A: one pair per wavefront, the lanes splitting the
 *             dimension, no tiling and no matrix cores; same exact result,
 *             only for measuring the tensor form against it (never chosen
 *             by the planner or the tuner).
 *   out       device array of `capacity` pairs; order of pairs is unspecified.
 *   n_out     (host) receives the number of matching pairs, or, with
 *             EJOIN_NO_SYNC, a DEVICE int64 that will hold it.
 *   ws        device workspace of ws_bytes >= ejoin_threshold_workspace(...).
 *   stream    HIP stream for all work.
 *   stats     (host, may be NULL) per-call report; filled only in sync mode.
 * Returns EJOIN_E_OVERFLOW when more pairs matched than `capacity`: out then
 * holds an arbitrary `capacity`-sized subset and *n_out the true count.
 */
ejoin_status ejoin_threshold(const ejoin_rel *R, const ejoin_rel *S, double theta,
                             const ejoin_opts *opts, ejoin_pair *out, int64_t capacity,
                             int64_t *n_out, void *ws, size_t ws_bytes,
                             hipStream_t stream, ejoin_stats *stats);

/*
 * Allocation-free threshold join, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, semantics and results as
 * ejoin_threshold, without the workspace: the call runs on a scratch array of
 * EJOIN_NOALLOC_SCRATCH_BYTES that the library holds in device memory on every
 * GPU it runs on until the process ends.  It calls no allocator.
 *   - Joins whose workspace (ejoin_threshold_workspace with the same
 *     arguments) exceeds EJOIN_NOALLOC_SCRATCH_BYTES are refused with
 *     EJOIN_E_WORKSPACE (stats->ws_needed holds the size they need); for
 *     FP32 rows of 300 dims that is about 48k rows of R and S together.
 *   - All calls on one GPU share that GPU's array: calls that overlap in time
 *     on one GPU (different streams, or different host threads) race and give
 *     undefined results.  Calls ordered on one stream are safe.  Every call
 *     starts by clearing the counters it uses; it reads nothing else that an
 *     earlier call left there.
 *   - EJOIN_TIMING is ignored (it would create events).
 */
#define EJOIN_NOALLOC_SCRATCH_BYTES (64u << 20)
ejoin_status ejoin_threshold_noalloc(const ejoin_rel *R, const ejoin_rel *S, double theta,
                                     const ejoin_opts *opts, ejoin_pair *out, int64_t capacity,
                                     int64_t *n_out, hipStream_t stream, ejoin_stats *stats);
/* EJOIN_NOALLOC_SCRATCH_BYTES as built into the library. */
size_t ejoin_noalloc_scratch_bytes(void);

/*
 * Workspace bytes needed by ejoin_topk (host arguments; 0 on bad arguments or
 * an unsupported combination).
 */
size_t ejoin_topk_workspace(const ejoin_rel *R, const ejoin_rel *S, int32_t k,
                            const ejoin_opts *opts);

/*
 * Top-k E-join (the top-k join condition of Section VI.E): for every R row i,
 * the first min(k, |S|) S indices in the order (sim64 desc, index asc).
 *   out_idx    device int32 [|R| * k], row-major; slots past |S| hold -1.
 *   out_score  device float [|R| * k]: float(sim64); -inf in empty slots.
 *   opts->prec precision of the contraction sweep: EJOIN_FP32 (the plain
 *              form), EJOIN_BF16 or EJOIN_FP8_E4M3, any dim; the result is
 *              exact in all three.  Rows of up to six 128-byte K slices (BF16
 *              and FP32 also 8, 9, 10 or 12) sweep on register panels, other
 *              depths on the 128 x 128 LDS tile kernel (stats->tile names the
 *              form).  The panels give each workgroup all of S for 128 R rows,
 *              so the planner (opts->tile 0) takes them for |R| >= 65536 and
 *              the tile kernel below that; opts->tile forces the form: a
 *              panel tile of the precision (12-15, 20, 21; rows of a depth
 *              with a panel form) or its 128 x 128 tile (1 FP32, 3 BF16,
 *              5 FP8); other ids give EJOIN_E_INVAL.
 *   opts->topk_cand  candidate slots per row (k..256; <= 0: 256).
 * With EJOIN_TOPK_MIN_SIM the condition is the range predicate combined
 * with the top-k one (Section VI.E evaluates such a range join with k = 32):
 * per R row the first min(k, m) of the m S rows with sim64 >= topk_min_sim
 * in the same order, the other slots padded; the candidate floor is raised
 * to topk_min_sim minus the error bound.
 * 1 <= k <= 256.  The call runs a pilot (exact FP64 top-k of up to 256 sample
 * rows) to set a candidate floor, one contraction sweep that keeps every
 * column above the floor, and a per-row finalize that certifies the candidate
 * set (no slot overflow, k-th score minus twice the row's error bound at or
 * above the floor), rescores it in FP64 and sorts it.  Rows whose slots
 * overflowed are swept again (synchronous calls) with a floor of their own:
 * their k-th best kept approximate score minus twice their error bound, a
 * lower bound of every exact top-k member's approximate score (counted in
 * stats->topk_refined); rows that still fail take an exact FP64 scan
 * (stats->n_fallback).
 */
ejoin_status ejoin_topk(const ejoin_rel *R, const ejoin_rel *S, int32_t k, const ejoin_opts *opts,
                        int32_t *out_idx, float *out_score, void *ws, size_t ws_bytes,
                        hipStream_t stream, ejoin_stats *stats);

/* ------------------------------------------------------------------------
 * Relational selections pushed below the join
 * ------------------------------------------------------------------------
 * The scan-versus-probe study of the paper (Section VI.E) runs the E-join
 * after a relational pre-filter on another attribute, at selectivities from
 * 1% to 100%; the tensor (scan) join then contracts only the tuples that
 * pass (the selection is pushed below the join, Section III.C's equivalences
 * of selections and joins).  A selection is the list of a relation's rows
 * that passed, as device int32 row ids in strictly ascending order, each in
 * [0, rows); a NULL selection keeps every row.  Results name the caller's
 * rows: offsets in threshold pairs and indices in top-k output are row ids of
 * R and S, not positions in the lists.  A list that is not strictly
 * ascending or holds an id out of range gives EJOIN_E_INVAL (found on the
 * device; with EJOIN_NO_SYNC the device count holds -EJOIN_E_INVAL). */
typedef struct {
    const int32_t *ids;  /* device, n ids, strictly ascending */
    int64_t n;           /* 0 <= n <= rows of the relation */
} ejoin_sel;

/*
 * sigma(lo <= col[i] < hi) over a float attribute column of n rows (device),
 * as a selection: ids (device, room for n) receives the passing row ids in
 * ascending order and n_sel (DEVICE int64) their number.  NaN never passes.
 * ws: device workspace of ejoin_select_workspace() bytes.  Asynchronous (no
 * host wait).  n < 2^31.
 */
size_t ejoin_select_workspace(void);
ejoin_status ejoin_select_range(const float *col, int64_t n, float lo, float hi, int32_t *ids,
                                int64_t *n_sel, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Threshold join over selections: every (i, j) with i in sel_r, j in sel_s
 * and sim64(R_i, S_j) >= theta, i and j being row ids of R and S.  The prep
 * pass reads the selected rows through the lists (no copy of the relations)
 * and only they are contracted; band pairs are rescored from the caller's
 * rows; the emitted offsets are mapped back to row ids at the end.  Other
 * arguments as ejoin_threshold; R and S alias only with the same selection.
 */
size_t ejoin_threshold_sel_workspace(const ejoin_rel *R, const ejoin_sel *sel_r,
                                     const ejoin_rel *S, const ejoin_sel *sel_s,
                                     const ejoin_opts *opts);
ejoin_status ejoin_threshold_sel(const ejoin_rel *R, const ejoin_sel *sel_r, const ejoin_rel *S,
                                 const ejoin_sel *sel_s, double theta, const ejoin_opts *opts,
                                 ejoin_pair *out, int64_t capacity, int64_t *n_out, void *ws,
                                 size_t ws_bytes, hipStream_t stream, ejoin_stats *stats);

/*
 * Top-k join over selections: for the i-th selected R row (output row i,
 * out_idx and out_score hold sel_r->n * k entries, or |R| * k without a
 * selection) the first min(k, |sel_s|) selected S rows in the order (sim64
 * desc, S row id asc), as S row ids.  The selected rows are copied into
 * compact buffers in the workspace first.  Other arguments as ejoin_topk.
 */
size_t ejoin_topk_sel_workspace(const ejoin_rel *R, const ejoin_sel *sel_r, const ejoin_rel *S,
                                const ejoin_sel *sel_s, int32_t k, const ejoin_opts *opts);
ejoin_status ejoin_topk_sel(const ejoin_rel *R, const ejoin_sel *sel_r, const ejoin_rel *S,
                            const ejoin_sel *sel_s, int32_t k, const ejoin_opts *opts,
                            int32_t *out_idx, float *out_score, void *ws, size_t ws_bytes,
                            hipStream_t stream, ejoin_stats *stats);

/* ------------------------------------------------------------------------
 * Batched threshold joins
 * ------------------------------------------------------------------------
 * Many independent threshold joins (each its own R, S, theta, output) run
 * as ONE pass: a batched prep launch, one persistent contraction launch in
 * which workgroups pull (job, tile) work items from an atomic counter (jobs
 * ordered largest first), a batched FP64 rescore of the band pairs of all
 * jobs, and a count copy.  "Many queries as one join": the result of every
 * job is exactly its own threshold join (Section III.C); the partition of
 * the work into jobs and tiles does not change any result (the block
 * decomposition of Section IV.C). */
typedef struct {
    ejoin_rel R, S;       /* (host structs; data pointers on the device) */
    double theta;         /* finite */
    ejoin_pair *out;      /* device array of `capacity` pairs */
    int64_t capacity;
} ejoin_job;

/* Workspace bytes for ejoin_batch (host arguments; 0 on bad arguments).
 * opts->band_capacity is the size of the band list SHARED by all jobs
 * (<= 0: sum over jobs of max(65536, |R| + |S|)). */
size_t ejoin_batch_workspace(const ejoin_job *jobs, int32_t n_jobs, const ejoin_opts *opts);

/*
 * Run a batch of threshold joins.
 *   jobs, n_jobs  (host) 0 <= n_jobs <= 65536; all jobs use opts->prec.
 *   opts->tile    a tile of the LDS tile kernel for opts->prec; or 19 / 22,
 *                 the batch forms of the BF16 register panels (128-row
 *                 panels, each work item one panel over 16 S tiles of 128
 *                 rows; one workgroup per CU, or two with 32-row S tiles),
 *                 which need every non-empty
 *                 job's dim padded to 512, 576, 640 or 768 (dims 449-640 and
 *                 705-768), else EJOIN_E_INVAL; the other register-panel
 *                 tiles have no batch form (EJOIN_E_INVAL); or 0: the tuner's
 *                 choice, else 22 for a BF16 batch whose every job has such
 *                 a dim, else the planner's default tile.
 *   n_out         (host) int64[n_jobs] receives each job's true match count;
 *                 with EJOIN_NO_SYNC a DEVICE int64[n_jobs] (negative status
 *                 codes as for EJOIN_NO_SYNC above).
 * With EJOIN_APPROX_PREFILTER (BF16, tile 3, 19, 22 or 0, every job of the same dim
 * as the network, eager calls only): the prepared rows are coded by the
 * network; 2048 anchor codes drawn from the rows (SplitMix64, seed
 * 0x5EED) are grouped by leader clustering at cosine 0.6 and every relation
 * is reordered by the group of each row's nearest anchor; only the
 * 128 x 128 tile pairs whose bound reaches theta - eps are contracted, the
 * bound being the smaller of
 *     c_T . c_U + rho_T |c_U| + rho_U |c_T| + rho_T rho_U   and
 *     cos(max(0, angle(c_T, c_U) - a_T - a_U))
 * (c: mean code of a tile, rho: largest distance of a code from c, a:
 * largest angle of a code from c's direction); pairs are mapped back to the
 * caller's row numbers.  Tiles 19 and 22 contract the same tile pairs: a
 * panel sweeps only the kept S tiles of its 16-tile chunk, and chunks with
 * none are not visited.
 * With EJOIN_EXACT_PRUNE (BF16, tile 3, 19, 22 or 0, every job of one dim up
 * to 1024, eager calls only; not with EJOIN_APPROX_PREFILTER) the result is
 * the exact join: the rows are ordered as above but by the codes of a fixed
 * random +-1 projection to 64 dimensions, and a tile pair is skipped only
 * when, in the original space, for T's mean direction d_T and angular radius
 * A_T (largest angle of a row from d_T, widened by the rows' rounding error
 * norms) and the largest d_T . s over U's rows (widened likewise),
 *     cos(max(0, acos(max_s d_T . s) - A_T)) < theta,
 * or the same with T and U exchanged; every pair of such a tile pair has
 * cosine below theta.  Jobs with theta <= 0 are not pruned.
 * stats->tiles_kept counts the contracted tile pairs.
 * Returns EJOIN_E_OVERFLOW if any job matched more pairs than its capacity
 * (that job's `out` holds an arbitrary capacity-sized subset; re-run it with
 * more room), EJOIN_E_WORKSPACE if the shared band list was too small
 * (stats->band_needed), EJOIN_E_NONFINITE / EJOIN_E_RANGE if any job's
 * input is bad (that job's count is 0).  stats (may be NULL) sums over jobs.
 */
ejoin_status ejoin_batch(const ejoin_job *jobs, int32_t n_jobs, const ejoin_opts *opts,
                         int64_t *n_out, void *ws, size_t ws_bytes, hipStream_t stream,
                         ejoin_stats *stats);

/*
 * A captured HIP graph of the batch pass, replayable for new batches.
 *   create   captures the pass once on `stream` for up to max_jobs jobs and
 *            the workspace ws (ws_bytes); opts fixes prec, tile, band and the
 *            band-list capacity.  A pinned host staging table of
 *            max_jobs entries is allocated here (the only allocation).
 *   launch   plans `jobs` into the same workspace, writes the job table into
 *            the staging buffer (waiting for the previous replay to finish
 *            with it) and replays the graph on `stream`.  n_out is a DEVICE
 *            int64[n_jobs] as in asynchronous ejoin_batch, and must stay the
 *            same array between replays only if the caller wants that.
 *            EJOIN_E_WORKSPACE if the jobs do not fit the workspace.
 *   destroy  waits for outstanding replays and frees the graph.
 */
typedef struct ejoin_batch_graph ejoin_batch_graph;
ejoin_status ejoin_batch_graph_create(int32_t max_jobs, const ejoin_opts *opts, void *ws,
                                      size_t ws_bytes, hipStream_t stream,
                                      ejoin_batch_graph **graph /* host */);
ejoin_status ejoin_batch_graph_launch(ejoin_batch_graph *graph, const ejoin_job *jobs,
                                      int32_t n_jobs, int64_t *n_out, hipStream_t stream);
ejoin_status ejoin_batch_graph_destroy(ejoin_batch_graph *graph);

/* ------------------------------------------------------------------------
 * Autotuner: tile shapes measured on the caller's own data
 * ------------------------------------------------------------------------
 * A tuner maps (operation, precision, padded dimension, size bucket) to a
 * tile id; the size bucket is floor(log4(total |R| x |S|)).  It is a plain
 * host object owned by the caller (no global state); it can be saved to and
 * loaded from a small text file.  ejoin_autotune times every tile of
 * opts->prec that can run the given jobs (the batch pass for n_jobs > 1,
 * the single join for n_jobs == 1, panels included there), `reps` timed runs
 * each after one warm-up, records the fastest in the tuner and returns it in
 * *best_tile.  ms (host, may be NULL) receives ejoin_tile_count() + 1 values
 * indexed by tile id: median milliseconds, or -1 for tiles not timed. */
ejoin_tuner *ejoin_tuner_create(void);
void ejoin_tuner_destroy(ejoin_tuner *t);
int32_t ejoin_tuner_lookup(const ejoin_tuner *t, int32_t batch, int32_t prec, int32_t dim,
                           double pairs);
ejoin_status ejoin_tuner_save(const ejoin_tuner *t, const char *path /* host */);
ejoin_status ejoin_tuner_load(ejoin_tuner *t, const char *path /* host */);
ejoin_status ejoin_autotune(ejoin_tuner *t, const ejoin_job *jobs, int32_t n_jobs,
                            const ejoin_opts *opts, void *ws, size_t ws_bytes,
                            hipStream_t stream, int32_t reps, int32_t *best_tile /* host */,
                            float *ms /* host, may be NULL */);

/* ------------------------------------------------------------------------
 * Learned prefilter network (approximate mode; not part of the paper)
 * ------------------------------------------------------------------------
 * A two-layer MLP codes a normalised embedding row x (dim values) as a unit
 * vector: h = ReLU(x W1 + b1) (256), z = h W2 + b2 (64), u = z / ||z||; the
 * predicted similarity of a pair is u_r . u_s.  Weights are FP32 masters
 * with BF16 copies; products use the BF16 values and accumulate in FP32.
 * Training minimises, over a batch of pairs with targets t (their sim64),
 *     mean[(p - t)^2] + lambda * mean[max(0, t - p)^2 * 1{t >= theta_lo}]
 * with Adam.  All network state lives in ONE caller-owned device block whose
 * layout ejoin_mlp_layout_get describes. */
#define EJOIN_MLP_HIDDEN 256
#define EJOIN_MLP_OUT    64
#define EJOIN_MLP_GRAD_ONLY 0x1u  /* train step: compute gradients, do not update */

typedef struct {
    int32_t dim, dim_pad;   /* input width; its padding to a multiple of 64 */
    int64_t n_params;       /* dim*256 + 256 + 256*64 + 64 */
    /* byte offsets in the state block.  FP32 vectors of n_params values,
     * flat: W1 (dim x 256, row-major), b1 (256), W2 (256 x 64), b2 (64) */
    size_t off_params, off_grads, off_m, off_v;
    size_t off_w1t;         /* BF16 W1^T, 256 x dim_pad (zero beyond dim) */
    size_t off_w2t;         /* BF16 W2^T, 64 x 256 */
    size_t off_step;        /* int64 number of Adam steps taken */
    size_t total;           /* bytes of the state block */
} ejoin_mlp_layout;

typedef struct {
    float lr, beta1, beta2, eps;  /* Adam (defaults 1e-3, 0.9, 0.999, 1e-8) */
    float lambda, theta_lo;       /* recall term (defaults 4, 0.7) */
    uint32_t flags;               /* EJOIN_MLP_GRAD_ONLY */
} ejoin_mlp_hparams;

/* Layout of the state block for inputs of width dim (1..1024). */
ejoin_status ejoin_mlp_layout_get(int32_t dim, ejoin_mlp_layout *layout /* host */);
void ejoin_mlp_hparams_default(ejoin_mlp_hparams *hp /* host */);

/* Set the masters to `params` (device, n_params FP32 in the flat order; the
 * seeded initial weights are the caller's), zero gradients, moments and step
 * count, and build the BF16 copies. */
ejoin_status ejoin_mlp_init(void *state, int32_t dim, const float *params, hipStream_t stream);

/* Workspace bytes of a training step of `batch` pairs. */
size_t ejoin_mlp_train_workspace(int32_t dim, int32_t batch);

/*
 * One training step on `batch` pairs: rows pr[i] and ps[i] (device int32,
 * 0 <= index < rows; an index outside that range reads as a zero row) of X
 * (device BF16 rows, ldx elements apart, the first dim used), targets
 * target[i] (device FP32).  Writes the batch loss to *loss (device FP32) and
 * the gradients into the state; unless hp->flags has EJOIN_MLP_GRAD_ONLY,
 * applies Adam and refreshes the BF16 copies.  hp: host, NULL = defaults.
 */
ejoin_status ejoin_mlp_train_step(void *state, int32_t dim, const uint16_t *X, int64_t ldx,
                                  int64_t rows, const int32_t *pr, const int32_t *ps,
                                  const float *target, int32_t batch,
                                  const ejoin_mlp_hparams *hp, void *ws, size_t ws_bytes,
                                  float *loss, hipStream_t stream);

/* Workspace bytes of ejoin_mlp_forward over n rows. */
size_t ejoin_mlp_forward_workspace(int32_t dim, int64_t n);

/*
 * Codes of n rows on the matrix cores: U (device FP32, n x 64) = u(X_i).
 * X: device BF16 rows of exactly dim_pad values each (zero beyond dim), and
 * round_up(n, 128) rows must be readable (the layout of the join's prepared
 * BF16 operands).  The hidden layer is kept in BF16.
 */
ejoin_status ejoin_mlp_forward(const void *state, int32_t dim, const uint16_t *X, int64_t n,
                               float *U, void *ws, size_t ws_bytes, hipStream_t stream);

/* Training of the prefilter on the caller's batch: pairs are drawn from the
 * exact join's outputs (share pos_frac) and uniformly from R x S of the
 * jobs (job chosen in proportion to |R| |S|), their targets are their sim64
 * (the canonical FP64 rule, on the GPU), their rows are prepared exactly as
 * the BF16 join prepares operands, and `steps` training steps of `batch`
 * pairs are taken.  Draws use SplitMix64 seeded with `seed`. */
typedef struct {
    int32_t steps;          /* default 300 */
    int32_t batch;          /* pairs per step, default 4096 */
    uint64_t seed;          /* default 1 */
    float pos_frac;         /* default 0.5 */
    ejoin_mlp_hparams hp;   /* defaults of ejoin_mlp_hparams_default */
} ejoin_prefilter_train_opts;

void ejoin_prefilter_train_opts_default(ejoin_prefilter_train_opts *to /* host */);
size_t ejoin_prefilter_train_workspace(int32_t n_jobs, int32_t dim, int32_t batch);

/*
 * jobs: the batch whose exact join was run (jobs[i].out holds n_out[i]
 * pairs, n_out host int64[n_jobs]; only min(n_out[i], capacity) are drawn
 * from); all jobs of the network's dim.  losses (host, may be NULL)
 * receives the loss of every step (this synchronises once per step).
 */
ejoin_status ejoin_prefilter_train(void *state, const ejoin_job *jobs, int32_t n_jobs,
                                   const int64_t *n_out, const ejoin_prefilter_train_opts *to,
                                   void *ws, size_t ws_bytes, float *losses, hipStream_t stream);

/*
 * Checkpoint and resume of a prefilter network (host file).  save writes the
 * state block's FP32 masters, Adam moments and step count for inputs of width
 * dim, with the caller's margin eps and training seed, to `path` (a binary
 * file: an 8-byte magic "EJPFNET1", int32 dim, int32 0, int64 n_params,
 * int64 step, float eps, uint32 0, uint64 seed, then masters, first and
 * second moments as n_params little-endian FP32 values each) and
 * synchronises the stream.  load restores such a file into a state block of
 * the same dim: masters, moments and step as saved, gradients zero, BF16
 * copies rebuilt (codes and further training steps equal the saved
 * network's); eps and seed (host, may be NULL) receive the saved values.
 * EJOIN_E_INVAL: bad arguments, a file that cannot be read or written, a
 * different dim or a malformed file (checked before the device is touched);
 * EJOIN_E_NONFINITE: a non-finite value in the file.  The state block is
 * caller-owned device memory, so there is nothing to free.
 */
ejoin_status ejoin_prefilter_save(const void *state, int32_t dim, float eps, uint64_t seed,
                                  const char *path /* host */, hipStream_t stream);
ejoin_status ejoin_prefilter_load(void *state, int32_t dim, const char *path /* host */,
                                  float *eps /* host */, uint64_t *seed /* host */,
                                  hipStream_t stream);

/* Number of tile shapes the library was built with, and the name of one
 * ("prec:BMxBNxBK"); id 0 is "planner's choice".  Static storage. */
int32_t ejoin_tile_count(void);
const char *ejoin_tile_name(int32_t tile);

/* Resident workgroups per CU of the register-panel kernel that a threshold
 * join with `tile` (12, 13, 14, 15, 20, 21, 24, 25) and rows of `dim`
 * elements would launch: *designed (host) receives the count the kernel is
 * laid out for (its launch bound; the two-workgroup forms 14, 15 and 21 are
 * laid out for 2), *resident (host) what the runtime reports for the
 * compiled kernel on the current device.  Nothing is launched.  Returns
 * EJOIN_E_INVAL for another tile or a depth the tile does not take. */
ejoin_status ejoin_tile_occupancy(int32_t tile, int32_t dim, int32_t *designed, int32_t *resident);

#ifdef __cplusplus
}
#endif

#endif /* EJOIN_H */
