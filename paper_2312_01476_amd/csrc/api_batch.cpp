// api_batch.cpp -- C ABI of the batched threshold join: the batch plan (job
// order, workspace carve-up, job table), the eager call and the captured
// graph of the pass.
#include <hip/hip_runtime.h>

#include <vector>

#include "batch.hpp"
#include "mlp.hpp"
#include "plan.hpp"
#include "prefilter.hpp"

using namespace ej;
using namespace ej::plan;

namespace {

constexpr int kAnchors = 2048;      // prefilter: anchor codes of the ordering key
constexpr float kAnchorTau = 0.6f;  // prefilter: leader-clustering cosine of the anchors
constexpr uint64_t kAnchorSeed = 0x5EED;

// SplitMix64 (Steele, Lea and Flood, 2014): golden-ratio counter and a
// MurmurHash3-style finaliser
struct SplitMix64 {
    uint64_t x;
    uint64_t next() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint64_t below(uint64_t n) { return (uint64_t)(((unsigned __int128)next() * n) >> 64); }
};
constexpr int kRescoreGrid = 2048;  // batched rescore: grid-stride over the band list

// measured on the 64-job 768-d workload: BF16 register panels in two
// workgroups per CU (tile 22, also with the prefilter) where every job's
// row depth has one, else the 256 x 256 staged tile; FP32 and FP8 keep their
// 128 x 128 tiles
int batch_default_tile(int prec) { return prec == P_FP32 ? 1 : prec == P_BF16 ? 16 : 5; }

// the batch forms of the BF16 register panels: one (19) or two (22)
// workgroups per CU
bool batch_panel_tile(int tile) { return tile == 19 || tile == 22; }

bool panel_jobs_ok(const ejoin_job* jobs, int n) {
    for (int i = 0; i < n; ++i)
        if (jobs[i].R.rows > 0 && jobs[i].S.rows > 0 &&
            !batch_panel_depth(padded_k(EJOIN_BF16, jobs[i].R.dim) * 2))
            return false;
    return true;
}

bool job_ok(const ejoin_job& j) {
    if (!rel_ok(&j.R) || !rel_ok(&j.S) || j.R.dim != j.S.dim) return false;
    if (!isfinite(j.theta) || j.capacity < 0) return false;
    if (j.capacity > 0 && j.out == nullptr) return false;
    return true;
}

// Device table image and workspace layout of one batch.
struct BatchPlan {
    int prec = 0, tile = 0, bm = 0, bn = 0, n_jobs = 0, table_jobs = 0;
    double band_max = 0.0;
    int64_t band_cap = 0, n_tiles = 0, n_rows = 0, pairs_total = 0;
    size_t off_table = 0, table_bytes = 0, off_hdrs = 0, off_band = 0, total = 0;
    // prefilter mode (approx) and exact pruning (approx and exact: the same
    // ordering and work-list machinery with certified bounds)
    bool approx = false, exact = false;
    int kp = 0;            // exact pruning: padded depth of the jobs (BF16 elements)
    int kp_max = 0;        // deepest padded row of the batch (elements)
    size_t off_proj = 0;   // exact pruning: the 64 x kp projection
    size_t off_hb = 0, off_u = 0, off_key = 0, off_pa = 0, off_pb = 0, off_hist = 0,
           off_offs = 0, off_c = 0, off_rho = 0, off_cn = 0, off_alpha = 0, off_work = 0,
           off_ub = 0, off_aidx = 0, off_af = 0, off_ab = 0, off_lab = 0, off_up = 0,
           off_dir = 0, off_m1 = 0, off_m2 = 0, off_keep = 0, off_wmask = 0, off_abits = 0;
    int64_t n_side = 0, n_chunks = 0;
    int n_anchor = 0;
    std::vector<int64_t> anchor_idx;  // flat rows whose codes are the anchors
    std::vector<char> image;  // head, jobs[table_jobs], segs[2 * table_jobs]
    BatchHead* head() { return (BatchHead*)image.data(); }
    BatchJob* jobs() { return (BatchJob*)(image.data() + sizeof(BatchHead)); }
    PrepSeg* segs() { return (PrepSeg*)(image.data() + sizeof(BatchHead) +
                                         (size_t)table_jobs * sizeof(BatchJob)); }
};

size_t table_size(int table_jobs) {
    return align256(sizeof(BatchHead) + (size_t)table_jobs * sizeof(BatchJob) +
                    2 * (size_t)table_jobs * sizeof(PrepSeg));
}

int pick_batch_tile(const ejoin_opts& o, const ejoin_job* jobs, int n) {
    if (o.tile > 0) return o.tile;
    // prefilter mode: 128 x 128 tiles or 128-row panels, the statistics' grain
    if (o.flags & (EJOIN_APPROX_PREFILTER | EJOIN_EXACT_PRUNE))
        return o.prec == EJOIN_BF16 && n > 0 && panel_jobs_ok(jobs, n) ? 22 : 3;
    if (o.tuner && n > 0) {
        double pairs = 0.0;
        int dim = jobs[0].R.dim;
        for (int i = 0; i < n; ++i) pairs += (double)jobs[i].R.rows * (double)jobs[i].S.rows;
        const int t = tuner_pick(o.tuner, 1, o.prec, dim, pairs);
        const TileDesc* td = t > 0 ? tile_get(t) : nullptr;
        if (td && td->prec == o.prec && batch_has_tile(t) &&
            (!batch_panel_tile(t) || panel_jobs_ok(jobs, n)))
            return t;
    }
    if (o.prec == EJOIN_BF16 && n > 0 && panel_jobs_ok(jobs, n)) return 22;
    return batch_default_tile(o.prec);
}

// Plan `jobs` for a table of `table_jobs` entries.  With ws == nullptr only
// the sizes are computed; otherwise every device pointer of the table is
// filled in for that workspace.
ejoin_status make_batch_plan(const ejoin_job* jobs, int n, const ejoin_opts& o, int tile,
                             int table_jobs, char* ws, int64_t* n_out_dev, BatchPlan& bp) {
    if (n < 0 || n > 65536 || (n > 0 && !jobs) || table_jobs < n) return EJOIN_E_INVAL;
    bp.exact = (o.flags & EJOIN_EXACT_PRUNE) != 0;
    bp.approx = (o.flags & EJOIN_APPROX_PREFILTER) != 0 || bp.exact;
    if ((o.flags & EJOIN_APPROX_PREFILTER) && bp.exact) return EJOIN_E_INVAL;
    if (bp.approx) {
        // the network (or the projection) reads BF16 prepared rows; tile
        // statistics are per 128 rows
        if (o.prec != EJOIN_BF16) return EJOIN_E_INVAL;
        if (!bp.exact && (!o.prefilter || !(o.prefilter_eps >= 0.0f))) return EJOIN_E_INVAL;
        if (tile != 3 && !batch_panel_tile(tile)) return EJOIN_E_INVAL;
        for (int i = 1; i < n; ++i)
            if (jobs && jobs[i].R.dim != jobs[0].R.dim) return EJOIN_E_INVAL;
        if (n > 0 && jobs && (jobs[0].R.dim < 1 || jobs[0].R.dim > 1024)) return EJOIN_E_UNSUPPORTED;
    }
    if (o.prec < EJOIN_FP32 || o.prec > EJOIN_FP8_E4M3) return EJOIN_E_INVAL;
    const TileDesc* td = tile_get(tile);
    if (!td || td->prec != o.prec || !batch_has_tile(tile)) return EJOIN_E_INVAL;
    if (batch_panel_tile(tile) && !panel_jobs_ok(jobs, n)) return EJOIN_E_INVAL;
    bp.prec = o.prec;
    bp.tile = tile;
    bp.bm = td->bm;
    bp.bn = td->bn;
    bp.n_jobs = n;
    bp.table_jobs = table_jobs;
    const size_t eb = (size_t)elem_bytes(o.prec);

    // largest first (tile count), ties by caller order
    std::vector<int> order(n);
    std::vector<int64_t> ntile(n);
    for (int i = 0; i < n; ++i) {
        if (!job_ok(jobs[i])) return EJOIN_E_INVAL;
        if (jobs[i].R.dim > 65536) return EJOIN_E_UNSUPPORTED;
        const int64_t tm = (jobs[i].R.rows + bp.bm - 1) / bp.bm;
        const int64_t tn = (jobs[i].S.rows + bp.bn - 1) / bp.bn;
        if (tm * tn > 0x7fffffffLL) return EJOIN_E_UNSUPPORTED;
        ntile[i] = tm * tn;
        order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return ntile[a] > ntile[b]; });

    bp.image.assign(sizeof(BatchHead) + (size_t)table_jobs * (sizeof(BatchJob) + 2 * sizeof(PrepSeg)),
                    0);
    size_t off = align256(B_COUNT * sizeof(unsigned long long));
    bp.off_table = off;
    bp.table_bytes = table_size(table_jobs);
    off += bp.table_bytes;
    bp.off_hdrs = off;
    off = align256(off + (size_t)n * H_COUNT * sizeof(unsigned long long));

    BatchJob* J = bp.jobs();
    PrepSeg* G = bp.segs();
    int nseg = 0;
    int64_t tile_base = 0, row_base = 0, band_default = 0;
    std::vector<int64_t> rb_r(n, 0), rb_s(n, 0);
    auto at = [&](size_t o_) -> char* { return ws ? ws + o_ : nullptr; };
    for (int q = 0; q < n; ++q) {
        const ejoin_job& u = jobs[order[q]];
        BatchJob& b = J[q];
        const int dim = u.R.dim;
        const int Kp = padded_k(o.prec, dim);
        bp.kp_max = std::max(bp.kp_max, Kp);
        const double rig = band_rigorous(o.prec, dim);
        double band = rig;
        if (o.band >= 0) {
            if (!(o.band >= rig) || !isfinite(o.band)) return EJOIN_E_INVAL;
            band = o.band;
        }
        bp.band_max = std::max(bp.band_max, band);
        const bool alias = u.R.data == u.S.data && u.R.rows == u.S.rows && u.R.ld == u.S.ld;
        const int64_t padR = padded_rows(u.R.rows), padS = alias ? padR : padded_rows(u.S.rows);
        const bool empty = u.R.rows == 0 || u.S.rows == 0;
        b.R = u.R.data;
        b.S = u.S.data;
        b.ldR = u.R.ld;
        b.ldS = u.S.ld;
        b.nR = u.R.rows;
        b.nS = u.S.rows;
        b.out = (Pair*)u.out;
        b.capacity = u.capacity;
        b.hdr = (unsigned long long*)at(bp.off_hdrs + (size_t)q * H_COUNT * 8);
        b.theta = u.theta;
        b.lo = round_down_f(u.theta - band);
        b.hi = round_up_f(u.theta + band);
        b.all64 = (o.flags & EJOIN_FP64_SCORES) ? 1 : 0;
        if (b.all64) b.hi = INFINITY;  // no pair is certain: every candidate is rescored
        b.measured = o.band < 0 && o.prec != EJOIN_FP32 ? 1 : 0;
        b.alias = alias ? 1 : 0;
        b.band_f = band_fp32_terms(Kp);
        b.band_rig = band;
        b.tiles_m = empty ? 0 : (int32_t)((u.R.rows + bp.bm - 1) / bp.bm);
        b.tiles_n = empty ? 0 : (int32_t)((u.S.rows + bp.bn - 1) / bp.bn);
        b.Kp_bytes = Kp * (int)eb;
        b.dim = dim;
        b.kg_last = last_slice_groups(o.prec, dim);
        b.user = order[q];
        b.tile_base = tile_base;
        b.chunk_tiles = 0;
        b.chunk_base = bp.n_chunks;
        if (batch_panel_tile(tile)) {
            // panel items: every 128-row panel over chunks of S tiles; the
            // prefilter keeps flat tile numbers for its statistics and
            // lists the chunks separately
            b.chunk_tiles = kPanelChunkTiles;
            const int64_t items =
                (int64_t)b.tiles_m * ((b.tiles_n + kPanelChunkTiles - 1) / kPanelChunkTiles);
            bp.n_chunks += items;
            tile_base += bp.approx ? (int64_t)b.tiles_m * b.tiles_n : items;
        } else {
            tile_base += (int64_t)b.tiles_m * b.tiles_n;
        }
        bp.pairs_total += u.R.rows * u.S.rows;
        if (empty) continue;
        band_default += std::max<int64_t>(65536, u.R.rows + u.S.rows);
        // operands: info_r, [info_s], xr, [xs]
        const size_t o_ir = off;
        off = align256(off + (size_t)padR * sizeof(RowInfo));
        size_t o_is = o_ir;
        if (!alias) {
            o_is = off;
            off = align256(off + (size_t)padS * sizeof(RowInfo));
        }
        const size_t o_xr = off;
        off = align256(off + (size_t)padR * Kp * eb);
        size_t o_xs = o_xr;
        if (!alias) {
            o_xs = off;
            off = align256(off + (size_t)padS * Kp * eb);
        }
        b.A = at(o_xr);
        b.B = at(o_xs);
        b.info_r = (const RowInfo*)at(o_ir);
        b.info_s = (const RowInfo*)at(o_is);
        auto seg = [&](const ejoin_rel& X, size_t o_x, size_t o_i, int64_t pad, int slot) {
            PrepSeg& g = G[nseg++];
            g.enorm_slot = slot;
            g.X = X.data;
            g.Xq = at(o_x);
            g.info = (RowInfo*)at(o_i);
            g.hdr = b.hdr;
            g.rows = X.rows;
            g.rows_pad = pad;
            g.ld = X.ld;
            g.row_base = row_base;
            g.dim = dim;
            g.Kp = Kp;
            row_base += pad;
        };
        rb_r[q] = row_base;
        seg(u.R, o_xr, o_ir, padR, H_ENORM_R);
        rb_s[q] = alias ? rb_r[q] : row_base;
        if (!alias) seg(u.S, o_xs, o_is, padS, H_ENORM_S);
    }
    bp.n_tiles = tile_base;
    bp.n_rows = row_base;
    if (bp.approx) {
        const size_t nr = (size_t)bp.n_rows;
        auto take = [&](size_t bytes) {
            const size_t at_ = off;
            off = align256(off + bytes);
            return at_;
        };
        // the network's hidden layer: learned pass only
        bp.off_hb = take(bp.exact ? 0 : nr * MLP_HIDDEN * 2);
        bp.off_u = take(nr * MLP_OUT * 4);
        bp.off_key = take(nr * 4);
        bp.off_pa = take(nr * 4);
        bp.off_pb = take(nr * 4);
        bp.off_hist = take(nr / 256 * 64 * 4);
        bp.off_offs = take(nr / 256 * 64 * 4);
        bp.kp = n > 0 && jobs ? padded_k(EJOIN_BF16, jobs[0].R.dim) : MLP_OUT;
        const size_t wid = bp.exact ? (size_t)bp.kp : (size_t)MLP_OUT;  // direction width
        bp.off_c = take(nr / 128 * MLP_OUT * 4);
        bp.off_rho = take(nr / 128 * 4);
        bp.off_cn = take(nr / 128 * 4);
        bp.off_alpha = take(nr / 128 * 4);
        bp.off_work = take((size_t)bp.n_tiles * 8);
        bp.off_proj = take((size_t)MLP_OUT * wid * 2);
        bp.off_ub = take(nr * MLP_OUT * 2);
        bp.off_up = take(nr * MLP_OUT * 2);
        bp.off_dir = take((nr / 128 + 128) * wid * 2);
        bp.off_m1 = take((size_t)bp.n_tiles * 4);
        bp.off_m2 = take((size_t)bp.n_tiles * 4);
        if (batch_panel_tile(tile)) {
            bp.off_keep = take((size_t)bp.n_tiles);
            bp.off_wmask = take((size_t)bp.n_chunks * 4);
        }
        for (int q = 0; q < n; ++q) {
            J[q].side_base = bp.n_side;
            bp.n_side += (int64_t)((J[q].tiles_m + 127) / 128) * J[q].tiles_n +
                         (int64_t)((J[q].tiles_n + 127) / 128) * J[q].tiles_m;
        }
        // anchors: rows drawn uniformly over the real rows of all relations
        int64_t real = 0;
        for (int i = 0; i < nseg; ++i) real += G[i].rows;
        bp.n_anchor = (int)std::min<int64_t>(kAnchors, real);
        bp.off_aidx = take((size_t)std::max(1, bp.n_anchor) * 8);
        bp.off_af = take((size_t)std::max(1, bp.n_anchor) * MLP_OUT * 4);
        bp.off_ab = take((size_t)((bp.n_anchor + 127) / 128 * 128 + 128) * MLP_OUT * 2);
        bp.off_lab = take((size_t)std::max(1, bp.n_anchor) * 4);
        bp.off_abits = take((size_t)std::max(1, bp.n_anchor) *
                            (size_t)pf_anchor_words(std::max(1, bp.n_anchor)) * 8);
        if (ws) {
            SplitMix64 rng{kAnchorSeed};
            bp.anchor_idx.resize(bp.n_anchor);
            for (int k = 0; k < bp.n_anchor; ++k) {
                int64_t r = (int64_t)rng.below((uint64_t)real);
                int i = 0;
                while (r >= G[i].rows) r -= G[i++].rows;
                bp.anchor_idx[k] = G[i].row_base + r;
            }
        }
        for (int q = 0; q < n; ++q) {
            J[q].perm_r = (const int32_t*)at(bp.off_pa + (size_t)rb_r[q] * 4);
            J[q].perm_s = (const int32_t*)at(bp.off_pa + (size_t)rb_s[q] * 4);
            J[q].rtile0 = rb_r[q] / 128;
            J[q].stile0 = rb_s[q] / 128;
        }
        for (int i = 0; i < nseg; ++i) G[i].perm = (const int32_t*)at(bp.off_pa + (size_t)G[i].row_base * 4);
    }
    bp.band_cap = o.band_capacity > 0 ? o.band_capacity : std::max<int64_t>(65536, band_default);
    bp.off_band = off;
    off = align256(off + (size_t)bp.band_cap * sizeof(int4));
    bp.total = off;

    BatchHead* h = bp.head();
    h->n_tiles = bp.n_tiles;
    h->n_rows = bp.n_rows;
    h->band_cap = bp.band_cap;
    h->band = (int4*)at(bp.off_band);
    h->n_out = n_out_dev;
    h->hdrs = (unsigned long long*)at(bp.off_hdrs);
    h->n_jobs = n;
    h->n_segs = nseg;
    if (bp.approx) {
        h->work = (const int64_t*)at(bp.off_work);
        h->n_side = bp.n_side;
        h->n_work = (const unsigned long long*)at(B_WORK * sizeof(unsigned long long));
        if (batch_panel_tile(tile)) {
            h->work_mask = (const uint32_t*)at(bp.off_wmask);
            h->n_chunks = bp.n_chunks;
        }
    }
    return EJOIN_OK;
}

int cu_count() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return n;
}

// The pass: table upload (by the caller), zero, prep, persistent tiles,
// rescore, counts.  Grids are fixed when `fixed` (graph capture).
hipError_t launch_pass(const BatchPlan& bp, char* ws, int tile_grid, bool fixed, hipStream_t st,
                       hipEvent_t* ev) {
    const BatchHead* head = (const BatchHead*)(ws + bp.off_table);
    const BatchJob* jobs = (const BatchJob*)(ws + bp.off_table + sizeof(BatchHead));
    const PrepSeg* segs = (const PrepSeg*)(ws + bp.off_table + sizeof(BatchHead) +
                                           (size_t)bp.table_jobs * sizeof(BatchJob));
    unsigned long long* bctr = (unsigned long long*)ws;
    hipError_t e;
    auto rec = [&](int i) { return ev ? hipEventRecord(ev[i], st) : hipSuccess; };
    if ((e = rec(0)) != hipSuccess) return e;
    if ((e = launch_batch_zero(head, bctr, st)) != hipSuccess) return e;
    // a captured pass may be replayed on deeper rows than its first batch
    const int kp_prep = fixed ? 1024 : bp.kp_max;
    if ((e = launch_batch_prep(bp.prec, kp_prep, head, segs, false, st)) != hipSuccess) return e;
    if ((e = launch_batch_band_edges(head, (BatchJob*)jobs, st)) != hipSuccess) return e;
    if ((e = rec(1)) != hipSuccess) return e;
    int tg = tile_grid;
    if (!fixed) tg = (int)std::max<int64_t>(1, std::min<int64_t>(tile_grid, bp.n_tiles));
    if ((e = launch_batch_tile(bp.tile, head, jobs, bctr, tg, st)) != hipSuccess) return e;
    if ((e = rec(2)) != hipSuccess) return e;
    int rg = kRescoreGrid;
    if (!fixed) rg = (int)std::max<int64_t>(1, std::min<int64_t>(kRescoreGrid, (bp.band_cap + 255) / 256));
    if ((e = launch_batch_rescore(head, jobs, bctr, rg, st)) != hipSuccess) return e;
    if ((e = rec(3)) != hipSuccess) return e;
    return launch_batch_counts(head, jobs, bctr, st);
}

// The pruned passes: codes and keys (learned: the network on rows prepared
// in input order; exact: the projection of the input rows), per-relation
// order, prep in that order, tile statistics and bounds (work list),
// persistent tiles over the work list, rescore, counts.
hipError_t launch_pass_approx(const BatchPlan& bp, char* ws, int tile_grid, const ejoin_opts& o,
                              hipStream_t st, hipEvent_t* ev) {
    const BatchHead* head = (const BatchHead*)(ws + bp.off_table);
    const BatchJob* jobs = (const BatchJob*)(ws + bp.off_table + sizeof(BatchHead));
    const PrepSeg* segs = (const PrepSeg*)(ws + bp.off_table + sizeof(BatchHead) +
                                           (size_t)bp.table_jobs * sizeof(BatchJob));
    unsigned long long* bctr = (unsigned long long*)ws;
    const int n_segs = ((const BatchHead*)bp.image.data())->n_segs;
    hipError_t e;
    auto rec = [&](int i) { return ev ? hipEventRecord(ev[i], st) : hipSuccess; };
    const int dim0 = bp.n_jobs ? ((const BatchJob*)(bp.image.data() + sizeof(BatchHead)))[0].dim : 1;
    ejoin_mlp_layout L;
    if (ejoin_mlp_layout_get(dim0, &L) != EJOIN_OK) return hipErrorInvalidValue;
    MlpDev m;
    if (!bp.exact) {
        char* b = (char*)o.prefilter;
        m.dim = L.dim;
        m.Dp = L.dim_pad;
        m.np = L.n_params;
        m.P = (float*)(b + L.off_params);
        m.W1t = (uint16_t*)(b + L.off_w1t);
        m.W2t = (uint16_t*)(b + L.off_w2t);
    }
    if ((e = rec(0)) != hipSuccess) return e;
    if ((e = launch_batch_zero(head, bctr, st)) != hipSuccess) return e;
    // the learned codes read prepared rows; the exact pass codes the
    // caller's rows directly and prepares them once, in the pruning order
    if (!bp.exact &&
        (e = launch_batch_prep(bp.prec, bp.kp_max, head, segs, false, st)) != hipSuccess)
        return e;
    int32_t* perm_a = (int32_t*)(ws + bp.off_pa);
    if (bp.exact) {
        // codes of the fixed projection, normalised
        if ((e = launch_xp_codes(head, segs, bp.n_rows, dim0, bp.kp,
                                 (uint16_t*)(ws + bp.off_proj), (float*)(ws + bp.off_u),
                                 (uint16_t*)(ws + bp.off_ub), st)) != hipSuccess)
            return e;
    } else if ((e = launch_pf_codes(head, segs, bp.n_rows, m, (uint16_t*)(ws + bp.off_hb),
                                    (float*)(ws + bp.off_u),
                                    (uint16_t*)(ws + bp.off_ub), st)) != hipSuccess) {
        return e;
    }
    if (bp.n_anchor > 0) {
        if ((e = hipMemcpyAsync(ws + bp.off_aidx, bp.anchor_idx.data(), bp.n_anchor * 8,
                                hipMemcpyHostToDevice, st)) != hipSuccess)
            return e;
        if ((e = launch_pf_keys(head, segs, bp.n_rows, (const float*)(ws + bp.off_u),
                                (const uint16_t*)(ws + bp.off_ub),
                                (const int64_t*)(ws + bp.off_aidx), bp.n_anchor, kAnchorTau,
                                (float*)(ws + bp.off_af), (uint16_t*)(ws + bp.off_ab),
                                (uint64_t*)(ws + bp.off_abits), (int32_t*)(ws + bp.off_lab),
                                (int32_t*)(ws + bp.off_key), st)) !=
            hipSuccess)
            return e;
    }
    if ((e = launch_pf_sort(head, segs, n_segs, bp.n_rows, (const int32_t*)(ws + bp.off_key),
                            perm_a, (int32_t*)(ws + bp.off_pb), (int32_t*)(ws + bp.off_hist),
                            (int32_t*)(ws + bp.off_offs), st)) != hipSuccess)
        return e;
    if ((e = launch_batch_prep(bp.prec, bp.kp_max, head, segs, true, st)) != hipSuccess) return e;
    if ((e = launch_batch_band_edges(head, (BatchJob*)jobs, st)) != hipSuccess) return e;
    if (bp.exact) {
        if ((e = launch_xp_tiles(head, segs, jobs, bp.n_rows, bp.kp, (uint16_t*)(ws + bp.off_dir),
                                 (float*)(ws + bp.off_alpha), (float*)(ws + bp.off_rho),
                                 (float*)(ws + bp.off_m1), (float*)(ws + bp.off_m2), bp.n_side,
                                 (int64_t*)(ws + bp.off_work), bctr + B_WORK, bp.n_tiles,
                                 batch_panel_tile(bp.tile) ? (uint8_t*)(ws + bp.off_keep)
                                                           : nullptr,
                                 st)) != hipSuccess)
            return e;
    } else if ((e = launch_pf_tiles(head, segs, jobs, bp.n_rows, (const float*)(ws + bp.off_u), perm_a,
                             (float*)(ws + bp.off_c), (float*)(ws + bp.off_rho),
                             (float*)(ws + bp.off_cn), (float*)(ws + bp.off_alpha),
                             (uint16_t*)(ws + bp.off_up), (uint16_t*)(ws + bp.off_dir),
                             (float*)(ws + bp.off_m1), (float*)(ws + bp.off_m2), bp.n_side,
                             o.prefilter_eps,
                             (int64_t*)(ws + bp.off_work), bctr + B_WORK, bp.n_tiles,
                             batch_panel_tile(bp.tile) ? (uint8_t*)(ws + bp.off_keep) : nullptr,
                             st)) !=
        hipSuccess)
        return e;
    if (batch_panel_tile(bp.tile) &&
        (e = launch_pf_chunks(head, jobs, (const uint8_t*)(ws + bp.off_keep),
                              (int64_t*)(ws + bp.off_work), (uint32_t*)(ws + bp.off_wmask),
                              bctr + B_WORK, bctr + B_KEPT, bp.n_chunks, st)) != hipSuccess)
        return e;
    if ((e = rec(1)) != hipSuccess) return e;
    const int tg = (int)std::max<int64_t>(1, std::min<int64_t>(tile_grid, bp.n_tiles));
    if ((e = launch_batch_tile(bp.tile, head, jobs, bctr, tg, st, true)) != hipSuccess) return e;
    if ((e = rec(2)) != hipSuccess) return e;
    const int rg =
        (int)std::max<int64_t>(1, std::min<int64_t>(kRescoreGrid, (bp.band_cap + 255) / 256));
    if ((e = launch_batch_rescore(head, jobs, bctr, rg, st)) != hipSuccess) return e;
    if ((e = rec(3)) != hipSuccess) return e;
    return launch_batch_counts(head, jobs, bctr, st);
}

}  // namespace

struct ejoin_batch_graph {
    int max_jobs = 0, tile = 0, tile_grid = 0;
    ejoin_opts opts;
    char* ws = nullptr;
    size_t ws_bytes = 0, off_table = 0, table_bytes = 0;
    void* staging = nullptr;  // pinned host copy of the job table
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool pending = false;
};

extern "C" {

size_t ejoin_batch_workspace(const ejoin_job* jobs, int32_t n_jobs, const ejoin_opts* opts) {
    ejoin_opts o = opts_or_default(opts);
    BatchPlan bp;
    const int tile = pick_batch_tile(o, jobs, std::max(0, (int)n_jobs));
    if (make_batch_plan(jobs, n_jobs, o, tile, std::max(1, (int)n_jobs), nullptr, nullptr, bp) !=
        EJOIN_OK)
        return 0;
    return bp.total;
}

ejoin_status ejoin_batch(const ejoin_job* jobs, int32_t n_jobs, const ejoin_opts* opts,
                         int64_t* n_out, void* ws, size_t ws_bytes, hipStream_t stream,
                         ejoin_stats* stats) {
    ejoin_opts o = opts_or_default(opts);
    if (n_jobs > 0 && !n_out) return EJOIN_E_INVAL;
    const bool sync = !(o.flags & EJOIN_NO_SYNC);
    const int tile = pick_batch_tile(o, jobs, std::max(0, (int)n_jobs));
    BatchPlan bp;
    ejoin_status s = make_batch_plan(jobs, n_jobs, o, tile, std::max(1, (int)n_jobs),
                                     (char*)ws, sync ? nullptr : n_out, bp);
    if (s != EJOIN_OK) return s;
    const int occ = batch_occupancy(tile);
    if (occ <= 0) return EJOIN_E_INVAL;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->ws_needed = bp.total;
        stats->band = bp.band_max;
        stats->tile = tile;
    }
    if (!ws || ws_bytes < bp.total) return EJOIN_E_WORKSPACE;
    if (n_jobs == 0) return EJOIN_OK;
    char* w = (char*)ws;
    // the table goes up with the pass; a pageable source is staged by the
    // runtime before this call returns
    HIP_TRY(hipMemcpyAsync(w + bp.off_table, bp.image.data(), bp.image.size(),
                           hipMemcpyHostToDevice, stream));
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    const bool timing = sync && (o.flags & EJOIN_TIMING) && stats;
    if (timing)
        for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    const int grid = cu_count() * occ;
    if (grid <= 0) return EJOIN_E_HIP;
    if (bp.approx)
        HIP_TRY(launch_pass_approx(bp, w, grid, o, stream, timing ? ev : nullptr));
    else
        HIP_TRY(launch_pass(bp, w, grid, false, stream, timing ? ev : nullptr));
    if (!sync) return EJOIN_OK;

    std::vector<unsigned long long> h((size_t)(n_jobs + 1) * H_COUNT);
    HIP_TRY(hipMemcpyAsync(h.data(), w, B_COUNT * 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(h.data() + H_COUNT, w + bp.off_hdrs, (size_t)n_jobs * H_COUNT * 8,
                           hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (timing) {
        hipEventElapsedTime(&stats->ms_prep, ev[0], ev[1]);
        hipEventElapsedTime(&stats->ms_main, ev[1], ev[2]);
        hipEventElapsedTime(&stats->ms_rescore, ev[2], ev[3]);
        hipEventElapsedTime(&stats->ms_total, ev[0], ev[3]);
        for (auto& e : ev) hipEventDestroy(e);
    }
    const unsigned long long band_found = h[B_BAND];
    ejoin_status st = EJOIN_OK;
    bool overflow = false, nonfinite = false, range = false;
    int64_t total = 0, acc = 0;
    const BatchJob* J = bp.jobs();
    for (int q = 0; q < n_jobs; ++q) {
        const unsigned long long* hj = h.data() + (size_t)(q + 1) * H_COUNT;
        const int u = J[q].user;
        n_out[u] = (int64_t)hj[H_OUT];
        if (hj[H_FLAGS] & F_NONFINITE) nonfinite = true;
        if (hj[H_FLAGS] & F_RANGE) range = true;
        if (hj[H_FLAGS]) n_out[u] = 0;
        if (n_out[u] > J[q].capacity) overflow = true;
        total += n_out[u];
        acc += (int64_t)hj[H_BAND_ACC];
    }
    if (stats) {
        stats->tiles_total = bp.n_tiles;
        stats->tiles_kept =
            bp.approx ? (int64_t)h[batch_panel_tile(bp.tile) ? B_KEPT : B_WORK] : bp.n_tiles;
        stats->n_pairs = total;
        stats->n_band = (int64_t)band_found;
        stats->n_band_accepted = acc;
        stats->n_certain = total - acc;
        stats->band_needed = (int64_t)band_found;
    }
    if (nonfinite) st = EJOIN_E_NONFINITE;
    else if (range) st = EJOIN_E_RANGE;
    else if ((int64_t)band_found > bp.band_cap) st = EJOIN_E_WORKSPACE;
    else if (overflow) st = EJOIN_E_OVERFLOW;
    return st;
}

ejoin_status ejoin_batch_graph_create(int32_t max_jobs, const ejoin_opts* opts, void* ws,
                                      size_t ws_bytes, hipStream_t stream,
                                      ejoin_batch_graph** graph) {
    if (!graph || max_jobs < 1 || max_jobs > 65536 || !ws) return EJOIN_E_INVAL;
    *graph = nullptr;
    ejoin_opts o = opts_or_default(opts);
    o.flags |= EJOIN_NO_SYNC;
    if (o.prec < EJOIN_FP32 || o.prec > EJOIN_FP8_E4M3) return EJOIN_E_INVAL;
    if (o.flags & (EJOIN_APPROX_PREFILTER | EJOIN_EXACT_PRUNE)) return EJOIN_E_UNSUPPORTED;
    const int tile = o.tile > 0 ? o.tile : batch_default_tile(o.prec);
    const TileDesc* td = tile_get(tile);
    if (!td || td->prec != o.prec || !batch_has_tile(tile)) return EJOIN_E_INVAL;
    const int occ = batch_occupancy(tile);
    const int grid = cu_count() * occ;
    if (grid <= 0) return EJOIN_E_INVAL;
    // an empty plan fixes the table position; launch() fills the rest
    BatchPlan bp;
    ejoin_status s = make_batch_plan(nullptr, 0, o, tile, max_jobs, (char*)ws, nullptr, bp);
    if (s != EJOIN_OK) return s;
    if (ws_bytes < bp.off_table + bp.table_bytes) return EJOIN_E_WORKSPACE;

    ejoin_batch_graph* g = new ejoin_batch_graph();
    g->max_jobs = max_jobs;
    g->tile = tile;
    g->tile_grid = grid;
    g->opts = o;
    g->opts.tile = tile;
    g->ws = (char*)ws;
    g->ws_bytes = ws_bytes;
    g->off_table = bp.off_table;
    g->table_bytes = bp.table_bytes;
    auto fail = [&](ejoin_status e) {
        ejoin_batch_graph_destroy(g);
        return e;
    };
    if (hipHostMalloc(&g->staging, g->table_bytes, hipHostMallocDefault) != hipSuccess) {
        g->staging = nullptr;
        return fail(EJOIN_E_HIP);
    }
    memset(g->staging, 0, g->table_bytes);
    if (hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess)
        return fail(EJOIN_E_HIP);
    batch_prep_query(bp.prec, 1024);  // device queries outside the capture
    if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(EJOIN_E_HIP);
    hipError_t e = hipMemcpyAsync(g->ws + g->off_table, g->staging, g->table_bytes,
                                  hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_pass(bp, g->ws, grid, true, stream, nullptr);
    hipGraph_t gr = nullptr;
    hipError_t e2 = hipStreamEndCapture(stream, &gr);
    g->graph = gr;
    if (e != hipSuccess || e2 != hipSuccess || !gr) return fail(EJOIN_E_HIP);
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess) {
        g->exec = nullptr;
        return fail(EJOIN_E_HIP);
    }
    *graph = g;
    return EJOIN_OK;
}

ejoin_status ejoin_batch_graph_launch(ejoin_batch_graph* g, const ejoin_job* jobs, int32_t n_jobs,
                                      int64_t* n_out, hipStream_t stream) {
    if (!g || n_jobs < 0 || n_jobs > g->max_jobs) return EJOIN_E_INVAL;
    if (n_jobs > 0 && !n_out) return EJOIN_E_INVAL;
    BatchPlan bp;
    ejoin_status s = make_batch_plan(jobs, n_jobs, g->opts, g->tile, g->max_jobs, g->ws, n_out, bp);
    if (s != EJOIN_OK) return s;
    if (bp.total > g->ws_bytes) return EJOIN_E_WORKSPACE;
    // the previous replay must have read the staging table before it changes
    if (g->pending && hipEventSynchronize(g->done) != hipSuccess) return EJOIN_E_HIP;
    g->pending = false;
    memcpy(g->staging, bp.image.data(), bp.image.size());
    HIP_TRY(hipGraphLaunch(g->exec, stream));
    HIP_TRY(hipEventRecord(g->done, stream));
    g->pending = true;
    return EJOIN_OK;
}

ejoin_status ejoin_batch_graph_destroy(ejoin_batch_graph* g) {
    if (!g) return EJOIN_OK;
    ejoin_status s = EJOIN_OK;
    if (g->pending && hipEventSynchronize(g->done) != hipSuccess) s = EJOIN_E_HIP;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    if (g->done) hipEventDestroy(g->done);
    if (g->staging) hipHostFree(g->staging);
    delete g;
    return s;
}

}  // extern "C"
