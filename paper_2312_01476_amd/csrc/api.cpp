// api.cpp -- the C ABI (include/ejoin.h): argument checks, the plan (padded
// sizes, band, tile), workspace carve-up and the launch sequence.
#include "plan.hpp"

#include <mutex>

using namespace ej;

namespace {

using namespace ej::plan;

struct Plan {
    int prec = 0, tile = 0, Kp = 0, dim = 0;
    bool alias = false;
    int64_t nR = 0, nS = 0, padR = 0, padS = 0;
    double band = 0.0;
    int64_t band_cap = 0;
    size_t off_info_r = 0, off_info_s = 0, off_xr = 0, off_xs = 0, off_band = 0, total = 0;
};

ejoin_status make_plan(const ejoin_rel* R, const ejoin_rel* S, const ejoin_opts* o, Plan& p,
                       bool may_alias = true) {
    if (!rel_ok(R) || !rel_ok(S) || R->dim != S->dim) return EJOIN_E_INVAL;
    if (o->prec < EJOIN_FP32 || o->prec > EJOIN_FP8_E4M3) return EJOIN_E_INVAL;
    p.prec = o->prec;
    p.dim = R->dim;
    if (p.dim > 65536) return EJOIN_E_UNSUPPORTED;
    p.Kp = padded_k(p.prec, p.dim);
    p.nR = R->rows;
    p.nS = S->rows;
    p.alias = may_alias && R->data == S->data && R->rows == S->rows && R->ld == S->ld;
    p.padR = padded_rows(p.nR);
    p.padS = p.alias ? p.padR : padded_rows(p.nS);
    const double rig = band_rigorous(p.prec, p.dim);
    if (o->band < 0) {
        p.band = rig;  // BF16 / FP8 single joins: narrowed on the device (threshold_run)
    } else {
        if (!(o->band >= rig) || !isfinite(o->band)) return EJOIN_E_INVAL;
        p.band = o->band;
    }
    p.tile = o->tile;
    if (p.tile <= 0) {
        // the tuner's measured choice for this shape when it has one that fits
        const int t = o->tuner ? tuner_pick(o->tuner, 0, p.prec, p.dim, (double)p.nR * p.nS) : 0;
        const TileDesc* td = t > 0 ? tile_get(t) : nullptr;
        const bool fits = td && td->prec == p.prec && t != 19 && t != 22 && t != kTileNlj &&
                          !(td->bm == 0 && !panel_fits(t, p.Kp * elem_bytes(p.prec)));
        p.tile = fits ? t : default_tile(p.prec, p.Kp);
    }
    const TileDesc* td = tile_get(p.tile);
    if (!td || td->prec != p.prec || p.tile == 19 || p.tile == 22)
        return EJOIN_E_INVAL;  // 19, 22: batches only
    if (p.tile == kTileNlj) {
        if (p.Kp > 1024) return EJOIN_E_UNSUPPORTED;
    } else if (td->bm == 0 && !panel_fits(p.tile, p.Kp * elem_bytes(p.prec))) {
        return EJOIN_E_INVAL;
    }
    p.band_cap = o->band_capacity > 0 ? o->band_capacity
                                      : std::max<int64_t>(1 << 16, p.nR + p.nS);
    const size_t eb = (size_t)elem_bytes(p.prec);
    size_t off = align256(H_COUNT * sizeof(unsigned long long));
    p.off_info_r = off;
    off = align256(off + (size_t)p.padR * sizeof(RowInfo));
    p.off_info_s = p.alias ? p.off_info_r : off;
    if (!p.alias) off = align256(off + (size_t)p.padS * sizeof(RowInfo));
    p.off_xr = off;
    off = align256(off + (size_t)p.padR * p.Kp * eb);
    p.off_xs = p.alias ? p.off_xr : off;
    if (!p.alias) off = align256(off + (size_t)p.padS * p.Kp * eb);
    p.off_band = off;
    off = align256(off + (size_t)p.band_cap * sizeof(int2));
    p.total = off;
    return EJOIN_OK;
}

// ---- top-k plan ----
struct TopkPlan {
    Plan base;      // prep part (no band list)
    int Kc = 0, n_pilot = 0;
    bool all_columns = false;
    bool panel = true;
    size_t off_nr = 0, off_ns = 0, off_cnt = 0, off_cand = 0, off_fb = 0, off_prow = 0,
           off_pkth = 0, off_keys = 0, off_counts = 0, off_order = 0, off_partv = 0,
           off_partj = 0, off_ref = 0, off_floor = 0, off_ca = 0, off_ci = 0, total = 0;
    int part_rows = 256;
    int64_t refine_rows = 0;  // rows one refinement pass gathers
};

ejoin_status make_topk_plan(const ejoin_rel* R, const ejoin_rel* S, int32_t k, const ejoin_opts* o,
                            TopkPlan& tp, bool may_alias = true) {
    if (k < 1) return EJOIN_E_INVAL;
    if (k > 256) return EJOIN_E_UNSUPPORTED;
    if (!rel_ok(R) || !rel_ok(S) || R->dim != S->dim) return EJOIN_E_INVAL;
    if (o->prec < EJOIN_FP32 || o->prec > EJOIN_FP8_E4M3) return EJOIN_E_INVAL;
    if ((o->flags & EJOIN_TOPK_MIN_SIM) && !isfinite(o->topk_min_sim)) return EJOIN_E_INVAL;
    ejoin_opts ob = *o;
    ob.tile = 0;
    ob.band = -1.0;
    ob.band_capacity = 1;
    ejoin_status s = make_plan(R, S, &ob, tp.base, may_alias);
    if (s != EJOIN_OK) return s;
    Plan& p = tp.base;
    // candidate sweep: register panels where the row depth has a panel form
    // and R fills the chip with 128-row panels (each panel sweeps all of S),
    // else the LDS tile kernel (any depth, one workgroup per 128 x 128 tile).
    // opts->tile forces a form: a panel tile of the precision, or its
    // 128 x 128 tile (1 FP32, 3 BF16, 5 FP8).
    const bool depth_ok = topk_panel_depth(p.prec, p.Kp * elem_bytes(p.prec));
    if (o->tile == 0) {
        tp.panel = depth_ok && p.nR >= 65536;
    } else {
        const TileDesc* td = tile_get(o->tile);
        if (!td || td->prec != p.prec) return EJOIN_E_INVAL;
        const bool square = o->tile == (p.prec == P_FP32 ? 1 : p.prec == P_BF16 ? 3 : 5);
        const bool panel = td->bm == 0 && o->tile != kTileNlj;
        if (!square && !(panel && depth_ok)) return EJOIN_E_INVAL;
        tp.panel = panel;
    }
    tp.Kc = o->topk_cand > 0 ? o->topk_cand : 256;
    if (tp.Kc < k) tp.Kc = k;
    if (tp.Kc > 256) return EJOIN_E_INVAL;
    tp.all_columns = p.nS <= tp.Kc;
    tp.n_pilot = (int)std::min<int64_t>(256, p.nR);
    size_t off = p.off_band;  // the band list is not used by top-k
    tp.off_nr = off;
    off = align256(off + (size_t)p.padR * sizeof(double));
    tp.off_ns = p.alias ? tp.off_nr : off;
    if (!p.alias) off = align256(off + (size_t)p.padS * sizeof(double));
    tp.off_cnt = off;
    off = align256(off + (size_t)p.padR * sizeof(int));
    tp.off_cand = off;
    off = align256(off + (size_t)p.padR * tp.Kc * sizeof(int2));
    tp.off_fb = off;
    off = align256(off + (size_t)p.padR * sizeof(int));
    tp.off_prow = off;
    off = align256(off + 256 * sizeof(int));
    tp.off_pkth = off;
    off = align256(off + 256 * sizeof(double));
    tp.off_keys = off;
    off = align256(off + (size_t)p.padR * sizeof(int));
    tp.off_counts = off;
    off = align256(off + (size_t)(p.nS + 1) * sizeof(int));
    tp.off_order = off;
    off = align256(off + (size_t)p.padR * sizeof(int));
    // partial lists of the exact scans: 256 rows x up to 64 S ranges x k
    tp.off_partv = off;
    off = align256(off + (size_t)tp.part_rows * 64 * k * sizeof(double));
    tp.off_partj = off;
    off = align256(off + (size_t)tp.part_rows * 64 * k * sizeof(int));
    // refinement of overflowed rows: their list, per-row floors, and their
    // prepared rows and row data gathered in passes of up to 65536 rows
    tp.refine_rows = std::min<int64_t>(p.padR, 65536);
    tp.off_ref = off;
    off = align256(off + (size_t)p.padR * sizeof(int));
    tp.off_floor = off;
    off = align256(off + (size_t)p.padR * sizeof(float));
    tp.off_ca = off;
    off = align256(off + (size_t)tp.refine_rows * p.Kp * elem_bytes(p.prec));
    tp.off_ci = off;
    off = align256(off + (size_t)tp.refine_rows * sizeof(RowInfo));
    tp.total = off;
    return EJOIN_OK;
}

// A selection pushed below the join: the positions 0..n-1 of the joined
// relation stand for the caller's rows ids[0..n-1].
struct SelArgs {
    const int32_t* r = nullptr;
    const int32_t* s = nullptr;
    int64_t src_r = 0, src_s = 0;  // rows of the caller's relations
};

// The relation a selection leaves (rows = selected count) and its checks.
bool sel_view(const ejoin_rel* X, const ejoin_sel* sel, ejoin_rel& v) {
    if (!X) return false;
    v = *X;
    if (!sel) return true;
    if (sel->n < 0 || sel->n > X->rows || (sel->n > 0 && !sel->ids)) return false;
    v.rows = sel->n;
    return true;
}

bool same_selection(const ejoin_sel* a, const ejoin_sel* b) {
    if (!a || !b) return a == b;
    return a->ids == b->ids && a->n == b->n;
}

}  // namespace

extern "C" {

const char* ejoin_version(void) { return "ejoin-gfx950 0.1.0"; }

const char* ejoin_strerror(ejoin_status s) {
    switch (s) {
        case EJOIN_OK: return "ok";
        case EJOIN_E_INVAL: return "invalid argument";
        case EJOIN_E_OVERFLOW: return "output capacity too small (n_out holds the true count)";
        case EJOIN_E_WORKSPACE: return "workspace too small";
        case EJOIN_E_NONFINITE: return "input row holds NaN or Inf";
        case EJOIN_E_HIP: return "HIP runtime error";
        case EJOIN_E_UNSUPPORTED: return "unsupported configuration";
        case EJOIN_E_RANGE: return "row norm outside [2^-100, 2^100]";
    }
    return "unknown status";
}

void ejoin_opts_default(ejoin_opts* o) {
    if (o) opts_init(o);
}

double ejoin_band_default(int32_t prec, int32_t dim) {
    if (prec < EJOIN_FP32 || prec > EJOIN_FP8_E4M3) return -1.0;
    return band_rigorous(prec, dim);
}

int32_t ejoin_tile_count(void) { return tile_count(); }

const char* ejoin_tile_name(int32_t tile) {
    if (tile == 0) return "auto";
    const TileDesc* t = tile_get(tile);
    return t ? t->name : nullptr;
}

ejoin_status ejoin_tile_occupancy(int32_t tile, int32_t dim, int32_t* designed,
                                  int32_t* resident) {
    if (!designed || !resident || dim < 1) return EJOIN_E_INVAL;
    int prec, form;
    switch (tile) {
        case 12: prec = P_BF16; form = 0; break;
        case 13: prec = P_FP8; form = 0; break;
        case 14: prec = P_BF16; form = 1; break;
        case 15: prec = P_FP8; form = 1; break;
        case 20: prec = P_FP32; form = 0; break;
        case 21: prec = P_FP32; form = 1; break;
        case 24: prec = P_BF16; form = 2; break;
        case 25: prec = P_FP8; form = 2; break;
        default: return EJOIN_E_INVAL;
    }
    // K padded to whole 128-byte slices, as the planner pads it
    const int per = 128 / (int)elem_bytes(prec);
    const int Kp = (dim + per - 1) / per * per;
    if (!panel_fits(tile, Kp * (int)elem_bytes(prec))) return EJOIN_E_INVAL;
    PanelQuery q = {0, 0, 0};
    if (panel_query(prec, form, Kp, &q) != hipSuccess) return EJOIN_E_INVAL;
    *designed = q.designed;
    *resident = q.resident;
    return EJOIN_OK;
}

size_t ejoin_threshold_workspace(const ejoin_rel* R, const ejoin_rel* S, const ejoin_opts* opts) {
    ejoin_opts o = opts_or_default(opts);
    Plan p;
    if (make_plan(R, S, &o, p) != EJOIN_OK) return 0;
    return p.total;
}

size_t ejoin_topk_workspace(const ejoin_rel* R, const ejoin_rel* S, int32_t k,
                            const ejoin_opts* opts) {
    ejoin_opts o = opts_or_default(opts);
    TopkPlan tp;
    if (make_topk_plan(R, S, k, &o, tp) != EJOIN_OK) return 0;
    return tp.total;
}

// Selections of a top-k join: the selected rows are first copied into
// compact buffers at the end of the workspace (offsets off_r, off_s), the
// join runs on those, and the S indices of the result are mapped back.
struct TopkGather {
    const ejoin_rel* R = nullptr;  // the caller's relations (null: no selection)
    const ejoin_rel* S = nullptr;
    const int32_t* sel_r = nullptr;
    const int32_t* sel_s = nullptr;  // null also when S is R with R's selection
    const int32_t* map_s = nullptr;  // result indices: selection positions -> S ids
    size_t off_r = 0, off_s = 0, total = 0;
};

static ejoin_status topk_run(const ejoin_rel* R, const ejoin_rel* S, int32_t k, const ejoin_opts& o,
                             const TopkPlan& tp, int32_t* out_idx, float* out_score, void* ws,
                             size_t ws_bytes, hipStream_t stream, ejoin_stats* stats,
                             const TopkGather& g) {
    const Plan& p = tp.base;
    const size_t need = g.total ? g.total : tp.total;
    const bool sync = !(o.flags & EJOIN_NO_SYNC);
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->ws_needed = need;
        stats->topk_slots = tp.Kc;
        // the sweep's form: the panel tile of the precision, or its 128 x 128 tile
        stats->tile = tp.panel ? (p.prec == P_BF16 ? 14 : p.prec == P_FP8 ? 13 : 21)
                               : (p.prec == P_BF16 ? 3 : p.prec == P_FP8 ? 5 : 1);
    }
    if (p.nR == 0) return EJOIN_OK;
    if (!out_idx || !out_score) return EJOIN_E_INVAL;
    if (!ws || ws_bytes < need) return EJOIN_E_WORKSPACE;

    char* w = (char*)ws;
    unsigned long long* hdr = (unsigned long long*)w;
    RowInfo* info_r = (RowInfo*)(w + p.off_info_r);
    RowInfo* info_s = (RowInfo*)(w + p.off_info_s);
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    const bool timing = sync && (o.flags & EJOIN_TIMING) && stats;
    if (timing)
        for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    auto rec = [&](int i) { return timing ? hipEventRecord(ev[i], stream) : hipSuccess; };

    HIP_TRY(rec(0));
    HIP_TRY(launch_zero_header(hdr, stream));
    ejoin_rel Rg = *R, Sg = *S;  // a selected side: its compact copy
    if (g.sel_r) {
        Rg.data = (const float*)(w + g.off_r);
        Rg.ld = p.dim;
        HIP_TRY(launch_gather_rows(g.R->data, g.R->ld, p.dim, g.sel_r, p.nR, g.R->rows,
                                   (float*)(w + g.off_r), hdr, stream));
    }
    if (p.alias) {
        Sg = Rg;
    } else if (g.sel_s) {
        Sg.data = (const float*)(w + g.off_s);
        Sg.ld = p.dim;
        HIP_TRY(launch_gather_rows(g.S->data, g.S->ld, p.dim, g.sel_s, p.nS, g.S->rows,
                                   (float*)(w + g.off_s), hdr, stream));
    }
    R = &Rg;
    S = &Sg;
    HIP_TRY(launch_prep(p.prec, R->data, p.nR, p.dim, R->ld, w + p.off_xr, p.Kp, p.padR, info_r,
                        hdr, H_ENORM_R, stream));
    if (!p.alias)
        HIP_TRY(launch_prep(p.prec, S->data, p.nS, p.dim, S->ld, w + p.off_xs, p.Kp, p.padS,
                            info_s, hdr, H_ENORM_S, stream));
    else
        HIP_TRY(hipMemcpyAsync(hdr + H_ENORM_S, hdr + H_ENORM_R, 8, hipMemcpyDeviceToDevice,
                               stream));
    double* nr64 = (double*)(w + tp.off_nr);
    double* ns64 = (double*)(w + tp.off_ns);
    HIP_TRY(launch_norms64(R->data, p.nR, p.dim, R->ld, nr64, stream));
    if (!p.alias) HIP_TRY(launch_norms64(S->data, p.nS, p.dim, S->ld, ns64, stream));

    TopkArgs ta;
    ta.R = R->data;
    ta.ldR = R->ld;
    ta.S = S->data;
    ta.ldS = S->ld;
    ta.dim = p.dim;
    ta.nR = p.nR;
    ta.nS = p.nS;
    ta.nr64 = nr64;
    ta.ns64 = ns64;
    ta.info_r = info_r;
    ta.cnt = (const int*)(w + tp.off_cnt);
    ta.cand = (const int2*)(w + tp.off_cand);
    ta.Kc = tp.Kc;
    ta.k = k;
    ta.fp32_terms = band_fp32_terms(p.Kp);
    ta.hdr = hdr;
    ta.fb_rows = (int*)(w + tp.off_fb);
    ta.pilot_rows = (int*)(w + tp.off_prow);
    ta.pilot_kth = (double*)(w + tp.off_pkth);
    ta.n_pilot = tp.n_pilot;
    ta.keys = (int*)(w + tp.off_keys);
    ta.counts = (int*)(w + tp.off_counts);
    ta.order = (int*)(w + tp.off_order);
    ta.part_v = (double*)(w + tp.off_partv);
    ta.part_j = (int*)(w + tp.off_partj);
    ta.part_rows = tp.part_rows;
    ta.all_columns = tp.all_columns;
    ta.out_idx = out_idx;
    ta.out_score = out_score;
    ta.min_sim = (o.flags & EJOIN_TOPK_MIN_SIM) ? o.topk_min_sim : -INFINITY;
    if (p.nS > 0) HIP_TRY(launch_topk_pilot(ta, stream));
    HIP_TRY(rec(1));

    if (p.nS > 0) {
        CandArgs ca;
        ca.A = w + p.off_xr;
        ca.B = w + p.off_xs;
        ca.info_r = info_r;
        ca.info_s = info_s;
        ca.Kp = p.Kp;
        ca.nR = p.nR;
        ca.nS = p.nS;
        ca.hdr = hdr;
        ca.cnt = (int*)(w + tp.off_cnt);
        ca.cand = (int2*)(w + tp.off_cand);
        ca.Kc = tp.Kc;
        if (tp.panel) {
            HIP_TRY(launch_topk_candidates(p.prec, ca, stream));
        } else {
            HIP_TRY(launch_fill_int(ca.cnt, p.padR, 0, stream));
            HIP_TRY(launch_topk_candidates_tile(p.prec, ca, stream));
        }
    }
    HIP_TRY(rec(2));
    HIP_TRY(launch_topk_finalize(ta, stream));
    if (!sync) {
        HIP_TRY(launch_topk_fallback(ta, -1, stream));
        HIP_TRY(launch_map_topk(out_idx, p.nR * k, g.map_s, p.nS, hdr, stream));
        return EJOIN_OK;
    }
    unsigned long long h[H_COUNT];
    HIP_TRY(hipMemcpyAsync(h, hdr, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    int64_t n_refined = 0;
    if (h[H_FLAGS] == 0 && h[H_TOPK_FB] > 0 && !tp.all_columns) {
        // rows that failed the certificate: those whose slots overflowed are
        // swept again with a floor of their own, then certified again
        const int64_t n_fb = (int64_t)h[H_TOPK_FB];
        int* ref = (int*)(w + tp.off_ref);
        float* floors = (float*)(w + tp.off_floor);
        HIP_TRY(hipMemcpyAsync(ref, ta.fb_rows, (size_t)n_fb * sizeof(int),
                               hipMemcpyDeviceToDevice, stream));
        HIP_TRY(launch_fill_int((int*)(hdr + H_TOPK_FB), 2, 0, stream));
        HIP_TRY(launch_topk_refine_floor(ta, ref, n_fb, floors, stream));
        const int kpb = p.Kp * elem_bytes(p.prec);
        for (int64_t b0 = 0; b0 < n_fb; b0 += tp.refine_rows) {
            const int64_t nb = std::min<int64_t>(tp.refine_rows, n_fb - b0);
            const int64_t nb_pad = (nb + 127) / 128 * 128;
            HIP_TRY(launch_gather_prepared(w + p.off_xr, kpb, ref + b0, nb, nb_pad, w + tp.off_ca,
                                           stream));
            HIP_TRY(launch_gather_prepared(info_r, (int)sizeof(RowInfo), ref + b0, nb, nb_pad,
                                           w + tp.off_ci, stream));
            CandArgs cr;
            cr.A = w + tp.off_ca;
            cr.B = w + p.off_xs;
            cr.info_r = (const RowInfo*)(w + tp.off_ci);
            cr.info_s = info_s;
            cr.Kp = p.Kp;
            cr.nR = nb;
            cr.nS = p.nS;
            cr.hdr = hdr;
            cr.cnt = (int*)(w + tp.off_cnt);
            cr.cand = (int2*)(w + tp.off_cand);
            cr.Kc = tp.Kc;
            cr.row_map = ref + b0;
            cr.floors = floors + b0;
            HIP_TRY(launch_topk_candidates_tile(p.prec, cr, stream));
        }
        HIP_TRY(launch_topk_finalize_rows(ta, ref, n_fb, floors, stream));
        HIP_TRY(hipMemcpyAsync(h, hdr, sizeof(h), hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        n_refined = n_fb;
    }
    if (h[H_FLAGS] == 0) {
        HIP_TRY(launch_topk_fallback(ta, (int64_t)h[H_TOPK_FB], stream));
        HIP_TRY(launch_map_topk(out_idx, p.nR * k, g.map_s, p.nS, hdr, stream));
    }
    HIP_TRY(rec(3));
    HIP_TRY(hipStreamSynchronize(stream));
    if (timing) {
        hipEventElapsedTime(&stats->ms_prep, ev[0], ev[1]);
        hipEventElapsedTime(&stats->ms_main, ev[1], ev[2]);
        hipEventElapsedTime(&stats->ms_rescore, ev[2], ev[3]);
        hipEventElapsedTime(&stats->ms_total, ev[0], ev[3]);
        for (auto& e : ev) hipEventDestroy(e);
    }
    if (h[H_FLAGS] & F_BADSEL) return EJOIN_E_INVAL;
    if (h[H_FLAGS] & F_NONFINITE) return EJOIN_E_NONFINITE;
    if (h[H_FLAGS] & F_RANGE) return EJOIN_E_RANGE;
    if (stats) {
        stats->n_fallback = (int32_t)h[H_TOPK_FB];
        stats->topk_refined = n_refined;
        stats->topk_floor = (double)__builtin_bit_cast(float, (uint32_t)h[H_TOPK_F]);
        stats->band = (double)__builtin_bit_cast(float, (uint32_t)h[H_TOPK_EMAX]);
    }
    return EJOIN_OK;
}

ejoin_status ejoin_topk(const ejoin_rel* R, const ejoin_rel* S, int32_t k, const ejoin_opts* opts,
                        int32_t* out_idx, float* out_score, void* ws, size_t ws_bytes,
                        hipStream_t stream, ejoin_stats* stats) {
    ejoin_opts o = opts_or_default(opts);
    TopkPlan tp;
    ejoin_status s = make_topk_plan(R, S, k, &o, tp);
    if (s != EJOIN_OK) return s;
    return topk_run(R, S, k, o, tp, out_idx, out_score, ws, ws_bytes, stream, stats, TopkGather());
}

// plan of a top-k join over selections: the join's own plan on the selected
// row counts, then the two compact copies
static ejoin_status topk_sel_plan(const ejoin_rel* R, const ejoin_sel* sel_r, const ejoin_rel* S,
                                  const ejoin_sel* sel_s, int32_t k, const ejoin_opts& o,
                                  ejoin_rel& Rv, ejoin_rel& Sv, TopkPlan& tp, TopkGather& g) {
    if (!sel_view(R, sel_r, Rv) || !sel_view(S, sel_s, Sv)) return EJOIN_E_INVAL;
    ejoin_status s = make_topk_plan(&Rv, &Sv, k, &o, tp, same_selection(sel_r, sel_s));
    if (s != EJOIN_OK) return s;
    if (!sel_r && !sel_s) return EJOIN_OK;  // nothing to gather
    const Plan& p = tp.base;
    g.R = R;
    g.S = S;
    g.sel_r = sel_r ? sel_r->ids : nullptr;
    g.sel_s = sel_s && !p.alias ? sel_s->ids : nullptr;
    g.map_s = sel_s ? sel_s->ids : nullptr;
    size_t off = align256(tp.total);
    g.off_r = off;
    if (g.sel_r) off = align256(off + (size_t)p.nR * p.dim * 4);
    g.off_s = off;
    if (g.sel_s) off = align256(off + (size_t)p.nS * p.dim * 4);
    g.total = off;
    return EJOIN_OK;
}

size_t ejoin_topk_sel_workspace(const ejoin_rel* R, const ejoin_sel* sel_r, const ejoin_rel* S,
                                const ejoin_sel* sel_s, int32_t k, const ejoin_opts* opts) {
    ejoin_opts o = opts_or_default(opts);
    ejoin_rel Rv, Sv;
    TopkPlan tp;
    TopkGather g;
    if (topk_sel_plan(R, sel_r, S, sel_s, k, o, Rv, Sv, tp, g) != EJOIN_OK) return 0;
    return g.total ? g.total : tp.total;
}

ejoin_status ejoin_topk_sel(const ejoin_rel* R, const ejoin_sel* sel_r, const ejoin_rel* S,
                            const ejoin_sel* sel_s, int32_t k, const ejoin_opts* opts,
                            int32_t* out_idx, float* out_score, void* ws, size_t ws_bytes,
                            hipStream_t stream, ejoin_stats* stats) {
    ejoin_opts o = opts_or_default(opts);
    ejoin_rel Rv, Sv;
    TopkPlan tp;
    TopkGather g;
    ejoin_status s = topk_sel_plan(R, sel_r, S, sel_s, k, o, Rv, Sv, tp, g);
    if (s != EJOIN_OK) return s;
    return topk_run(&Rv, &Sv, k, o, tp, out_idx, out_score, ws, ws_bytes, stream, stats, g);
}

}  // extern "C"

namespace {

// The threshold join on a workspace that is already known to be large enough
// for plan p (both entry points below check that first).
ejoin_status threshold_run(const ejoin_rel* R, const ejoin_rel* S, double theta,
                           const ejoin_opts& o, const Plan& p, ejoin_pair* out, int64_t capacity,
                           int64_t* n_out, void* ws, hipStream_t stream, ejoin_stats* stats,
                           const SelArgs& sel = SelArgs()) {
    const bool sync = !(o.flags & EJOIN_NO_SYNC);
    if (p.nR == 0 || p.nS == 0) {
        if (sync) {
            *n_out = 0;
        } else {
            // still need a defined device count
            unsigned long long* hdr = (unsigned long long*)ws;
            HIP_TRY(launch_zero_header(hdr, stream));
            HIP_TRY(launch_copy_count(hdr, p.band_cap, n_out, stream));
        }
        return EJOIN_OK;
    }

    char* w = (char*)ws;
    unsigned long long* hdr = (unsigned long long*)w;
    RowInfo* info_r = (RowInfo*)(w + p.off_info_r);
    RowInfo* info_s = (RowInfo*)(w + p.off_info_s);
    void* xr = w + p.off_xr;
    void* xs = w + p.off_xs;
    int2* band = (int2*)(w + p.off_band);

    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    const bool timing = sync && (o.flags & EJOIN_TIMING) && stats;
    if (timing)
        for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
    auto rec = [&](int i) { return timing ? hipEventRecord(ev[i], stream) : hipSuccess; };

    HIP_TRY(rec(0));
    HIP_TRY(launch_zero_header(hdr, stream));
    HIP_TRY(launch_prep(p.prec, R->data, p.nR, p.dim, R->ld, xr, p.Kp, p.padR, info_r, hdr,
                        H_ENORM_R, stream, sel.r, sel.src_r));
    if (!p.alias)
        HIP_TRY(launch_prep(p.prec, S->data, p.nS, p.dim, S->ld, xs, p.Kp, p.padS, info_s, hdr,
                            H_ENORM_S, stream, sel.s, sel.src_s));
    HIP_TRY(rec(1));

    ThresholdArgs a;
    a.A = xr;
    a.B = xs;
    a.info_r = info_r;
    a.info_s = info_s;
    a.Kp = p.Kp;
    a.nR = p.nR;
    a.nS = p.nS;
    a.lo = round_down_f(theta - p.band);
    a.hi = round_up_f(theta + p.band);
    // the default band of the narrow formats: measured on the device from the
    // rows' quantisation error norms (never wider than the rigorous bound)
    const bool measured = o.band < 0 && p.prec != P_FP32;
    const bool all64 = (o.flags & EJOIN_FP64_SCORES) != 0;
    if (all64) a.hi = INFINITY;  // no pair is certain: every candidate is rescored
    if (measured) {
        HIP_TRY(launch_band_edges(hdr, theta, band_fp32_terms(p.Kp), p.band, p.alias, all64,
                                  stream));
        a.lohi = hdr + H_LO;
    }
    a.out = (Pair*)out;
    a.capacity = capacity;
    a.band = band;
    a.band_cap = p.band_cap;
    a.hdr = hdr;
    a.kg_last = last_slice_groups(p.prec, p.dim);
    HIP_TRY(launch_threshold(p.tile, a, stream));
    HIP_TRY(rec(2));
    HIP_TRY(launch_rescore_band(R->data, R->ld, S->data, S->ld, p.dim, band, p.band_cap, theta,
                                (Pair*)out, capacity, hdr, stream, sel.r, sel.s));
    HIP_TRY(launch_map_pairs((Pair*)out, capacity, hdr, sel.r, sel.s, stream));
    HIP_TRY(rec(3));

    if (!sync) {
        HIP_TRY(launch_copy_count(hdr, p.band_cap, n_out, stream));
        return EJOIN_OK;
    }
    unsigned long long h[H_COUNT];
    HIP_TRY(hipMemcpyAsync(h, hdr, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (timing) {
        hipEventElapsedTime(&stats->ms_prep, ev[0], ev[1]);
        hipEventElapsedTime(&stats->ms_main, ev[1], ev[2]);
        hipEventElapsedTime(&stats->ms_rescore, ev[2], ev[3]);
        hipEventElapsedTime(&stats->ms_total, ev[0], ev[3]);
        for (auto& e : ev) hipEventDestroy(e);
    }
    if (h[H_FLAGS] & F_BADSEL) return EJOIN_E_INVAL;
    if (h[H_FLAGS] & F_NONFINITE) return EJOIN_E_NONFINITE;
    if (h[H_FLAGS] & F_RANGE) return EJOIN_E_RANGE;
    *n_out = (int64_t)h[H_OUT];
    if (stats) {
        if (measured) stats->band = __builtin_bit_cast(double, (uint64_t)h[H_BAND_W]);
        stats->n_pairs = (int64_t)h[H_OUT];
        stats->n_band = (int64_t)h[H_BAND];
        stats->n_band_accepted = (int64_t)h[H_BAND_ACC];
        stats->n_certain = stats->n_pairs - stats->n_band_accepted;
        stats->band_needed = (int64_t)h[H_BAND];
    }
    if ((int64_t)h[H_BAND] > p.band_cap) return EJOIN_E_WORKSPACE;
    if ((int64_t)h[H_OUT] > capacity) return EJOIN_E_OVERFLOW;
    return EJOIN_OK;
}

ejoin_status threshold_args(const ejoin_rel* R, const ejoin_rel* S, double theta,
                            const ejoin_opts& o, ejoin_pair* out, int64_t capacity,
                            int64_t* n_out, Plan& p, ejoin_stats* stats, bool may_alias = true) {
    if (!isfinite(theta) || capacity < 0 || !n_out) return EJOIN_E_INVAL;
    if (capacity > 0 && !out) return EJOIN_E_INVAL;
    ejoin_status s = make_plan(R, S, &o, p, may_alias);
    if (s != EJOIN_OK) return s;
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        stats->ws_needed = p.total;
        stats->band = p.band;
        stats->tile = p.tile;
    }
    return EJOIN_OK;
}

// ---- the allocation-free variant's scratch ----
// One array per GPU in the library's code object, resident until the process
// ends.  Host code never passes `scratch` itself to a kernel: its device
// address is looked up once per device (hipGetSymbolAddress with that device
// current) and only that address is used.
static __device__ __align__(256) unsigned char scratch[EJOIN_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (nullptr on failure).
void* scratch_address() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

ejoin_status ejoin_threshold(const ejoin_rel* R, const ejoin_rel* S, double theta,
                             const ejoin_opts* opts, ejoin_pair* out, int64_t capacity,
                             int64_t* n_out, void* ws, size_t ws_bytes, hipStream_t stream,
                             ejoin_stats* stats) {
    ejoin_opts o = opts_or_default(opts);
    Plan p;
    ejoin_status s = threshold_args(R, S, theta, o, out, capacity, n_out, p, stats);
    if (s != EJOIN_OK) return s;
    if (!ws || ws_bytes < p.total) return EJOIN_E_WORKSPACE;
    return threshold_run(R, S, theta, o, p, out, capacity, n_out, ws, stream, stats);
}

ejoin_status ejoin_threshold_noalloc(const ejoin_rel* R, const ejoin_rel* S, double theta,
                                     const ejoin_opts* opts, ejoin_pair* out, int64_t capacity,
                                     int64_t* n_out, hipStream_t stream, ejoin_stats* stats) {
    ejoin_opts o = opts_or_default(opts);
    o.flags &= ~EJOIN_TIMING;  // timing would create events
    Plan p;
    ejoin_status s = threshold_args(R, S, theta, o, out, capacity, n_out, p, stats);
    if (s != EJOIN_OK) return s;
    if (p.total > (size_t)EJOIN_NOALLOC_SCRATCH_BYTES) return EJOIN_E_WORKSPACE;
    void* ws = scratch_address();
    if (!ws) return EJOIN_E_HIP;
    return threshold_run(R, S, theta, o, p, out, capacity, n_out, ws, stream, stats);
}

size_t ejoin_noalloc_scratch_bytes(void) { return (size_t)EJOIN_NOALLOC_SCRATCH_BYTES; }

size_t ejoin_threshold_sel_workspace(const ejoin_rel* R, const ejoin_sel* sel_r,
                                     const ejoin_rel* S, const ejoin_sel* sel_s,
                                     const ejoin_opts* opts) {
    ejoin_opts o = opts_or_default(opts);
    ejoin_rel Rv, Sv;
    Plan p;
    if (!sel_view(R, sel_r, Rv) || !sel_view(S, sel_s, Sv)) return 0;
    if (make_plan(&Rv, &Sv, &o, p, same_selection(sel_r, sel_s)) != EJOIN_OK) return 0;
    return p.total;
}

ejoin_status ejoin_threshold_sel(const ejoin_rel* R, const ejoin_sel* sel_r, const ejoin_rel* S,
                                 const ejoin_sel* sel_s, double theta, const ejoin_opts* opts,
                                 ejoin_pair* out, int64_t capacity, int64_t* n_out, void* ws,
                                 size_t ws_bytes, hipStream_t stream, ejoin_stats* stats) {
    ejoin_opts o = opts_or_default(opts);
    ejoin_rel Rv, Sv;
    if (!sel_view(R, sel_r, Rv) || !sel_view(S, sel_s, Sv)) return EJOIN_E_INVAL;
    Plan p;
    ejoin_status s = threshold_args(&Rv, &Sv, theta, o, out, capacity, n_out, p, stats,
                                    same_selection(sel_r, sel_s));
    if (s != EJOIN_OK) return s;
    if (!ws || ws_bytes < p.total) return EJOIN_E_WORKSPACE;
    SelArgs sa;
    sa.r = sel_r ? sel_r->ids : nullptr;
    sa.s = sel_s ? sel_s->ids : nullptr;
    sa.src_r = R->rows;
    sa.src_s = S->rows;
    return threshold_run(&Rv, &Sv, theta, o, p, out, capacity, n_out, ws, stream, stats, sa);
}

size_t ejoin_select_workspace(void) { return select_range_workspace(); }

ejoin_status ejoin_select_range(const float* col, int64_t n, float lo, float hi, int32_t* ids,
                                int64_t* n_sel, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n < 0 || n > 0x7fffffffLL || !n_sel || isnan(lo) || isnan(hi)) return EJOIN_E_INVAL;
    if (n > 0 && (!col || !ids)) return EJOIN_E_INVAL;
    if (!ws || ws_bytes < select_range_workspace()) return EJOIN_E_WORKSPACE;
    HIP_TRY(launch_select_range(col, n, lo, hi, ids, n_sel, ws, stream));
    return EJOIN_OK;
}

}  // extern "C"
