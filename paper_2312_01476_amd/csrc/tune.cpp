// tune.cpp -- the autotuner: tile shapes measured on the caller's data and
// kept in a caller-owned table keyed by (single or batch, precision, padded
// depth, size bucket).
#include <hip/hip_runtime.h>
#include <stdio.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "plan.hpp"

using namespace ej;
using namespace ej::plan;

struct ejoin_tuner {
    // (batch, prec, Kp, bucket) -> tile id
    std::map<std::tuple<int, int, int, int>, int> best;
};

namespace {

int size_bucket(double pairs) {
    if (!(pairs >= 1.0)) return 0;
    return (int)floor(log(pairs) / log(4.0));
}

bool tile_runs(int tile, int prec, int Kp, bool batch) {
    const TileDesc* td = tile_get(tile);
    if (!td || td->prec != prec) return false;
    if (batch)
        return td->bm != 0 && batch_has_tile(tile) &&
               ((tile != 19 && tile != 22) || batch_panel_depth(Kp * elem_bytes(prec)));
    if (tile == 19 || tile == 22) return false;  // batch-only forms
    if (tile == kTileNlj) return false;          // the comparator is never tuned
    return !(td->bm == 0 && !panel_fits(tile, Kp * elem_bytes(prec)));
}

}  // namespace

namespace ej {
namespace plan {

int tuner_pick(const ejoin_tuner* t, int batch, int prec, int dim, double pairs) {
    if (!t) return 0;
    const int Kp = padded_k(prec, dim);
    const int b = size_bucket(pairs);
    // exact bucket, else the nearest measured bucket of the same shape class
    int best = 0, dist = 1 << 30;
    for (const auto& kv : t->best) {
        int kb, kp, kk, kbu;
        std::tie(kb, kp, kk, kbu) = kv.first;
        if (kb != (batch ? 1 : 0) || kp != prec || kk != Kp) continue;
        const int d = std::abs(kbu - b);
        if (d < dist) {
            dist = d;
            best = kv.second;
        }
    }
    return best;
}

}  // namespace plan
}  // namespace ej

extern "C" {

ejoin_tuner* ejoin_tuner_create(void) { return new ejoin_tuner(); }

void ejoin_tuner_destroy(ejoin_tuner* t) { delete t; }

int32_t ejoin_tuner_lookup(const ejoin_tuner* t, int32_t batch, int32_t prec, int32_t dim,
                           double pairs) {
    if (!t || dim < 1 || prec < EJOIN_FP32 || prec > EJOIN_FP8_E4M3) return 0;
    return tuner_pick(t, batch, prec, dim, pairs);
}

ejoin_status ejoin_tuner_save(const ejoin_tuner* t, const char* path) {
    if (!t || !path) return EJOIN_E_INVAL;
    FILE* f = fopen(path, "w");
    if (!f) return EJOIN_E_INVAL;
    fprintf(f, "# ejoin tuner v1: batch prec Kp bucket tile name\n");
    for (const auto& kv : t->best) {
        int b, p, k, bu;
        std::tie(b, p, k, bu) = kv.first;
        const TileDesc* td = tile_get(kv.second);
        fprintf(f, "%d %d %d %d %d %s\n", b, p, k, bu, kv.second, td ? td->name : "?");
    }
    const bool ok = fclose(f) == 0;
    return ok ? EJOIN_OK : EJOIN_E_INVAL;
}

ejoin_status ejoin_tuner_load(ejoin_tuner* t, const char* path) {
    if (!t || !path) return EJOIN_E_INVAL;
    FILE* f = fopen(path, "r");
    if (!f) return EJOIN_E_INVAL;
    char line[256];
    std::map<std::tuple<int, int, int, int>, int> m;
    ejoin_status s = EJOIN_OK;
    while (fgets(line, sizeof(line), f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        int b, p, k, bu, tile;
        if (sscanf(line, "%d %d %d %d %d", &b, &p, &k, &bu, &tile) != 5 || (b != 0 && b != 1) ||
            !tile_runs(tile, p, k, b == 1)) {
            s = EJOIN_E_INVAL;
            break;
        }
        m[std::make_tuple(b, p, k, bu)] = tile;
    }
    fclose(f);
    if (s == EJOIN_OK)
        for (const auto& kv : m) t->best[kv.first] = kv.second;
    return s;
}

ejoin_status ejoin_autotune(ejoin_tuner* t, const ejoin_job* jobs, int32_t n_jobs,
                            const ejoin_opts* opts, void* ws, size_t ws_bytes, hipStream_t stream,
                            int32_t reps, int32_t* best_tile, float* ms) {
    if (n_jobs < 1 || !jobs || !best_tile || reps < 1 || reps > 1000) return EJOIN_E_INVAL;
    ejoin_opts o = opts_or_default(opts);
    o.flags &= ~(EJOIN_NO_SYNC | EJOIN_TIMING);
    const bool batch = n_jobs > 1;
    const int dim = jobs[0].R.dim;
    if (dim < 1) return EJOIN_E_INVAL;
    const int Kp = padded_k(o.prec, dim);
    double pairs = 0.0;
    for (int i = 0; i < n_jobs; ++i) pairs += (double)jobs[i].R.rows * (double)jobs[i].S.rows;
    const int nt = tile_count();
    if (ms)
        for (int i = 0; i <= nt; ++i) ms[i] = -1.0f;
    std::vector<int64_t> counts((size_t)n_jobs);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return EJOIN_E_HIP;
    }
    int best = 0;
    float best_ms = 0.0f;
    ejoin_status last = EJOIN_E_UNSUPPORTED;
    for (int tile = 1; tile <= nt; ++tile) {
        if (!tile_runs(tile, o.prec, Kp, batch)) continue;
        o.tile = tile;
        auto call = [&]() -> ejoin_status {
            if (batch) return ejoin_batch(jobs, n_jobs, &o, counts.data(), ws, ws_bytes, stream,
                                          nullptr);
            return ejoin_threshold(&jobs[0].R, &jobs[0].S, jobs[0].theta, &o, jobs[0].out,
                                   jobs[0].capacity, counts.data(), ws, ws_bytes, stream, nullptr);
        };
        ejoin_status s = call();  // warm-up; an overflowing output still does all the work
        if (s != EJOIN_OK && s != EJOIN_E_OVERFLOW) {
            last = s;
            continue;
        }
        std::vector<float> v;
        for (int r = 0; r < reps && s != EJOIN_E_HIP; ++r) {
            if (hipEventRecord(e0, stream) != hipSuccess) { s = EJOIN_E_HIP; break; }
            s = call();
            if (s != EJOIN_OK && s != EJOIN_E_OVERFLOW) break;
            if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
                s = EJOIN_E_HIP;
                break;
            }
            float x = 0.0f;
            hipEventElapsedTime(&x, e0, e1);
            v.push_back(x);
        }
        if (s != EJOIN_OK && s != EJOIN_E_OVERFLOW) {
            last = s;
            continue;
        }
        std::sort(v.begin(), v.end());
        const float med = v[v.size() / 2];
        if (ms) ms[tile] = med;
        if (best == 0 || med < best_ms) {
            best = tile;
            best_ms = med;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (best == 0) return last;
    *best_tile = best;
    if (t) t->best[std::make_tuple(batch ? 1 : 0, (int)o.prec, Kp, size_bucket(pairs))] = best;
    return EJOIN_OK;
}

}  // extern "C"
