// api_mlp.cpp -- C ABI of the prefilter network: state layout, init,
// training step and inference.
#include <hip/hip_runtime.h>

#include <stdio.h>

#include <vector>

#include "batch.hpp"
#include "mlp.hpp"
#include "plan.hpp"

using namespace ej;
using namespace ej::plan;

namespace {

bool layout_of(int32_t dim, ejoin_mlp_layout& L) {
    if (dim < 1 || dim > 1024) return false;
    memset(&L, 0, sizeof(L));
    L.dim = dim;
    L.dim_pad = ((dim + 63) / 64) * 64;
    L.n_params = (int64_t)dim * MLP_HIDDEN + MLP_HIDDEN + (int64_t)MLP_HIDDEN * MLP_OUT + MLP_OUT;
    size_t off = 0;
    const size_t pv = align256((size_t)L.n_params * 4);
    L.off_params = off;
    off += pv;
    L.off_grads = off;
    off += pv;
    L.off_m = off;
    off += pv;
    L.off_v = off;
    off += pv;
    L.off_w1t = off;
    off = align256(off + (size_t)MLP_HIDDEN * L.dim_pad * 2);
    L.off_w2t = off;
    off = align256(off + (size_t)MLP_OUT * MLP_HIDDEN * 2);
    L.off_step = off;
    off = align256(off + 8);
    L.total = off;
    return true;
}

MlpDev dev_of(void* state, const ejoin_mlp_layout& L) {
    char* b = (char*)state;
    MlpDev m;
    m.dim = L.dim;
    m.Dp = L.dim_pad;
    m.np = L.n_params;
    m.P = (float*)(b + L.off_params);
    m.G = (float*)(b + L.off_grads);
    m.M = (float*)(b + L.off_m);
    m.V = (float*)(b + L.off_v);
    m.W1t = (uint16_t*)(b + L.off_w1t);
    m.W2t = (uint16_t*)(b + L.off_w2t);
    m.step = (int64_t*)(b + L.off_step);
    return m;
}

size_t train_ws(int dim_pad, int batch) {
    const size_t r2 = 2 * (size_t)batch;
    return align256(r2 * dim_pad * 4) + 2 * align256(r2 * MLP_HIDDEN * 4) +
           2 * align256(r2 * MLP_OUT * 4);
}

size_t fwd_ws(int64_t n) {
    const size_t rows = (size_t)((n + 127) / 128) * 128;
    return align256(rows * MLP_HIDDEN * 2) + align256(rows * MLP_OUT * 4);
}

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", 2014): a 64-bit counter advanced by the golden-ratio
// increment, then a variant of the MurmurHash3 finaliser.
struct SplitMix64T {
    uint64_t x;
    uint64_t next() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    // uniform in [0, n) (n >= 1), by the high product (bias < n / 2^64)
    uint64_t below(uint64_t n) { return (uint64_t)(((unsigned __int128)next() * n) >> 64); }
    double unit() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct TrainWs {
    size_t jobs, samples, pool, info, hdr, idx, targets, loss, mlp, total;
};

TrainWs train_layout(int n_jobs, int dim_pad, int batch) {
    TrainWs t;
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t a = off;
        off = align256(off + b);
        return a;
    };
    t.jobs = take((size_t)n_jobs * sizeof(TrainJob));
    t.samples = take((size_t)batch * 16);
    t.pool = take(2 * (size_t)batch * dim_pad * 2);
    t.info = take(2 * (size_t)batch * sizeof(RowInfo));
    t.hdr = take(H_COUNT * 8);
    t.idx = take(2 * (size_t)batch * 4);
    t.targets = take((size_t)batch * 4);
    t.loss = take(4);
    t.mlp = take(train_ws(dim_pad, batch));
    t.total = off;
    return t;
}

}  // namespace

extern "C" {

void ejoin_prefilter_train_opts_default(ejoin_prefilter_train_opts* to) {
    if (!to) return;
    to->steps = 300;
    to->batch = 4096;
    to->seed = 1;
    to->pos_frac = 0.5f;
    ejoin_mlp_hparams_default(&to->hp);
}

size_t ejoin_prefilter_train_workspace(int32_t n_jobs, int32_t dim, int32_t batch) {
    ejoin_mlp_layout L;
    if (n_jobs < 1 || !layout_of(dim, L) || batch < 1 || batch > (1 << 20)) return 0;
    return train_layout(n_jobs, L.dim_pad, batch).total;
}

ejoin_status ejoin_prefilter_train(void* state, const ejoin_job* jobs, int32_t n_jobs,
                                   const int64_t* n_out, const ejoin_prefilter_train_opts* to_,
                                   void* ws, size_t ws_bytes, float* losses, hipStream_t stream) {
    ejoin_prefilter_train_opts to;
    ejoin_prefilter_train_opts_default(&to);
    if (to_) to = *to_;
    if (!state || !jobs || n_jobs < 1 || !n_out || to.steps < 0 || to.batch < 1 ||
        to.batch > (1 << 20) || !(to.pos_frac >= 0.0f && to.pos_frac <= 1.0f))
        return EJOIN_E_INVAL;
    const int dim = jobs[0].R.dim;
    ejoin_mlp_layout L;
    if (!layout_of(dim, L)) return EJOIN_E_UNSUPPORTED;
    std::vector<TrainJob> tj(n_jobs);
    std::vector<double> cum_pos(n_jobs), cum_all(n_jobs);
    double tp = 0.0, ta = 0.0;
    for (int i = 0; i < n_jobs; ++i) {
        const ejoin_job& j = jobs[i];
        if (!rel_ok(&j.R) || !rel_ok(&j.S) || j.R.dim != dim || j.S.dim != dim || n_out[i] < 0)
            return EJOIN_E_INVAL;
        const int64_t np = std::min(n_out[i], j.capacity);
        if (np > 0 && !j.out) return EJOIN_E_INVAL;
        tj[i] = TrainJob{j.R.data, j.S.data, (const Pair*)j.out, j.R.ld, j.S.ld, j.R.rows,
                         j.S.rows, dim, 0};
        tp += (double)np;
        ta += (double)j.R.rows * (double)j.S.rows;
        cum_pos[i] = tp;
        cum_all[i] = ta;
    }
    if (ta <= 0.0) return EJOIN_E_INVAL;
    const int B = to.batch;
    const TrainWs lay = train_layout(n_jobs, L.dim_pad, B);
    if (!ws || ws_bytes < lay.total) return EJOIN_E_WORKSPACE;
    char* w = (char*)ws;
    HIP_TRY(hipMemcpyAsync(w + lay.jobs, tj.data(), tj.size() * sizeof(TrainJob),
                           hipMemcpyHostToDevice, stream));
    {
        std::vector<int32_t> idx(2 * (size_t)B);
        for (int i = 0; i < 2 * B; ++i) idx[i] = i;
        HIP_TRY(hipMemcpyAsync(w + lay.idx, idx.data(), idx.size() * 4, hipMemcpyHostToDevice,
                               stream));
        HIP_TRY(hipStreamSynchronize(stream));
    }
    MlpDev m = dev_of(state, L);
    ejoin_mlp_hparams& h = to.hp;
    MlpHyper hy{h.lr, h.beta1, h.beta2, h.eps, h.lambda, h.theta_lo,
                (h.flags & EJOIN_MLP_GRAD_ONLY) != 0};
    const size_t r2 = 2 * (size_t)B;
    MlpTrainWs t;
    {
        char* b = w + lay.mlp;
        t.Xb = (float*)b;
        b += align256(r2 * L.dim_pad * 4);
        t.A1 = (float*)b;
        b += align256(r2 * MLP_HIDDEN * 4);
        t.dA1 = (float*)b;
        b += align256(r2 * MLP_HIDDEN * 4);
        t.Z = (float*)b;
        b += align256(r2 * MLP_OUT * 4);
        t.dZ = (float*)b;
    }
    SplitMix64T rng{to.seed};
    std::vector<int32_t> smp(4 * (size_t)B);
    auto pick = [&](const std::vector<double>& cum, double tot) {
        const double u = rng.unit() * tot;
        return (int)(std::upper_bound(cum.begin(), cum.end(), u) - cum.begin());
    };
    for (int step = 0; step < to.steps; ++step) {
        for (int i = 0; i < B; ++i) {
            int32_t* e = &smp[4 * (size_t)i];
            if (tp > 0.0 && rng.unit() < to.pos_frac) {
                const int j = std::min(pick(cum_pos, tp), n_jobs - 1);
                const int64_t np = std::min(n_out[j], jobs[j].capacity);
                e[0] = j;
                e[1] = 1;
                e[2] = (int32_t)rng.below((uint64_t)np);
                e[3] = 0;
            } else {
                const int j = std::min(pick(cum_all, ta), n_jobs - 1);
                e[0] = j;
                e[1] = 0;
                e[2] = (int32_t)rng.below((uint64_t)jobs[j].R.rows);
                e[3] = (int32_t)rng.below((uint64_t)jobs[j].S.rows);
            }
        }
        // the previous step has consumed the sample buffer once the stream
        // is idle; a synchronous copy keeps the host array reusable at once
        HIP_TRY(hipStreamSynchronize(stream));
        HIP_TRY(hipMemcpy(w + lay.samples, smp.data(), smp.size() * 4, hipMemcpyHostToDevice));
        const TrainJob* dj = (const TrainJob*)(w + lay.jobs);
        const int4* ds = (const int4*)(w + lay.samples);
        HIP_TRY(launch_train_rows(dj, ds, B, L.dim_pad, (uint16_t*)(w + lay.pool),
                                  (RowInfo*)(w + lay.info), (unsigned long long*)(w + lay.hdr),
                                  stream));
        HIP_TRY(launch_train_targets(dj, ds, B, (float*)(w + lay.targets), stream));
        const int32_t* idx = (const int32_t*)(w + lay.idx);
        HIP_TRY(launch_mlp_train_step(m, (const uint16_t*)(w + lay.pool), L.dim_pad, 2 * B, idx,
                                      idx + B, (const float*)(w + lay.targets), B, hy, t,
                                      (float*)(w + lay.loss), stream));
        if (losses) {
            HIP_TRY(hipMemcpyAsync(&losses[step], w + lay.loss, 4, hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
        }
    }
    HIP_TRY(hipStreamSynchronize(stream));
    return EJOIN_OK;
}

ejoin_status ejoin_mlp_layout_get(int32_t dim, ejoin_mlp_layout* layout) {
    if (!layout) return EJOIN_E_INVAL;
    return layout_of(dim, *layout) ? EJOIN_OK : EJOIN_E_INVAL;
}

void ejoin_mlp_hparams_default(ejoin_mlp_hparams* hp) {
    if (!hp) return;
    hp->lr = 1e-3f;
    hp->beta1 = 0.9f;
    hp->beta2 = 0.999f;
    hp->eps = 1e-8f;
    hp->lambda = 4.0f;
    hp->theta_lo = 0.7f;
    hp->flags = 0;
}

// ---- checkpoints: masters, Adam moments and step count in a host file ----
namespace {
constexpr char kCkptMagic[8] = {'E', 'J', 'P', 'F', 'N', 'E', 'T', '1'};
struct CkptHead {
    char magic[8];
    int32_t dim, reserved;
    int64_t n_params, step;
    float eps;
    uint32_t pad;
    uint64_t seed;
};
static_assert(sizeof(CkptHead) == 48, "checkpoint header layout");
}  // namespace

ejoin_status ejoin_prefilter_save(const void* state, int32_t dim, float eps, uint64_t seed,
                                  const char* path, hipStream_t stream) {
    ejoin_mlp_layout L;
    if (!state || !path || !layout_of(dim, L)) return EJOIN_E_INVAL;
    const size_t n = (size_t)L.n_params;
    std::vector<float> buf(3 * n);
    CkptHead h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, kCkptMagic, 8);
    h.dim = dim;
    h.n_params = L.n_params;
    h.eps = eps;
    h.seed = seed;
    const char* b = (const char*)state;
    HIP_TRY(hipMemcpyAsync(buf.data(), b + L.off_params, n * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(buf.data() + n, b + L.off_m, n * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(buf.data() + 2 * n, b + L.off_v, n * 4, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipMemcpyAsync(&h.step, b + L.off_step, 8, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    FILE* f = fopen(path, "wb");
    if (!f) return EJOIN_E_INVAL;
    const bool ok = fwrite(&h, sizeof(h), 1, f) == 1 && fwrite(buf.data(), 4, 3 * n, f) == 3 * n;
    if (fclose(f) != 0 || !ok) return EJOIN_E_INVAL;
    return EJOIN_OK;
}

ejoin_status ejoin_prefilter_load(void* state, int32_t dim, const char* path, float* eps,
                                  uint64_t* seed, hipStream_t stream) {
    ejoin_mlp_layout L;
    if (!state || !path || !layout_of(dim, L)) return EJOIN_E_INVAL;
    FILE* f = fopen(path, "rb");
    if (!f) return EJOIN_E_INVAL;
    CkptHead h;
    const size_t n = (size_t)L.n_params;
    std::vector<float> buf(3 * n);
    bool ok = fread(&h, sizeof(h), 1, f) == 1 && memcmp(h.magic, kCkptMagic, 8) == 0 &&
              h.dim == dim && h.n_params == L.n_params && h.step >= 0 &&
              fread(buf.data(), 4, 3 * n, f) == 3 * n;
    if (ok) {  // nothing may follow the three vectors
        char extra;
        ok = fread(&extra, 1, 1, f) == 0;
    }
    fclose(f);
    if (!ok) return EJOIN_E_INVAL;
    for (size_t i = 0; i < 3 * n; ++i)
        if (!isfinite(buf[i])) return EJOIN_E_NONFINITE;
    char* b = (char*)state;
    const MlpDev m = dev_of(state, L);
    HIP_TRY(hipMemcpyAsync(b + L.off_params, buf.data(), n * 4, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(b + L.off_m, buf.data() + n, n * 4, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(b + L.off_v, buf.data() + 2 * n, n * 4, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipMemcpyAsync(b + L.off_step, &h.step, 8, hipMemcpyHostToDevice, stream));
    HIP_TRY(launch_mlp_restored(m, stream));
    HIP_TRY(hipStreamSynchronize(stream));  // the host buffers go out of scope
    if (eps) *eps = h.eps;
    if (seed) *seed = h.seed;
    return EJOIN_OK;
}

ejoin_status ejoin_mlp_init(void* state, int32_t dim, const float* params, hipStream_t stream) {
    ejoin_mlp_layout L;
    if (!state || !params || !layout_of(dim, L)) return EJOIN_E_INVAL;
    HIP_TRY(launch_mlp_init(dev_of(state, L), params, stream));
    return EJOIN_OK;
}

size_t ejoin_mlp_train_workspace(int32_t dim, int32_t batch) {
    ejoin_mlp_layout L;
    if (!layout_of(dim, L) || batch < 1 || batch > (1 << 20)) return 0;
    return train_ws(L.dim_pad, batch);
}

ejoin_status ejoin_mlp_train_step(void* state, int32_t dim, const uint16_t* X, int64_t ldx,
                                  int64_t rows, const int32_t* pr, const int32_t* ps,
                                  const float* target, int32_t batch,
                                  const ejoin_mlp_hparams* hp, void* ws, size_t ws_bytes,
                                  float* loss, hipStream_t stream) {
    ejoin_mlp_layout L;
    if (!state || !layout_of(dim, L) || batch < 1 || batch > (1 << 20)) return EJOIN_E_INVAL;
    if (!X || !pr || !ps || !target || !loss || ldx < dim || rows < 1) return EJOIN_E_INVAL;
    ejoin_mlp_hparams h;
    ejoin_mlp_hparams_default(&h);
    if (hp) h = *hp;
    if (!(h.lr > 0) || !(h.beta1 >= 0 && h.beta1 < 1) || !(h.beta2 >= 0 && h.beta2 < 1) ||
        !(h.eps > 0) || !(h.lambda >= 0) || !isfinite(h.theta_lo))
        return EJOIN_E_INVAL;
    const size_t need = train_ws(L.dim_pad, batch);
    if (!ws || ws_bytes < need) return EJOIN_E_WORKSPACE;
    const size_t r2 = 2 * (size_t)batch;
    char* w = (char*)ws;
    MlpTrainWs t;
    t.Xb = (float*)w;
    w += align256(r2 * L.dim_pad * 4);
    t.A1 = (float*)w;
    w += align256(r2 * MLP_HIDDEN * 4);
    t.dA1 = (float*)w;
    w += align256(r2 * MLP_HIDDEN * 4);
    t.Z = (float*)w;
    w += align256(r2 * MLP_OUT * 4);
    t.dZ = (float*)w;
    MlpHyper hy{h.lr, h.beta1, h.beta2, h.eps, h.lambda, h.theta_lo,
                (h.flags & EJOIN_MLP_GRAD_ONLY) != 0};
    HIP_TRY(launch_mlp_train_step(dev_of(state, L), X, ldx, rows, pr, ps, target, batch, hy, t,
                                  loss, stream));
    return EJOIN_OK;
}

size_t ejoin_mlp_forward_workspace(int32_t dim, int64_t n) {
    ejoin_mlp_layout L;
    if (!layout_of(dim, L) || n < 0) return 0;
    return fwd_ws(n) + 256;
}

ejoin_status ejoin_mlp_forward(const void* state, int32_t dim, const uint16_t* X, int64_t n,
                               float* U, void* ws, size_t ws_bytes, hipStream_t stream) {
    ejoin_mlp_layout L;
    if (!state || !layout_of(dim, L) || n < 0) return EJOIN_E_INVAL;
    if (n == 0) return EJOIN_OK;
    if (!X || !U) return EJOIN_E_INVAL;
    if (!ws || ws_bytes < fwd_ws(n)) return EJOIN_E_WORKSPACE;
    const size_t rows = (size_t)((n + 127) / 128) * 128;
    uint16_t* Hb = (uint16_t*)ws;
    float* Z = (float*)((char*)ws + align256(rows * MLP_HIDDEN * 2));
    HIP_TRY(launch_mlp_forward(dev_of((void*)state, L), X, n, Hb, Z, U, stream));
    return EJOIN_OK;
}

}  // extern "C"
