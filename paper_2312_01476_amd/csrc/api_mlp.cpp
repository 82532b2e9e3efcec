// api_mlp.cpp -- C ABI of the prefilter network: state layout, init,
// training step and inference.
#include <hip/hip_runtime.h>

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
    L.off_planes = off;
    off = align256(off + (size_t)MLP_PLANES * MLP_OUT * 4);
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
    m.planes = (float*)(b + L.off_planes);
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

}  // namespace

extern "C" {

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

ejoin_status ejoin_mlp_init(void* state, int32_t dim, const float* params, const float* planes,
                            hipStream_t stream) {
    ejoin_mlp_layout L;
    if (!state || !params || !planes || !layout_of(dim, L)) return EJOIN_E_INVAL;
    HIP_TRY(launch_mlp_init(dev_of(state, L), params, planes, stream));
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
