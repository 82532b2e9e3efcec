"""Pins of the FP64 prefilter reference (oracle/mlp.py) against facts that
do not come from it: a library's BF16 conversion, central finite differences,
closed forms of Adam, the scale invariance that the normalisation of the
code implies, and brute force over tile pairs."""
import numpy as np
import pytest

from oracle import mlp as M

torch = pytest.importorskip("torch")


def _params(d, H, O, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return {"W1": rng.standard_normal((d, H)) * scale * np.sqrt(2.0 / d),
            "b1": rng.standard_normal(H) * 0.1,
            "W2": rng.standard_normal((H, O)) * scale * np.sqrt(2.0 / H),
            "b2": rng.standard_normal(O) * 0.1}


def _batch(n_rows, d, B, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n_rows, d))
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    pr = rng.integers(0, n_rows, B)
    ps = rng.integers(0, n_rows, B)
    t = rng.uniform(-0.2, 1.0, B)
    return X, pr, ps, t


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(20000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38, 1e-40],
                                 np.float32)])
    # ties: values exactly half-way between two bfloat16 numbers
    a = np.concatenate([a, (np.arange(1, 200, dtype=np.uint32) << 16 | 0x8000)
                        .view(np.float32)])
    want = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    got = M.bf16_round(a)
    assert np.array_equal(got, want)


def test_forward_invariants():
    p = _params(24, 32, 8, 1)
    X, _, _, _ = _batch(50, 24, 1, 2)
    f = M.forward(M.forward_weights(p), X)
    assert (f["h"] >= 0).all()
    assert np.allclose(np.linalg.norm(f["u"], axis=1), 1.0, atol=1e-14)
    # scaling the second layer by c > 0 leaves the code unchanged
    q = dict(p)
    q["W2"] = p["W2"] * 3.0
    q["b2"] = p["b2"] * 3.0
    g = M.forward(M.forward_weights(q, round_bf16=False), X)
    f0 = M.forward(M.forward_weights(p, round_bf16=False), X)
    assert np.allclose(g["u"], f0["u"], atol=1e-14)


def test_forward_closed_form_identity_network():
    # W1 = I, b1 = 0, W2 = I, b2 = 0: u = ReLU(x) / ||ReLU(x)||
    d = 16
    W = {"W1": np.eye(d), "b1": np.zeros(d), "W2": np.eye(d), "b2": np.zeros(d)}
    rng = np.random.default_rng(3)
    X = rng.standard_normal((20, d))
    u = M.forward(W, X)["u"]
    r = np.maximum(X, 0)
    assert np.allclose(u, r / np.linalg.norm(r, axis=1, keepdims=True), atol=1e-15)


def test_pair_loss_special_cases():
    t = np.array([0.9, 0.5, 0.95, 0.1])
    loss, dp = M.pair_loss(t.copy(), t, 4.0, 0.7)
    assert loss == 0.0 and np.all(dp == 0.0)
    p = np.array([0.8, 0.6, 1.0, 0.0])
    l0, d0 = M.pair_loss(p, t, 0.0, 0.7)
    assert np.isclose(l0, np.mean((p - t) ** 2))
    # the recall term charges only under-predicted pairs with t >= theta_lo
    l4, d4 = M.pair_loss(p, t, 4.0, 0.7)
    extra = 4.0 * np.mean(np.array([0.1, 0.0, 0.0, 0.0]) ** 2)
    assert np.isclose(l4 - l0, extra)
    assert np.isclose(d4[0] - d0[0], -4.0 * 2.0 / 4 * 0.1)
    assert np.all(d4[1:] == d0[1:])


@pytest.mark.parametrize("lam", [0.0, 4.0])
def test_gradients_match_central_differences(lam):
    """Backward through pair product, normalisation, second layer, ReLU and
    first layer against central differences of the loss (FP64 masters, no
    BF16 rounding so the loss is smooth in the weights)."""
    d, H, O = 12, 16, 6
    p = _params(d, H, O, 5)
    X, pr, ps, t = _batch(30, d, 40, 6)
    loss, g, _ = M.loss_and_grads(p, X, pr, ps, t, lam, 0.3, round_bf16=False)
    rng = np.random.default_rng(7)
    h = 1e-6
    for k in ("W1", "b1", "W2", "b2"):
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(flat.size, 12), replace=False):
            up = {kk: vv.copy() for kk, vv in p.items()}
            dn = {kk: vv.copy() for kk, vv in p.items()}
            up[k].reshape(-1)[idx] += h
            dn[k].reshape(-1)[idx] -= h
            lu = M.loss_and_grads(up, X, pr, ps, t, lam, 0.3, round_bf16=False)[0]
            ld = M.loss_and_grads(dn, X, pr, ps, t, lam, 0.3, round_bf16=False)[0]
            fd = (lu - ld) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, an)


def test_gradient_orthogonal_to_second_layer():
    """z is linear-homogeneous in (W2, b2) and the loss sees z only through
    z / ||z||, so the directional derivative along (W2, b2) itself is 0."""
    p = _params(20, 32, 8, 9)
    X, pr, ps, t = _batch(40, 20, 64, 10)
    _, g, _ = M.loss_and_grads(p, X, pr, ps, t, 4.0, 0.7)
    W = M.forward_weights(p)
    s = np.sum(W["W2"] * g["W2"]) + np.sum(W["b2"] * g["b2"])
    scale = np.sqrt(np.sum(W["W2"] ** 2) * np.sum(g["W2"] ** 2))
    assert abs(s) <= 1e-12 * scale


def test_adam_first_step_closed_form():
    p = _params(6, 8, 4, 11)
    rng = np.random.default_rng(12)
    g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
    z = {k: np.zeros_like(v) for k, v in p.items()}
    P, Mo, V = M.adam_step(p, g, z, z, 1, lr=1e-3)
    for k in p:
        # bias-corrected m = g and v = g^2 after one step
        want = p[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(P[k], want, rtol=0, atol=1e-15)
        assert np.allclose(Mo[k], 0.1 * g[k]) and np.allclose(V[k], 0.001 * g[k] ** 2)


def test_adam_constant_gradient_moves_linearly():
    # with the same gradient every step the corrected moments stay g and g^2
    p = {"w": np.array([0.5, -2.0, 3.0])}
    g = {"w": np.array([0.25, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    for step in range(1, 26):
        p, m, v = M.adam_step(p, g, m, v, step, lr=1e-2)
    want = np.array([0.5, -2.0, 3.0]) - 25 * 1e-2 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(p["w"], want, rtol=0, atol=1e-12)


def test_tile_bound_dominates_brute_force():
    rng = np.random.default_rng(13)
    U = rng.standard_normal((300, 64))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    # clustered rows as well as spread ones
    V = np.repeat(rng.standard_normal((5, 64)), 40, axis=0) + 0.05 * rng.standard_normal((200, 64))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    for A in (U, V):
        C, rho = M.tile_stats(A, 32)
        for i in range(C.shape[0]):
            for j in range(C.shape[0]):
                bi = A[i * 32:(i + 1) * 32]
                bj = A[j * 32:(j + 1) * 32]
                true_max = (bi @ bj.T).max()
                assert M.tile_pair_bound(C[i], rho[i], C[j], rho[j]) >= true_max - 1e-12
    # single-row tiles: radius 0 and the bound is the dot product itself
    C, rho = M.tile_stats(U[:10], 1)
    assert np.all(rho == 0)
    assert np.isclose(M.tile_pair_bound(C[2], 0.0, C[7], 0.0), U[2] @ U[7])


def test_angular_tile_bound_dominates_brute_force_and_can_be_tighter():
    rng = np.random.default_rng(17)
    base = rng.standard_normal((6, 64))
    V = np.repeat(base, 32, axis=0) + 0.08 * rng.standard_normal((192, 64))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    C, rho = M.tile_stats(V, 32)
    A = M.tile_angles(V, 32)
    tighter = 0
    for i in range(6):
        for j in range(6):
            bi, bj = V[i * 32:(i + 1) * 32], V[j * 32:(j + 1) * 32]
            true_max = (bi @ bj.T).max()
            ang = M.tile_pair_bound_angular(C[i], A[i], C[j], A[j])
            lin = M.tile_pair_bound(C[i], rho[i], C[j], rho[j])
            assert ang >= true_max - 1e-12
            tighter += ang < lin
    assert tighter > 0
    # one-point tiles: zero angle, the bound is the dot product itself
    A1 = M.tile_angles(V[:4], 1)
    assert np.allclose(A1, 0.0, atol=1e-7)
    assert np.isclose(M.tile_pair_bound_angular(V[0], 0.0, V[3], 0.0), V[0] @ V[3])


def test_anchor_key_groups_tight_clusters_and_orders_stably():
    rng = np.random.default_rng(19)
    cent = rng.standard_normal((7, 64))
    cent /= np.linalg.norm(cent, axis=1, keepdims=True)
    lab = rng.integers(0, 7, 500)
    U = cent[lab] + 0.02 * rng.standard_normal((500, 64))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    A = U[rng.choice(500, 60, replace=False)]
    L = M.leader_labels(A, 0.6)
    key = M.anchor_key(U, A, L)
    # one key per cluster, and different clusters never share a key
    for c in range(7):
        assert len(set(key[lab == c].tolist())) <= 1
    seen = {}
    for c, k in zip(lab, key):
        assert seen.setdefault(k, c) == c
    # leaders come in anchor order: the first anchor leads group 0
    assert L[0] == 0 and L.max() == len(set(L.tolist())) - 1
    keys = np.array([3, 1, 3, 0, 1])
    assert M.order_by_key(keys).tolist() == [3, 1, 4, 0, 2]


def test_tile_rows_bound_dominates_brute_force():
    """cos(max(0, acos(max_v dir_T . v) - a_T)) bounds every u . v of the
    tile pair from above (slack 0), is tight for a one-row tile, and the
    library's margin only loosens it."""
    rng = np.random.default_rng(23)
    base = rng.standard_normal((6, 64))
    V = np.repeat(base, 32, axis=0) + 0.1 * rng.standard_normal((192, 64))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    C, rho = M.tile_stats(V, 32)
    A = M.tile_angles(V, 32)
    tighter = 0
    for i in range(6):
        di = C[i] / np.linalg.norm(C[i])
        for j in range(6):
            bi, bj = V[i * 32:(i + 1) * 32], V[j * 32:(j + 1) * 32]
            true_max = (bi @ bj.T).max()
            b = M.tile_rows_bound(di, A[i], bj)
            assert b >= true_max - 1e-12
            assert M.tile_rows_bound(di, A[i], bj, 0.02) >= b
            tighter += b < M.tile_pair_bound_angular(C[i], A[i], C[j], A[j]) - 1e-9
    assert tighter > 0
    # one-row tile T: direction = the row, angle 0: the bound is the best dot
    for j in range(6):
        bj = V[j * 32:(j + 1) * 32]
        assert np.isclose(M.tile_rows_bound(V[0], 0.0, bj), (bj @ V[0]).max())


def test_splitmix64_reference_outputs():
    import json
    import os
    from oracle import prefilter as P
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "splitmix64_seed1234567.json")))
    rng = P.SplitMix64(g["seed"])
    assert [rng.next() for _ in g["outputs"]] == [int(x) for x in g["outputs"]]
    # draws below n are the high words of next() * n: uniform in [0, n)
    rng = P.SplitMix64(5)
    d = np.array([rng.below(7) for _ in range(7000)])
    assert d.min() == 0 and d.max() == 6 and np.all(np.abs(np.bincount(d) - 1000) < 150)


def test_prefilter_plan_invariants():
    """The reference plan on small clustered jobs: orders are permutations
    sorted by key, self-joins share one order, empty jobs are skipped, and
    the bound of every tile pair dominates the largest code product of its
    rows (the library's margin only adds to it)."""
    from oracle import prefilter as P
    rng = np.random.default_rng(29)
    D = 24
    cent = rng.standard_normal((5, D))
    def pts(n):
        X = cent[rng.integers(0, 5, n)] + 0.05 * rng.standard_normal((n, D))
        return X.astype(np.float32)
    X = pts(300)
    jobs = [(pts(200), pts(330), 0.8, False), (np.zeros((0, D), np.float32), pts(5), 0.5, False),
            (X, X, 0.9, True)]
    W1 = (rng.standard_normal((D, 256)) / np.sqrt(D)).astype(np.float32)
    W2 = (rng.standard_normal((256, 64)) / 16).astype(np.float32)
    params = {"W1": W1, "b1": np.zeros(256, np.float32), "W2": W2, "b2": np.zeros(64, np.float32)}
    pl = P.plan(jobs, params, D, eps=0.1)
    assert pl["segs"] == [(2, "r"), (0, "r"), (0, "s")]  # most tiles first, empty job left out
    assert pl["A"].shape[0] == 830
    for (R, S, th, alias), J in zip(jobs, pl["jobs"]):
        if R.shape[0] == 0:
            assert J["bound"].size == 0
            continue
        assert sorted(J["order_r"].tolist()) == list(range(R.shape[0]))
        if alias:
            assert np.array_equal(J["order_r"], J["order_s"])
        ur = P.codes(params, R, D)[J["order_r"]]
        us = P.codes(params, S, D)[J["order_s"]]
        for a in range(J["bound"].shape[0]):
            for b in range(J["bound"].shape[1]):
                best = (ur[a * 128:(a + 1) * 128] @ us[b * 128:(b + 1) * 128].T).max()
                assert J["bound"][a, b] >= best - 1e-9
        assert np.array_equal(J["keep"], J["bound"] >= th - 0.1)
    k0 = pl["keys"][1]
    assert np.all(np.diff(k0[pl["jobs"][0]["order_r"]]) >= 0)



def test_tile_rows_bound_in_the_embedding_space():
    """The same bound on 300-d unit rows (the exact pruning of the batched
    join uses it in the original space): it dominates every pair's cosine of
    clustered tiles, and it separates tiles of different clusters."""
    rng = np.random.default_rng(31)
    cent = rng.standard_normal((4, 300))
    cent /= np.linalg.norm(cent, axis=1, keepdims=True)
    V = np.repeat(cent, 32, axis=0) + 0.25 / np.sqrt(300) * rng.standard_normal((128, 300))
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    C, _ = M.tile_stats(V, 32)
    A = M.tile_angles(V, 32)
    separated = 0
    for i in range(4):
        di = C[i] / np.linalg.norm(C[i])
        for j in range(4):
            bj = V[j * 32:(j + 1) * 32]
            b = M.tile_rows_bound(di, A[i], bj)
            assert b >= (V[i * 32:(i + 1) * 32] @ bj.T).max() - 1e-12
            separated += i != j and b < 0.75
    assert separated == 12
