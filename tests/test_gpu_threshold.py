"""Parity of the GPU threshold join (through the C ABI) with the FP64 oracle.

The bar: the GPU result set equals the oracle's set exactly; every score is
within 1e-3 of sim64 in FP32 mode and for every FP64-rescored pair, and within
the rigorous band for the BF16/FP8 certain pairs.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2312_01476_amd import datagen as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = None


def setup_module(module):
    global E
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_01476_amd import ejoin
    E = ejoin


def _dev(X):
    return torch.from_numpy(np.ascontiguousarray(X)).to("cuda")


def _run(R, S, theta, d=None, **kw):
    Rd = _dev(R)
    Sd = Rd if S is R else _dev(S)
    res = E.threshold(Rd, Sd, theta, d=d, **kw)
    r = res.r.cpu().numpy().astype(np.int64)
    s = res.s.cpu().numpy().astype(np.int64)
    sc = res.score.cpu().numpy().astype(np.float64)
    return r, s, sc, res.stats


def _check(R, S, theta, d=None, prec="fp32", score_tol=None, **kw):
    d_ = R.shape[1] if d is None else d
    r, s, sc, st = _run(R, S, theta, d=d, prec=prec, **kw)
    ori, osi, osc, _ = O.threshold(R, S, theta, d=d_)
    got = set(zip(r.tolist(), s.tolist()))
    want = set(zip(ori.tolist(), osi.tolist()))
    assert len(got) == len(r), "duplicate pairs in GPU output"
    missing = want - got
    extra = got - want
    assert not missing and not extra, (f"{prec}: {len(missing)} missing, {len(extra)} extra; "
                                       f"e.g. {sorted(missing)[:3]} {sorted(extra)[:3]}")
    assert st["n_pairs"] == len(r)
    if len(r):
        ref = O.sim64_pairs(R, S, r, s, d=d_)
        err = np.abs(sc - ref)
        tol = score_tol if score_tol is not None else (1e-3 if prec == "fp32" else st["band"])
        assert err.max() <= tol, (prec, err.max())
    return st


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_words_1k_full(prec):
    w = G.WORKLOADS["words_1k"]
    R, S, lr, ls = G.make_host(w)
    st = _check(R, S, w.theta, d=w.d, prec=prec)
    assert st["n_pairs"] == int((lr[:, None] == ls[None, :]).sum())


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (130, 257, 33), (300, 129, 300),
                                   (257, 513, 768)])
def test_ragged_random(prec, shape):
    nr, ns, d = shape
    R = G.gaussian_raw(nr, d, seed=nr * 7 + d)
    S = G.gaussian_raw(ns, d, seed=ns * 11 + d)
    sims = O.sim_matrix(R, S)
    for q in (0.5, 0.99):
        theta = float(np.quantile(sims, q))
        _check(R, S, theta, prec=prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_planted_pairs_around_theta(prec):
    """Pairs planted at theta +- tiny offsets land in the band and must be
    decided exactly by the FP64 rescore."""
    rng = np.random.Generator(np.random.PCG64(5))
    d = 300
    R = G.uniform_sphere(200, d, seed=1)
    S = G.uniform_sphere(300, d, seed=2)
    theta = 0.8
    # make S[j] = cos(phi) R[i] + sin(phi) u for u orthogonal to R[i]
    planted = []
    offs = [-1e-3, -1e-5, -1e-7, 0.0, 1e-7, 1e-5, 1e-3]
    for t, off in enumerate(offs * 4):
        i, j = 3 * t, 5 * t + 1
        r = R[i].astype(np.float64)
        u = rng.standard_normal(d)
        u -= (u @ r) / (r @ r) * r
        u /= np.linalg.norm(u)
        c = theta + off
        S[j] = (c * r / np.linalg.norm(r) + np.sqrt(1 - c * c) * u).astype(np.float32)
        planted.append((i, j))
    st = _check(R, S, theta, prec=prec)
    assert st["n_band"] >= len(planted) // 2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_self_join_alias_symmetric(prec):
    X = G.gaussian_raw(333, 64, seed=3)
    X[10] = X[4]
    res = E.threshold(_dev(X), _dev(X), 0.3, prec=prec)          # distinct buffers
    Xd = _dev(X)
    res2 = E.threshold(Xd, Xd, 0.3, prec=prec)                  # aliased
    a = set(zip(res.r.cpu().tolist(), res.s.cpu().tolist()))
    b = set(zip(res2.r.cpu().tolist(), res2.s.cpu().tolist()))
    assert a == b
    assert all((j, i) in b for (i, j) in b)
    assert all((i, i) in b for i in range(X.shape[0]))
    _check(X, X, 0.3, prec=prec)


def test_zero_rows_and_theta_extremes():
    R = G.gaussian_raw(70, 20, seed=8)
    S = G.gaussian_raw(90, 20, seed=9)
    R[5] = 0.0
    S[7] = 0.0
    for theta in (-2.0, -1.0, -1e-6, 0.0, 1e-6, 0.5, 1.0, 1.0 + 1e-6, 3.0):
        _check(R, S, theta)
        _check(R, S, theta, prec="bf16")


def test_padding_columns_never_read():
    w = G.WORKLOADS["words_1k"]
    R, S, _, _ = G.make_host(w, n_r=300, n_s=200, pad_value=np.nan)
    _check(R, S, w.theta, d=w.d)


def test_nonfinite_and_range_errors():
    R = G.gaussian_raw(40, 16, seed=1)
    S = G.gaussian_raw(50, 16, seed=2)
    R2 = R.copy()
    R2[3, 2] = np.inf
    with pytest.raises(E.EjoinError) as ei:
        E.threshold(_dev(R2), _dev(S), 0.5)
    assert ei.value.status == E.E_NONFINITE
    S2 = S.copy()
    S2[4] *= np.float32(2.0 ** -110)
    with pytest.raises(E.EjoinError) as ei:
        E.threshold(_dev(R), _dev(S2), 0.5)
    assert ei.value.status == E.E_RANGE


def test_empty_inputs():
    R = G.gaussian_raw(0, 16, seed=1)
    S = G.gaussian_raw(50, 16, seed=2)
    res = E.threshold(_dev(R).reshape(0, 16), _dev(S), 0.1)
    assert len(res) == 0
    res = E.threshold(_dev(S), _dev(R).reshape(0, 16), 0.1)
    assert len(res) == 0


def test_overflow_reports_true_count_then_retry():
    R = G.gaussian_raw(100, 8, seed=4)
    S = G.gaussian_raw(100, 8, seed=5)
    Rd, Sd = _dev(R), _dev(S)
    ws = torch.empty(E.threshold_workspace(Rd, Sd), dtype=torch.uint8, device="cuda")
    out = torch.empty((10, 3), dtype=torch.int32, device="cuda")
    rc, n, st = E.threshold_raw(Rd, Sd, 0.0, out, 10, ws)
    assert rc == E.E_OVERFLOW
    ori, _, _, _ = O.threshold(R, S, 0.0)
    assert n == len(ori)
    out = torch.empty((n, 3), dtype=torch.int32, device="cuda")
    rc, n2, st = E.threshold_raw(Rd, Sd, 0.0, out, n, ws)
    assert rc == E.OK and n2 == n


def test_band_capacity_too_small_reports_workspace():
    """Everything in the band (theta at the common similarity of identical
    rows): a tiny band list must be reported, then the retry is exact."""
    X = np.tile(G.gaussian_raw(1, 32, seed=6), (50, 1))
    Xd = _dev(X)
    ws_small = E.threshold_workspace(Xd, Xd, band_capacity=16)
    ws = torch.empty(ws_small, dtype=torch.uint8, device="cuda")
    out = torch.empty((4000, 3), dtype=torch.int32, device="cuda")
    rc, n, st = E.threshold_raw(Xd, Xd, 1.0, out, 4000, ws, band_capacity=16)
    assert rc == E.E_WORKSPACE and st["band_needed"] == 2500
    res = E.threshold(Xd, Xd, 1.0, band_capacity=16)
    assert len(res) == 2500


def test_invalid_arguments():
    R = _dev(G.gaussian_raw(10, 8, seed=1))
    S = _dev(G.gaussian_raw(10, 9, seed=2))
    with pytest.raises(E.EjoinError) as ei:
        E.threshold(R, S, 0.5)
    assert ei.value.status == E.E_INVAL
    with pytest.raises(E.EjoinError):
        E.threshold(R, R, float("nan"))
    with pytest.raises(E.EjoinError):
        E.threshold(R, R, 0.5, band=1e-9)  # narrower than the rigorous bound


@pytest.mark.parametrize("tile", [1, 2, 11, 18, 20, 21])
def test_tile_shapes_give_identical_sets_fp32(tile):
    w = G.WORKLOADS["fp32_100k"]
    R, S, lr, ls = G.make_host(w, n_r=3000, n_s=2500)
    _check(R, S, w.theta, d=w.d, tile=tile)


@pytest.mark.parametrize("tile", [3, 4, 8, 12, 14, 16, 24])
def test_tile_shapes_bf16(tile):
    w = G.WORKLOADS["bf16_1m"]
    R, S, lr, ls = G.make_host(w, n_r=2000, n_s=3000)
    st = _check(R, S, w.theta, d=w.d, prec="bf16", band=w.band, tile=tile)
    assert st["n_pairs"] == int((lr[:, None] == ls[None, :]).sum())


@pytest.mark.parametrize("tile", [5, 6, 10, 13, 17, 25])
def test_tile_shapes_fp8(tile):
    w = G.WORKLOADS["fp8_topk_2m"]
    R, S, lr, ls = G.make_host(w, n_r=1000, n_s=1500)
    _check(R, S, 0.8, d=w.d, prec="fp8", tile=tile)


@pytest.mark.parametrize("prec,d", [("bf16", 64), ("bf16", 160), ("bf16", 200), ("bf16", 300),
                                    ("bf16", 384), ("bf16", 500),
                                    ("bf16", 560), ("bf16", 640), ("bf16", 768), ("fp8", 128),
                                    ("fp8", 300), ("fp8", 700), ("fp32", 40), ("fp32", 100),
                                    ("fp32", 160), ("fp32", 250), ("fp32", 280), ("fp32", 300),
                                    ("fp32", 384)])
def test_panel_kernel_depths(prec, d):
    """Every resident-fragment depth of the panel kernel, ragged |R| and |S|
    (several panels, S chunks and a partial last tile); BF16 500 / 560 / 640 /
    768 are the deep rows (8, 9, 10, 12 K slices); BF16 runs as one workgroup
    (tile 12) and as two workgroups per CU (tile 14) at every depth; the FP32
    panels (tile 20 one workgroup, 21 two workgroups per CU) take the same
    slice counts (40 .. 384 floats)."""
    cent = G.centres(d, 40, seed=d)
    R, lr = G.clustered_points(cent, 1100, 0.3, seed=d + 1)
    S, ls = G.clustered_points(cent, 1900, 0.3, seed=d + 2)
    tiles = {"bf16": (12, 14), "fp8": (13,), "fp32": (20, 21)}[prec]
    for tile in tiles:
        st = _check(R, S, 0.7, prec=prec, tile=tile)
        assert st["tile"] == tile


@pytest.mark.parametrize("shape", [(1, 1, 1), (130, 257, 33), (300, 129, 300), (257, 513, 768),
                                   (70, 1100, 1024)])
def test_nlj_comparator_is_exact(shape):
    """The nested-loop comparator (tile 23: one pair per wavefront, no
    tiling) goes through the same band and FP64 rescore: its set equals the
    oracle's, ragged shapes and depths up to 1024 included."""
    nr, ns, d = shape
    R = G.gaussian_raw(nr, d, seed=nr + 3 * d)
    S = G.gaussian_raw(ns, d, seed=ns + 5 * d)
    sims = O.sim_matrix(R, S)
    for q in (0.5, 0.99):
        _check(R, S, float(np.quantile(sims, q)), tile=23)


def test_nlj_comparator_words_and_limits():
    w = G.WORKLOADS["words_1k"]
    R, S, lr, ls = G.make_host(w)
    st = _check(R, S, w.theta, d=w.d, tile=23)
    assert st["tile"] == 23 and st["n_pairs"] == int((lr[:, None] == ls[None, :]).sum())
    Rd = _dev(G.gaussian_raw(8, 1100, seed=1))
    with pytest.raises(E.EjoinError):        # rows deeper than 1024 elements
        E.threshold(Rd, Rd, 0.5, tile=23)
    with pytest.raises(E.EjoinError):        # FP32 only
        E.threshold(Rd[:, :64], Rd[:, :64], 0.5, prec="bf16", tile=23)



@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("self_join", [False, True])
def test_measured_band_is_narrower_and_exact(prec, self_join):
    """The default band of a BF16 / FP8 single join is measured on the device
    from the rows' quantisation error norms: well inside the worst-case
    bound, so fewer pairs go to the FP64 rescore, and the set stays exact."""
    cent = G.centres(300, 20, seed=90)
    R, _ = G.clustered_points(cent, 1500, 0.3, seed=91)
    S = R if self_join else G.clustered_points(cent, 1200, 0.3, seed=92)[0]
    sims = O.sim_matrix(R, S)
    theta = float(np.quantile(sims, 0.97))
    st = _check(R, S, theta, prec=prec)
    worst = E.band_default(prec, 300)
    assert st["band"] < 0.8 * worst, (st["band"], worst)
    near = lambda b: int((np.abs(sims - theta) < b).sum())
    assert st["n_band"] <= near(st["band"] + 1e-3) <= near(worst)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_approximate_score_error_against_fp64(prec):
    """Scores accepted straight from the narrow-format contraction carry the
    format's error: measured here over every returned pair.  BF16 stays
    within 1e-3 of sim64 at 300-d and above (at 33-d it does not: the error
    of a few quantised terms does not average out); FP8 e4m3 with per-row
    scales is within its band only.  The exact set does not depend on it."""
    w = G.WORKLOADS["words_1k"]
    R, S, _, _ = G.make_host(w)
    r, s, sc, st = _run(R, S, w.theta, d=w.d, prec=prec)
    err = np.abs(sc - O.sim64_pairs(R, S, r, s, d=w.d))
    assert st["n_certain"] > 0
    if prec == "bf16":
        assert err.max() <= 1e-3, err.max()
    else:
        assert 1e-3 < err.max() <= st["band"], (err.max(), st["band"])
    R = G.gaussian_raw(257, 768, seed=257 * 7 + 768)
    S = G.gaussian_raw(513, 768, seed=513 * 11 + 768)
    theta = float(np.quantile(O.sim_matrix(R, S), 0.9))
    r, s, sc, st = _run(R, S, theta, prec=prec)
    err = np.abs(sc - O.sim64_pairs(R, S, r, s))
    assert err.max() <= (1e-3 if prec == "bf16" else st["band"])


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("shape", [(5, 7, 3), (130, 257, 33), (300, 1100, 300)])
def test_fp64_scores_flag_returns_exact_scores(prec, shape):
    """EJOIN_FP64_SCORES: nothing is accepted on its approximate score, so
    every returned score is float32(sim64) in every precision (within 1e-3
    of sim64 whatever the format's error) and the set is still exact."""
    nr, ns, d = shape
    R = G.gaussian_raw(nr, d, seed=nr * 3 + d)
    S = G.gaussian_raw(ns, d, seed=ns * 5 + d)
    sims = O.sim_matrix(R, S)
    for q in (0.5, 0.95):
        theta = float(np.quantile(sims, q))
        r, s, sc, st = _run(R, S, theta, prec=prec, fp64_scores=True, band_capacity=nr * ns + 16)
        ori, osi, _, _ = O.threshold(R, S, theta)
        assert set(zip(r.tolist(), s.tolist())) == set(zip(ori.tolist(), osi.tolist()))
        ref = O.sim64_pairs(R, S, r, s).astype(np.float32).astype(np.float64)
        np.testing.assert_array_equal(sc, ref)
        assert st["n_certain"] == 0 and st["n_band_accepted"] == len(r)


def test_fp64_scores_flag_over_selections_and_in_a_batch():
    w = G.WORKLOADS["words_1k"]
    R, S, _, _ = G.make_host(w, n_r=700, n_s=900)
    Rd, Sd = _dev(R), _dev(S)
    ir = np.arange(1, 700, 2, dtype=np.int32)
    res = E.threshold_sel(Rd, _dev(ir), Sd, None, w.theta, d=w.d, prec="fp8", fp64_scores=True)
    r, s = res.r.cpu().numpy(), res.s.cpu().numpy()
    ref = O.sim64_pairs(R, S, r, s, d=w.d).astype(np.float32)
    np.testing.assert_array_equal(res.score.cpu().numpy(), ref)
    ori, osi, _, _ = O.threshold(R[ir], S, w.theta, d=w.d)
    assert set(zip(r.tolist(), s.tolist())) == set(zip(ir[ori].tolist(), osi.tolist()))
    jobs = [(Rd, Sd, w.theta), (Rd[:300], Rd[:300], 0.9), (Sd[:50], Rd, 0.85)]
    host = [(R, S, w.theta), (R[:300], R[:300], 0.9), (S[:50], R, 0.85)]
    for prec in ("bf16", "fp8"):
        out, _ = E.batch(jobs, d=w.d, prec=prec, fp64_scores=True)
        for got, (Rh, Sh, th) in zip(out, host):
            r, s = got.r.cpu().numpy(), got.s.cpu().numpy()
            ori, osi, _, _ = O.threshold(Rh, Sh, th, d=w.d)
            assert set(zip(r.tolist(), s.tolist())) == set(zip(ori.tolist(), osi.tolist()))
            ref = O.sim64_pairs(Rh, Sh, r, s, d=w.d).astype(np.float32)
            np.testing.assert_array_equal(got.score.cpu().numpy(), ref)


def test_panel_kernels_fit_the_workgroups_they_are_laid_out_for():
    """Every register-panel instantiation a threshold join can launch: the
    runtime's resident workgroups per CU reach the count the kernel's LDS
    ring, staging and registers were sized for (two for the two-workgroup
    forms, whose epilogues rely on the other workgroup's matrix work)."""
    depths = {"bf16": [64 * k for k in (1, 2, 3, 4, 5, 6, 8, 9, 10, 12)],
              "fp8": [128 * k for k in (1, 2, 3, 4, 5, 6)],
              "fp32": [32 * k for k in (1, 2, 3, 4, 5, 6, 8, 9, 10, 12)]}
    tiles = {12: "bf16", 13: "fp8", 14: "bf16", 15: "fp8", 20: "fp32", 21: "fp32",
             24: "bf16", 25: "fp8"}
    checked = 0
    for tile, prec in tiles.items():
        for d in depths[prec]:
            occ = E.tile_occupancy(tile, d)
            if occ is None:
                continue
            designed, resident = occ
            assert designed in (1, 2), (tile, d, designed)
            if tile in (14, 15, 21):
                assert designed == 2, (tile, d)
            assert resident >= designed, (tile, d, designed, resident)
            checked += 1
    assert checked >= 40
    assert E.tile_occupancy(3, 384) is None and E.tile_occupancy(14, 100000) is None


@pytest.mark.parametrize("prec,tile,d", [("bf16", 12, 96), ("bf16", 14, 96), ("fp8", 13, 128),
                                         ("fp32", 20, 64), ("fp32", 21, 64)])
def test_panel_epilogue_dense_hits(prec, tile, d):
    """The register panels' staged-record epilogue where hits are dense:
    every pair (each 32 x 32 block fills most of a wave's stage, so stages
    are written out inside a tile, and in the single join the workgroup's
    write-out step is called on every tile), half of the pairs (theta at the
    median: records mix certain pairs, band pairs and misses), and a pair
    list too small for the result (the true count, only valid distinct pairs
    written, then the exact set on retry).  Ragged |R| and |S| over several
    panels and S tiles."""
    R = G.gaussian_raw(600, d, seed=d + 31)
    S = G.gaussian_raw(900, d, seed=d + 32)
    Rn = R / np.linalg.norm(R, axis=1, keepdims=True)
    Sn = S / np.linalg.norm(S, axis=1, keepdims=True)
    median = float(np.median(Rn @ Sn.T))
    for theta in (-1.0, median):
        st = _check(R, S, theta, prec=prec, tile=tile)
        assert st["tile"] == tile
    Rd, Sd = _dev(R), _dev(S)
    ws = torch.empty(E.threshold_workspace(Rd, Sd, prec=prec, tile=tile), dtype=torch.uint8,
                     device="cuda")
    cap = 1000
    out = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
    rc, n, st = E.threshold_raw(Rd, Sd, -1.0, out, cap, ws, prec=prec, tile=tile)
    assert rc == E.E_OVERFLOW and n == 600 * 900
    o = out.cpu().numpy()
    assert o[:, 0].min() >= 0 and o[:, 0].max() < 600
    assert o[:, 1].min() >= 0 and o[:, 1].max() < 900
    assert len(set(zip(o[:, 0].tolist(), o[:, 1].tolist()))) == cap
    out = torch.empty((n, 3), dtype=torch.int32, device="cuda")
    rc, n2, st = E.threshold_raw(Rd, Sd, -1.0, out, n, ws, prec=prec, tile=tile)
    assert rc == E.OK and n2 == n
