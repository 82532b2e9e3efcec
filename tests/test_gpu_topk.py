"""Parity of the GPU top-k join (through the C ABI) with the FP64 oracle.

Indices must equal the oracle's exactly (including the order of ties, which
the canonical rule breaks by the smaller S index) and every score must equal
the oracle's sim64 rounded to float32.
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


PANEL = {"fp32": 21, "bf16": 14, "fp8": 13}   # register-panel sweep
SQUARE = {"fp32": 1, "bf16": 3, "fp8": 5}     # 128 x 128 tile sweep


def _check(R, S, k, prec, d=None, **kw):
    idx, sc, st = E.topk(_dev(R), _dev(S), k, d=d, prec=prec, **kw)
    oi, osc = O.topk(R, S, k, d=d)
    gi = idx.cpu().numpy().astype(np.int64)
    gs = sc.cpu().numpy()
    bad = np.nonzero(np.any(gi != oi, axis=1))[0]
    assert bad.size == 0, (prec, k, bad[:5], gi[bad[:2]], oi[bad[:2]], st)
    np.testing.assert_array_equal(gs, osc.astype(np.float32))
    return st


@pytest.mark.parametrize("form", ["panel", "tile"])
@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("k", [1, 3, 10, 37])
def test_clustered(prec, k, form):
    cent = G.centres(128, 30, seed=1)
    R, _ = G.clustered_points(cent, 700, 0.3, seed=2)
    S, _ = G.clustered_points(cent, 3000, 0.3, seed=3)
    tile = (PANEL if form == "panel" else SQUARE)[prec]
    st = _check(R, S, k, prec, tile=tile)
    assert st["tile"] == tile
    assert st["n_fallback"] < R.shape[0] // 10


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_ties_and_duplicates(prec):
    cent = G.centres(64, 10, seed=4)
    R, _ = G.clustered_points(cent, 300, 0.3, seed=5)
    S, _ = G.clustered_points(cent, 1500, 0.3, seed=6)
    S[100:110] = S[5]                         # exact ties: order by index
    S[200] = S[5] * np.float32(4.0)           # scaled copy: same similarity
    R[7] = S[5]
    R[8] = 0.0                                # zero row: all similarities 0
    _check(R, S, 16, prec, tile=PANEL[prec])
    _check(R, S, 16, prec, tile=SQUARE[prec])


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_k_larger_than_s_and_small_s(prec):
    R = G.gaussian_raw(50, 40, seed=7)
    S = G.gaussian_raw(9, 40, seed=8)
    _check(R, S, 12, prec)    # k > |S|: padding
    _check(R, S, 9, prec)
    S2 = G.gaussian_raw(200, 40, seed=9)
    _check(R, S2, 5, prec)    # |S| <= slots: every column a candidate


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_forced_fallback_is_exact(prec):
    """Few slots per row: most rows overflow and take the exact scan."""
    cent = G.centres(96, 5, seed=10)
    R, _ = G.clustered_points(cent, 400, 0.3, seed=11)
    S, _ = G.clustered_points(cent, 2500, 0.3, seed=12)
    st = _check(R, S, 8, prec, topk_cand=8, tile=PANEL[prec])
    assert st["n_fallback"] > 0
    st = _check(R, S, 8, prec, topk_cand=8, tile=SQUARE[prec])
    assert st["n_fallback"] > 0


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_unstructured_data(prec):
    R = G.uniform_sphere(333, 200, seed=13)
    S = G.uniform_sphere(4100, 200, seed=14)
    _check(R, S, 10, prec)


@pytest.mark.parametrize("prec,d", [("bf16", 384), ("fp8", 768), ("fp8", 300), ("bf16", 33)])
def test_depths_and_ragged(prec, d):
    cent = G.centres(d, 50, seed=d)
    R, _ = G.clustered_points(cent, 517, 0.3, seed=d + 1)
    S, _ = G.clustered_points(cent, 2711, 0.3, seed=d + 2)
    _check(R, S, 10, prec)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_large_s_strided_pilot(prec):
    """|S| >= 65536: the pilot sets the floor from every 4th column; the
    result must still be the exact top-k (rows checked in full)."""
    cent = G.centres(64, 400, seed=21)
    R, _ = G.clustered_points(cent, 256, 0.3, seed=22)
    S, _ = G.clustered_points(cent, 70000, 0.3, seed=23)
    for tile in (PANEL[prec], SQUARE[prec]):
        st = _check(R, S, 10, prec, tile=tile)
        assert st["n_fallback"] < R.shape[0] // 4


def test_invalid():
    R = _dev(G.gaussian_raw(10, 8, seed=1))
    for tile in (2, 12, 16, 23):              # not a top-k form of FP32
        with pytest.raises(E.EjoinError):
            E.topk(R, R, 4, prec="fp32", tile=tile)
    with pytest.raises(E.EjoinError):         # a panel form at a depth without one
        E.topk(_dev(G.gaussian_raw(10, 1024, seed=1)), _dev(G.gaussian_raw(10, 1024, seed=2)),
               4, prec="fp32", tile=21)
    with pytest.raises(E.EjoinError):
        E.topk(R, R, 0, prec="bf16")
    with pytest.raises(E.EjoinError):
        E.topk(R, R, 300, prec="bf16")


@pytest.mark.parametrize("prec,d", [("fp32", 40), ("fp32", 300), ("fp32", 384), ("fp32", 500),
                                    ("fp32", 1024), ("bf16", 448), ("bf16", 640),
                                    ("bf16", 768), ("bf16", 1024), ("fp8", 1024)])
def test_every_depth(prec, d):
    """Register-panel sweeps (FP32 up to 12 K slices, BF16 8-12) and the
    tile-kernel sweep for the other depths (FP32 500- and 1024-d, BF16 448-
    and 1024-d, FP8 1024-d): indices and scores exact."""
    cent = G.centres(d, 40, seed=d + 5)
    R, _ = G.clustered_points(cent, 300, 0.3, seed=d + 6)
    S, _ = G.clustered_points(cent, 3100, 0.3, seed=d + 7)
    S[50:60] = S[7]                            # exact ties
    st = _check(R, S, 10, prec)
    assert st["n_fallback"] < R.shape[0] // 10
    if d in (40, 300, 384, 640, 768):          # depths with a panel form
        st = _check(R, S, 10, prec, tile=PANEL[prec])
        assert st["tile"] == PANEL[prec]


@pytest.mark.parametrize("prec,d", [("fp32", 300), ("bf16", 1024)])
def test_deep_and_plain_forced_fallback(prec, d):
    cent = G.centres(d, 5, seed=30)
    R, _ = G.clustered_points(cent, 200, 0.3, seed=31)
    S, _ = G.clustered_points(cent, 1500, 0.3, seed=32)
    st = _check(R, S, 8, prec, topk_cand=8)
    assert st["n_fallback"] > 0


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("cand", [0, 8])
def test_async_call(prec, cand):
    """EJOIN_NO_SYNC: no host wait inside the call; uncertified rows take the
    device-side fallback (one workgroup per listed row).  With 8 slots for
    k = 8 most rows overflow and go that way."""
    cent = G.centres(96, 5, seed=40)
    R, _ = G.clustered_points(cent, 333, 0.3, seed=41)
    S, _ = G.clustered_points(cent, 2100, 0.3, seed=42)
    Rd, Sd = _dev(R), _dev(S)
    k = 8
    ws = torch.empty(E.topk_workspace(Rd, Sd, k, prec=prec, topk_cand=cand), dtype=torch.uint8,
                     device="cuda")
    idx = torch.full((R.shape[0], k), -7, dtype=torch.int32, device="cuda")
    sc = torch.zeros((R.shape[0], k), dtype=torch.float32, device="cuda")
    rc, _ = E.topk_raw(Rd, Sd, k, idx, sc, ws, prec=prec, topk_cand=cand, flags=E.NO_SYNC)
    assert rc == E.OK
    torch.cuda.synchronize()
    oi, osc = O.topk(R, S, k)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), oi)
    np.testing.assert_array_equal(sc.cpu().numpy(), osc.astype(np.float32))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("flags", [0, 1])
def test_failed_input_check_leaves_stale_workspace_unread(prec, flags):
    """A NaN row fails the input check, so the sweep writes no candidate
    counters; the finalize must not read the workspace's stale contents.  The
    workspace is filled with a pattern whose int32 counters read as 5 and
    whose candidate columns read as -1000000 (an index out of every buffer)."""
    R = G.gaussian_raw(200, 64, seed=50)
    S = G.gaussian_raw(700, 64, seed=51)
    R[17, 3] = np.nan
    Rd, Sd = _dev(R), _dev(S)
    k = 4
    n = E.topk_workspace(Rd, Sd, k, prec=prec)
    word = (5 << 32) | ((-1000000) & 0xFFFFFFFF)
    pat = torch.full(((n + 7) // 8,), word, dtype=torch.int64, device="cuda")
    ws = pat.view(torch.uint8)[:n]
    idx = torch.zeros((200, k), dtype=torch.int32, device="cuda")
    sc = torch.zeros((200, k), dtype=torch.float32, device="cuda")
    rc, _ = E.topk_raw(Rd, Sd, k, idx, sc, ws, prec=prec, flags=flags)
    torch.cuda.synchronize()
    assert rc == (E.OK if flags else E.E_NONFINITE)
    assert int(idx.abs().max()) == 0   # outputs untouched


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("form", ["panel", "tile"])
def test_overflowed_rows_are_refined(prec, form):
    """Clusters of ~600 rows against k = 32 and 256 slots: every row's slots
    overflow at the pilot's floor; the second sweep with per-row floors must
    certify them (exact indices and scores) without the exact scan in FP32
    and BF16.  FP8's error bound (about 0.06 per score here) keeps a whole
    cluster within twice the bound of the k-th score, more than 256 slots, so
    its rows still take the exact scan: the result is exact either way."""
    cent = G.centres(96, 8, seed=60)
    R, _ = G.clustered_points(cent, 300, 0.3, seed=61)
    S, _ = G.clustered_points(cent, 5000, 0.3, seed=62)
    tile = (PANEL if form == "panel" else SQUARE)[prec]
    st = _check(R, S, 32, prec, tile=tile)
    assert st["topk_refined"] > R.shape[0] // 2
    if prec != "fp8":
        assert st["n_fallback"] < R.shape[0] // 10


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("form", ["panel", "tile"])
@pytest.mark.parametrize("theta,k", [(0.9, 32), (0.93, 5), (0.5, 10), (-1.0, 7), (0.99, 3)])
def test_range_with_k_cap(prec, form, theta, k):
    """sim >= theta combined with the top-k condition: per row the first
    min(k, m) of its m passing S rows, padded; decided in FP64 (scores exact,
    indices exact, ties by index)."""
    cent = G.centres(128, 20, seed=70)
    R, _ = G.clustered_points(cent, 400, 0.3, seed=71)
    S, _ = G.clustered_points(cent, 3000, 0.3, seed=72)
    S[10:20] = S[0]
    tile = (PANEL if form == "panel" else SQUARE)[prec]
    idx, sc, st = E.topk(_dev(R), _dev(S), k, prec=prec, tile=tile, min_sim=theta)
    oi, osc = O.topk_range(R, S, k, theta)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), oi)
    np.testing.assert_array_equal(sc.cpu().numpy(), osc.astype(np.float32))
    if theta > 0.9:
        assert (oi < 0).any()        # rows with fewer than k passing S rows


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_range_with_k_cap_fallback_and_async(prec):
    cent = G.centres(96, 5, seed=73)
    R, _ = G.clustered_points(cent, 200, 0.3, seed=74)
    S, _ = G.clustered_points(cent, 2000, 0.3, seed=75)
    Rd, Sd = _dev(R), _dev(S)
    oi, osc = O.topk_range(R, S, 8, 0.9)
    # 8 slots for k = 8: overflow, refinement and exact scans with the bound
    idx, sc, st = E.topk(Rd, Sd, 8, prec=prec, topk_cand=8, min_sim=0.9)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), oi)
    np.testing.assert_array_equal(sc.cpu().numpy(), osc.astype(np.float32))
    ws = torch.empty(E.topk_workspace(Rd, Sd, 8, prec=prec, topk_cand=8, min_sim=0.9),
                     dtype=torch.uint8, device="cuda")
    idx = torch.empty((200, 8), dtype=torch.int32, device="cuda")
    sc = torch.empty((200, 8), dtype=torch.float32, device="cuda")
    rc, _ = E.topk_raw(Rd, Sd, 8, idx, sc, ws, prec=prec, topk_cand=8, flags=E.NO_SYNC,
                       min_sim=0.9)
    torch.cuda.synchronize()
    assert rc == E.OK
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), oi)
    with pytest.raises(E.EjoinError):
        E.topk(Rd, Sd, 8, prec=prec, min_sim=float("nan"))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("nq", [1, 7, 100])
def test_e_selection_query_batches(prec, nq):
    """E-selection: a batch of query vectors as R against a relation,
    answered by the same join (threshold, top-k and range + top-k)."""
    cent = G.centres(200, 50, seed=80)
    Q, _ = G.clustered_points(cent, nq, 0.3, seed=81)
    S, _ = G.clustered_points(cent, 20000, 0.3, seed=82)
    Qd, Sd = _dev(Q), _dev(S)
    res = E.threshold(Qd, Sd, 0.85, prec=prec)
    got = set(zip(res.r.cpu().tolist(), res.s.cpu().tolist()))
    ri, si, _, _ = O.threshold(Q, S, 0.85)
    assert got == set(zip(ri.tolist(), si.tolist()))
    idx, sc, _ = E.topk(Qd, Sd, 12, prec=prec)
    oi, osc = O.topk(Q, S, 12)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), oi)
    idx, sc, _ = E.topk(Qd, Sd, 12, prec=prec, min_sim=0.9)
    oi, osc = O.topk_range(Q, S, 12, 0.9)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), oi)
    np.testing.assert_array_equal(sc.cpu().numpy(), osc.astype(np.float32))
