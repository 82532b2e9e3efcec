"""Relational selections pushed below the join (the pre-filter of the
scan-versus-probe study, Section VI.E), against the oracle run on the
filtered relations.

The oracle side applies the selection the plain way (keep the passing rows,
join them, name the results by the original row ids); the GPU side takes the
id lists through the C ABI: the device range predicate, the threshold join
whose prep reads through the lists, and the top-k join over gathered rows.
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


def _ids(mask):
    return np.nonzero(mask)[0].astype(np.int32)


def _oracle_threshold(R, S, ir, is_, theta, d):
    ri, si, sc, _ = O.threshold(R[ir], S[is_], theta, d=d)
    return set(zip(ir[ri].tolist(), is_[si].tolist()))


@pytest.mark.parametrize("n,lo,hi", [(1_000_003, 0.25, 0.6), (5000, -1.0, 2.0), (777, 0.5, 0.5),
                                     (0, 0.0, 1.0), (300_000, 0.999, 1.0)])
def test_select_range_matches_the_predicate(n, lo, hi):
    rng = np.random.default_rng(n)
    col = rng.random(n).astype(np.float32)
    if n > 10:
        col[::97] = np.nan
    got = E.select_range(_dev(col), lo, hi).cpu().numpy()
    want = _ids((lo <= col) & (col < hi))
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("sr,ss", [(0.3, 0.5), (1.0, 0.01), (0.0, 0.5), (0.7, 1.0)])
def test_threshold_over_selections(prec, sr, ss):
    w = G.WORKLOADS["words_1k"]
    R, S, _, _ = G.make_host(w, n_r=1500, n_s=2300)
    rng = np.random.default_rng(int(sr * 100 + ss * 1000))
    ar, as_ = rng.random(R.shape[0]).astype(np.float32), rng.random(S.shape[0]).astype(np.float32)
    Rd, Sd = _dev(R), _dev(S)
    sel_r = E.select_range(_dev(ar), 0.0, sr)
    sel_s = E.select_range(_dev(as_), 0.0, ss)
    ir, is_ = _ids(ar < sr), _ids(as_ < ss)
    np.testing.assert_array_equal(sel_r.cpu().numpy(), ir)
    res = E.threshold_sel(Rd, sel_r, Sd, sel_s, w.theta, d=w.d, prec=prec,
                          band_capacity=1 << 20)
    got = set(zip(res.r.cpu().tolist(), res.s.cpu().tolist()))
    assert len(got) == len(res)
    assert got == _oracle_threshold(R, S, ir, is_, w.theta, w.d)
    if len(res):
        ref = O.sim64_pairs(R, S, res.r.cpu().numpy(), res.s.cpu().numpy(), d=w.d)
        tol = 1e-3 if prec == "fp32" else res.stats["band"]
        assert np.abs(res.score.cpu().numpy() - ref).max() <= tol


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_threshold_selection_of_one_side_and_self_join(prec):
    w = G.WORKLOADS["words_1k"]
    R, S, _, _ = G.make_host(w, n_r=900, n_s=1100)
    Rd, Sd = _dev(R), _dev(S)
    ir = np.arange(0, 900, 3, dtype=np.int32)
    is_ = np.arange(5, 1100, 7, dtype=np.int32)
    every_r, every_s = np.arange(900, dtype=np.int32), np.arange(1100, dtype=np.int32)
    res = E.threshold_sel(Rd, None, Sd, _dev(is_), w.theta, d=w.d, prec=prec)
    assert set(zip(res.r.cpu().tolist(), res.s.cpu().tolist())) == \
        _oracle_threshold(R, S, every_r, is_, w.theta, w.d)
    # self-join through one selection (prepared once) ...
    sr = _dev(ir)
    res = E.threshold_sel(Rd, sr, Rd, sr, w.theta, d=w.d, prec=prec)
    want = _oracle_threshold(R, R, ir, ir, w.theta, w.d)
    assert set(zip(res.r.cpu().tolist(), res.s.cpu().tolist())) == want
    assert all((i, i) in want for i in ir.tolist())
    # ... and the same relation under two different selections of one size
    other = _dev(ir + 1)
    res = E.threshold_sel(Rd, sr, Rd, other, w.theta, d=w.d, prec=prec)
    assert set(zip(res.r.cpu().tolist(), res.s.cpu().tolist())) == \
        _oracle_threshold(R, R, ir, ir + 1, w.theta, w.d)
    del every_s


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("k,ss", [(1, 0.05), (32, 0.4), (10, 1.0)])
def test_topk_over_selections(prec, k, ss):
    cent = G.centres(128, 40, seed=3)
    R, _ = G.clustered_points(cent, 400, 0.3, seed=4)
    S, _ = G.clustered_points(cent, 6000, 0.3, seed=5)
    S[100:110] = S[3]                            # ties across selected rows
    rng = np.random.default_rng(k)
    is_ = _ids(rng.random(S.shape[0]) < ss)
    ir = np.arange(1, 400, 2, dtype=np.int32)
    idx, sc, st = E.topk_sel(_dev(R), _dev(ir), _dev(S), _dev(is_), k, prec=prec)
    oi, osc = O.topk(R[ir], S[is_], k)
    want = np.where(oi >= 0, is_[np.maximum(oi, 0)], -1)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), want)
    np.testing.assert_array_equal(sc.cpu().numpy(), osc.astype(np.float32))


def test_topk_selection_self_join_and_no_sync():
    cent = G.centres(96, 10, seed=6)
    X, _ = G.clustered_points(cent, 3000, 0.3, seed=7)
    ids = np.arange(0, 3000, 4, dtype=np.int32)
    sel = _dev(ids)
    idx, sc, _ = E.topk_sel(_dev(X), sel, _dev(X), sel, 5, prec="bf16", flags=E.NO_SYNC)
    torch.cuda.synchronize()
    oi, osc = O.topk(X[ids], X[ids], 5)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), ids[oi])
    assert np.array_equal(idx.cpu().numpy()[:, 0], ids)  # every row is its own best match


def test_bad_selections_are_refused():
    R = _dev(G.gaussian_raw(300, 40, seed=1))
    for bad in (np.array([3, 2, 7], np.int32), np.array([1, 1], np.int32),
                np.array([0, 300], np.int32), np.array([-1, 4], np.int32)):
        with pytest.raises(E.EjoinError) as ex:
            E.threshold_sel(R, _dev(bad), R, None, 0.5, prec="bf16")
        assert ex.value.status == E.E_INVAL
        with pytest.raises(E.EjoinError) as ex:
            E.topk_sel(R, None, R, _dev(bad), 3, prec="fp32")
        assert ex.value.status == E.E_INVAL
    # asynchronous: the device count carries -EJOIN_E_INVAL
    bad = _dev(np.array([5, 4], np.int32))
    ws = torch.empty(E.threshold_sel_workspace(R, bad, R, None, prec="fp32"), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty((16, 3), dtype=torch.int32, device="cuda")
    n_dev = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc, _, _ = E.threshold_sel_raw(R, bad, R, None, 0.5, out, 16, ws, flags=E.NO_SYNC,
                                   n_out_dev=n_dev)
    assert rc == E.OK and int(n_dev.item()) == -E.E_INVAL
    # a selection longer than its relation is refused on the host
    with pytest.raises(E.EjoinError):
        E.threshold_sel(R, _dev(np.arange(301, dtype=np.int32)), R, None, 0.5)


def test_range_top_k_over_a_selection():
    """The paper's range join with k = 32 after a pre-filter on S."""
    cent = G.centres(300, 100, seed=9)
    R, _ = G.clustered_points(cent, 300, 0.25, seed=10)
    S, _ = G.clustered_points(cent, 20000, 0.25, seed=11)
    attr = np.random.default_rng(12).random(S.shape[0]).astype(np.float32)
    sel = E.select_range(_dev(attr), 0.0, 0.4)
    is_ = _ids(attr < 0.4)
    idx, sc, _ = E.topk_sel(_dev(R), None, _dev(S), sel, 32, prec="fp32", min_sim=0.9)
    oi, osc = O.topk_range(R, S[is_], 32, 0.9)
    want = np.where(oi >= 0, is_[np.maximum(oi, 0)], -1)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), want)
    np.testing.assert_array_equal(sc.cpu().numpy(), osc.astype(np.float32))
