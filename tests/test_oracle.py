"""Pins of the FP64 oracle against things other than itself.

* exact-rational brute force on tiny inputs (decision and top-k order);
* closed forms: d = 1, orthonormal rows, x versus 2^k x, theta <= -1,
  theta > 1, zero rows, self-join at theta = 1;
* invariants: bitwise symmetry, unit diagonal, count == list length;
* the clustered generator's closed-form count sum_c |R_c||S_c| (labels come
  from the generator, the margin from an independent numpy matmul);
* the paper's printed sizes (micro-sweep shapes).

A plausible slip in the oracle (a dropped term, a transposed operand, a wrong
comparison, a wrong tie rule) fails at least one of these.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import exact
from oracle import oracle as O
from paper_2312_01476_amd import datagen as G

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(seed, n_r, n_s, d, dup=True, zero=True):
    rng = np.random.Generator(np.random.PCG64(seed))
    R = rng.standard_normal((n_r, d)).astype(np.float32)
    S = rng.standard_normal((n_s, d)).astype(np.float32)
    if dup and n_s > 2:
        S[1] = R[0]                  # exact duplicate across relations
        S[2] = S[1] * np.float32(4)  # scaled copy: cosine exactly 1
    if zero and n_r > 3:
        R[3] = 0.0                   # zero row
    return R, S


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
def test_threshold_matches_exact_rational(seed, d):
    R, S = _tiny(seed, 7, 9, d)
    sims = O.sim_matrix(R, S)
    # thresholds between attained values, on attained values, and outside
    cand = np.unique(sims)
    thetas = [-1.5, -0.5, 0.0, 0.3, 0.999, 1.0, 1.5]
    thetas += list(cand[:: max(1, len(cand) // 6)])
    for th in thetas:
        ri, si, sc, ties = O.threshold(R, S, float(th))
        got = set(zip(ri.tolist(), si.tolist()))
        want = exact.threshold(R, S, float(th))
        if got != want:
            # only pairs that the FP64 oracle itself flags as ties may differ
            diff = got ^ want
            for (i, j) in diff:
                assert abs(sims[i, j] - th) < 1e-12, (th, i, j, sims[i, j])
        assert len(ri) == len(got)
        np.testing.assert_array_equal(sc, sims[ri, si])


def test_planted_near_ties_agree_with_exact():
    rng = np.random.Generator(np.random.PCG64(7))
    R = rng.standard_normal((5, 6)).astype(np.float32)
    S = rng.standard_normal((6, 6)).astype(np.float32)
    sims = O.sim_matrix(R, S)
    for (i, j) in [(0, 0), (1, 2), (4, 5)]:
        for off in (-1e-7, -1e-9, 1e-9, 1e-7):
            th = float(sims[i, j] + off)
            inside = exact.matches([exact.Fraction(float(v)) for v in R[i]],
                                   [exact.Fraction(float(v)) for v in S[j]], th)
            ri, si, _, _ = O.threshold(R[i:i + 1], S[j:j + 1], th)
            assert (len(ri) == 1) == inside == (off < 0)


@pytest.mark.parametrize("seed", range(4))
def test_topk_matches_exact_rational_with_ties(seed):
    R, S = _tiny(seed, 6, 10, 4)
    S[7] = S[5]          # exact tie inside S: smaller index must come first
    S[9] = S[5] * 2      # scaled tie
    for k in (1, 3, 10, 13):
        idx, sc = O.topk(R, S, k)
        want = exact.topk(R, S, k)
        np.testing.assert_array_equal(idx, want)
        # sorted by score desc, index asc; padding beyond |S|
        for row_i, row_s in zip(idx, sc):
            valid = row_i >= 0
            assert np.all(np.diff(row_s[valid]) <= 0)
            assert np.all(row_s[~valid] == -np.inf)
            assert valid.sum() == min(k, S.shape[0])


def test_d1_is_sign_agreement():
    rng = np.random.Generator(np.random.PCG64(3))
    R = rng.standard_normal((40, 1)).astype(np.float32)
    S = rng.standard_normal((50, 1)).astype(np.float32)
    sims = O.sim_matrix(R, S)
    want = np.where(np.sign(R[:, 0])[:, None] == np.sign(S[:, 0])[None, :], 1.0, -1.0)
    np.testing.assert_array_equal(sims, want)
    ri, si, _, _ = O.threshold(R, S, 0.5)
    assert len(ri) == int((want == 1.0).sum())


def test_orthonormal_rows_give_zero_or_one():
    d = 16
    E = np.eye(d, dtype=np.float32)
    sims = O.sim_matrix(E, E[::-1].copy())
    want = np.eye(d)[::-1]
    np.testing.assert_array_equal(sims, want)


@pytest.mark.parametrize("k", [-20, -3, 0, 5, 40])
def test_scaled_copy_is_exactly_one(k):
    rng = np.random.Generator(np.random.PCG64(11))
    for _ in range(50):
        x = rng.standard_normal(37).astype(np.float32)
        y = (x * np.float32(2.0 ** k)).astype(np.float32)
        assert O.sim64(x, y) == 1.0
        assert O.sim64(x, -y) == -1.0


def test_symmetry_and_unit_diagonal():
    X = G.gaussian_raw(200, 300, seed=5, scale=3.0)
    sims = O.sim_matrix(X, X)
    assert np.array_equal(sims, sims.T)          # bitwise symmetric
    assert np.all(np.diag(sims) == 1.0)          # exactly one


def test_theta_extremes_and_zero_rows():
    R, S = _tiny(1, 8, 9, 5)
    nz_r = np.count_nonzero(np.any(R != 0, axis=1))
    ri, si, _, _ = O.threshold(R, S, -1.0)
    assert len(ri) == R.shape[0] * S.shape[0]         # everything, incl. zero rows (0 >= -1)
    ri, si, _, _ = O.threshold(R, S, 1.0 + 1e-6)
    assert len(ri) == 0
    # zero row of R pairs with every S at similarity 0: in iff theta <= 0
    sims = O.sim_matrix(R, S)
    assert np.all(sims[3] == 0.0)
    ri, si, _, _ = O.threshold(R, S, 0.0)
    assert set(si[ri == 3].tolist()) == set(range(S.shape[0]))
    ri, si, _, _ = O.threshold(R, S, 1e-300)
    assert 3 not in set(ri.tolist())
    assert nz_r == R.shape[0] - 1


def test_self_join_theta_one_is_diagonal_plus_parallel_copies():
    X = G.gaussian_raw(30, 12, seed=9)
    X[10] = X[4]
    X[20] = X[4] * np.float32(0.5)
    ri, si, sc, _ = O.threshold(X, X, 1.0)
    got = set(zip(ri.tolist(), si.tolist()))
    grp = {4, 10, 20}
    want = {(i, i) for i in range(30)} | {(a, b) for a in grp for b in grp}
    assert got == want
    assert np.all(sc == 1.0)


def test_nonfinite_rejected():
    R, S = _tiny(0, 4, 4, 3)
    R[2, 1] = np.nan
    with pytest.raises(O.OracleError):
        O.threshold(R, S, 0.5)
    with pytest.raises(O.OracleError):
        O.topk(R, S, 2)


def test_padding_columns_ignored():
    R, S, _, _ = G.make_host(G.WORKLOADS["words_1k"], n_r=60, n_s=70, pad_value=np.nan)
    a = O.threshold(R, S, 0.8, d=300)
    b = O.threshold(np.ascontiguousarray(R[:, :300]), np.ascontiguousarray(S[:, :300]), 0.8)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)


def test_words_1k_closed_form_count():
    """All 10^6 pairs of the 1k x 1k word workload against the generator's
    label count; the margin is checked with an independent numpy product."""
    w = G.WORKLOADS["words_1k"]
    R, S, lr, ls = G.make_host(w)
    Rn = R[:, : w.d].astype(np.float64)
    Sn = S[:, : w.d].astype(np.float64)
    Rn /= np.linalg.norm(Rn, axis=1, keepdims=True)
    Sn /= np.linalg.norm(Sn, axis=1, keepdims=True)
    cos = Rn @ Sn.T
    same = lr[:, None] == ls[None, :]
    assert cos[same].min() > w.theta + 0.05 and cos[~same].max() < w.theta - 0.3
    ri, si, sc, ties = O.threshold(R, S, w.theta, d=w.d)
    assert len(ri) == int(same.sum())
    assert ties == 0
    # the pairs are exactly the same-cluster pairs, and the scores agree with
    # the library product to rounding
    assert np.all(lr[ri] == ls[si])
    np.testing.assert_allclose(sc, cos[ri, si], atol=1e-12)
    # sorted (i, j) output
    key = ri.astype(np.int64) * S.shape[0] + si
    assert np.all(np.diff(key) > 0)


def test_topk_closed_form_cluster_membership():
    """With many same-cluster S per row, every top-k entry shares the row's
    cluster label and scores agree with an independent numpy product."""
    cent = G.centres(64, 8, seed=21)
    R, lr = G.clustered_points(cent, 40, 0.3, seed=22)
    S, ls = G.clustered_points(cent, 400, 0.3, seed=23)
    idx, sc = O.topk(R, S, 10)
    assert np.all(ls[idx] == lr[:, None])
    Rn = R.astype(np.float64) / np.linalg.norm(R.astype(np.float64), axis=1, keepdims=True)
    Sn = S.astype(np.float64) / np.linalg.norm(S.astype(np.float64), axis=1, keepdims=True)
    full = Rn @ Sn.T
    np.testing.assert_allclose(sc, np.take_along_axis(full, idx, 1), atol=1e-12)
    # each row's list is the true top-10 of the numpy product (no near ties here)
    for i in range(R.shape[0]):
        order = np.argsort(-full[i], kind="stable")[:10]
        assert set(order.tolist()) == set(idx[i].tolist())


def test_threads_do_not_change_results():
    R = G.gaussian_raw(120, 33, seed=1)
    S = G.gaussian_raw(130, 33, seed=2)
    a = O.threshold(R, S, 0.2, threads=1)
    b = O.threshold(R, S, 0.2, threads=4)
    for x, y in zip(a[:3], b[:3]):
        np.testing.assert_array_equal(x, y)
    i1, s1 = O.topk(R, S, 7, threads=1)
    i4, s4 = O.topk(R, S, 7, threads=3)
    np.testing.assert_array_equal(i1, i4)
    np.testing.assert_array_equal(s1, s4)


def test_paper_printed_sizes():
    gold = json.load(open(os.path.join(GOLD, "paper_sizes.json")))
    for ops, dim, side in gold["micro_sweep"]["cases"]:
        assert G.micro_sweep_side(ops, dim) == side
    dn = gold["dense_intermediate"]
    dense = dn["n_r"] * dn["n_s"] * dn["bytes_per_value"]
    assert math.isclose(dense, dn["approx_bytes"], rel_tol=1e-9)
    l1 = gold["l1_capacity"]
    assert l1["cache_bytes"] // (l1["dim"] * l1["bytes_per_value"]) == l1["vectors"]



@pytest.mark.parametrize("seed", [1, 2, 3])
def test_topk_range_matches_exact_rational(seed):
    """Range + top-k: the FP64 definition agrees with the exact-rational
    brute force (ties planted by duplicate rows; thresholds inside the
    similarity range so that rows have fewer, more or exactly k matches)."""
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((7, 5)).astype(np.float32)
    S = rng.standard_normal((23, 5)).astype(np.float32)
    S[4] = S[9]
    S[11] = 2 * S[3]
    for theta in (-0.2, 0.1, 0.4, 0.95):
        gi, gs = O.topk_range(R, S, 4, theta)
        want = exact.topk_range(R, S, 4, theta)
        np.testing.assert_array_equal(gi, want)
        assert np.all(np.isfinite(gs) == (gi >= 0))
        assert np.all(gs[gi >= 0] >= theta)


def test_topk_range_reduces_to_topk_and_to_threshold():
    """theta <= -1 keeps every column (plain top-k); k >= |S| gives each
    row's whole threshold set, sorted."""
    rng = np.random.default_rng(5)
    R = rng.standard_normal((9, 12)).astype(np.float32)
    S = rng.standard_normal((40, 12)).astype(np.float32)
    gi, gs = O.topk_range(R, S, 6, -1.0)
    ti, ts = O.topk(R, S, 6)
    np.testing.assert_array_equal(gi, ti)
    np.testing.assert_array_equal(gs, ts)
    gi, gs = O.topk_range(R, S, 40, 0.2)
    ri, si, sc, _ = O.threshold(R, S, 0.2)
    for i in range(9):
        m = ri == i
        assert sorted(gi[i][gi[i] >= 0].tolist()) == sorted(si[m].tolist())
