"""Bit-identity of the GPU's FP64 rescore with the canonical rule.

The exact result set rests on the GPU evaluating
    sim64(r, s) = dot(r, s) / sqrt(dot(r, r) * dot(s, s))
with the same sequential sums, one rounding per product and per sum and the
correctly rounded sqrt and divide as the oracle (the cosine equation of
Section III.A, evaluated as the canonical FP64 rule).  A fused multiply-add,
another summation order or an approximate sqrt/divide would move sim64 by a
few ulps; these tests are built so that a few ulps change the answer:

  * theta set to a pair's exact sim64 must accept it, and theta one ulp
    above must reject it (one job per pair in a batch, every precision);
  * relations whose similarities differ only in the last bits: S holds
    permutations of one vector and R an all-ones row, so every dot sums the
    same values in another order; threshold joins cut inside that spread
    and top-k rankings are decided by it (sweep and fallback paths).
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


def _perm_family(d, n, seed):
    """An all-ones row, a scaled copy of it and two Gaussian rows (R); n
    permutations of one Gaussian vector (S)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal(d).astype(np.float32)
    S = np.stack([v[rng.permutation(d)] for _ in range(n)]).astype(np.float32)
    R = np.stack([np.ones(d, np.float32), np.full(d, 3.0, np.float32),
                  rng.standard_normal(d).astype(np.float32), v]).astype(np.float32)
    return R, S


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("d", [1, 3, 300, 768])
def test_theta_at_sim64_accepts_and_next_ulp_rejects(prec, d):
    n = 1024
    R = G.gaussian_raw(n, d, seed=1000 + d)
    S = G.gaussian_raw(n, d, seed=2000 + d)
    if d > 1:
        S[: n // 4] = R[: n // 4] * np.float32(0.5) + S[: n // 4] * np.float32(0.01)  # near 1
    idx = np.arange(n)
    sims = O.sim64_pairs(R, S, idx, idx)
    up = np.nextafter(sims, np.inf)
    Rd, Sd = _dev(R), _dev(S)
    jobs = []
    for p in range(n):
        jobs.append((Rd[p:p + 1], Sd[p:p + 1], float(sims[p])))
        jobs.append((Rd[p:p + 1], Sd[p:p + 1], float(up[p])))
    res, st = E.batch(jobs, prec=prec, capacities=[1] * len(jobs), band_capacity=2 * len(jobs))
    got_at = np.array([len(res[2 * p]) for p in range(n)])
    got_up = np.array([len(res[2 * p + 1]) for p in range(n)])
    assert got_at.min() == 1, f"{prec} d={d}: pairs at theta = sim64 rejected: " \
                              f"{np.nonzero(got_at == 0)[0][:5]}"
    assert got_up.max() == 0, f"{prec} d={d}: pairs at theta = next ulp above accepted: " \
                              f"{np.nonzero(got_up)[0][:5]}"
    scores = np.array([float(res[2 * p].score.cpu()[0]) for p in range(0, n, 97)])
    np.testing.assert_array_equal(scores, sims[::97].astype(np.float32))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("d", [300, 768])
def test_threshold_cut_inside_ulp_spread(prec, d):
    R, S = _perm_family(d, 4000, seed=d)
    sims = O.sim_matrix(R, S)
    spread = np.unique(sims[0])
    assert spread.size >= 5 and spread[-1] - spread[0] < 1e-15  # a few ulps apart
    Rd, Sd = _dev(R), _dev(S)
    for theta in (float(np.median(sims[0])), float(spread[1]), float(spread[-2])):
        res = E.threshold(Rd, Sd, theta, prec=prec)
        got = set(zip(res.r.cpu().tolist(), res.s.cpu().tolist()))
        ri, si, sc, _ = O.threshold(R, S, theta)
        want = set(zip(ri.tolist(), si.tolist()))
        assert got == want, (prec, d, theta, len(got ^ want))
        # the rescored scores are float(sim64) of the same pairs
        r = res.r.cpu().numpy().astype(np.int64)
        s = res.s.cpu().numpy().astype(np.int64)
        row0 = r == 0
        np.testing.assert_array_equal(res.score.cpu().numpy()[row0],
                                      sims[0, s[row0]].astype(np.float32))


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
@pytest.mark.parametrize("cand", [0, 10])
def test_topk_ranked_by_last_ulps(prec, cand):
    """Candidates a few ulps apart are ranked by their exact sim64 (ties by
    index); with 10 slots for k = 10 the rows overflow and take the exact
    scan, which must rank them the same way."""
    R, S = _perm_family(300, 240, seed=5)
    S = np.concatenate([S, S[:16]])           # exact duplicates: ties broken by index
    k = 10
    idx, sc, st = E.topk(_dev(R), _dev(S), k, prec=prec, topk_cand=cand)
    oi, osc = O.topk(R, S, k)
    np.testing.assert_array_equal(idx.cpu().numpy().astype(np.int64), oi)
    np.testing.assert_array_equal(sc.cpu().numpy(), osc.astype(np.float32))
    if cand:
        assert st["n_fallback"] > 0
