"""The prefilter's inference side against the FP64 reference of its steps.

oracle/prefilter.py predicts, from the same seeded rows and network
weights, every step of the approximate batch pass: the codes, the SplitMix64
anchor draw, the leader labels, the nearest-anchor keys, the stable order of
every relation, the tile statistics and the four tile-pair bounds.  The
library exposes only the pass's result, so the prediction is checked through
it:

  * tiles_kept lies between the number of tile pairs the reference keeps by
    more than TOL and that number plus the pairs within TOL of theta - eps;
  * every returned pair is a pair of the exact join (FP64 oracle);
  * every exact pair whose tile pair (in the reference's order) is kept by
    more than TOL is returned, and none whose tile pair is pruned by more
    than TOL is.

A wrong label, key, order, statistic or bound moves pairs across tiles or
tiles across the cut, and one of these fails.  TOL = 0.02 covers the GPU's
FP32 arithmetic, its BF16 copies of the codes and hidden layer and its
rounding of the normalised rows against the FP64 reference (the reference
applies the library's 0.02 margin on the tile-to-rows dot itself).

The network is a fixed random linear projection written as a two-layer ReLU
network (W1 = [P, -P], W2 = [Q; -Q], zero biases: z = x P Q), so that the
codes keep the clusters apart with margins the test asserts on the reference
side: anchor pair cosines away from the leader threshold and every row's
nearest anchor well ahead of any anchor with another label.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import prefilter as P
from paper_2312_01476_amd import datagen as G

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

E = None
TOL = 0.02
EPS = 0.05


def setup_module(module):
    global E
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_01476_amd import ejoin
    E = ejoin


def _projection_net(D, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    Pm = rng.standard_normal((D, 128)) / np.sqrt(D)
    Q = rng.standard_normal((128, 64)) / np.sqrt(128)
    return {"W1": np.concatenate([Pm, -Pm], axis=1).astype(np.float32),
            "b1": np.zeros(256, np.float32),
            "W2": np.concatenate([Q, -Q], axis=0).astype(np.float32),
            "b2": np.zeros(64, np.float32)}


def _flat(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"]]).astype(np.float32)


def _host_jobs(D, seed=3):
    cent = G.centres(D, 8, seed)
    shapes = [(3000, 1500), (900, 2500), (1200, 1200), (257, 700), (0, 300), (2000, 129)]
    thetas = [0.80, 0.85, 0.75, 0.90, 0.8, 0.70]
    host = []
    for i, ((nr, ns), th) in enumerate(zip(shapes, thetas)):
        R = G.clustered_points(cent, nr, 0.2, seed * 100 + 2 * i)[0] if nr else \
            np.zeros((0, D), np.float32)
        S = G.clustered_points(cent, ns, 0.2, seed * 100 + 2 * i + 1)[0]
        host.append((R, S, th, False))
    X = G.clustered_points(cent, 1500, 0.2, seed * 100 + 77)[0]
    host.append((X, X, 0.82, True))
    return host


def _margins(pl):
    A, lab = pl["A"], pl["labels"]
    Gm = A @ A.T
    iu = np.triu_indices(A.shape[0], 1)
    anchor = np.abs(Gm[iu] - P.ANCHOR_TAU).min()
    label = 1.0
    for u in pl["U"]:
        dd = u @ A.T
        lb = lab[np.argmax(dd, 1)]
        other = np.where(lab[None, :] != lb[:, None], dd, -9.0).max(1)
        label = min(label, float((dd.max(1) - other).min()))
    return anchor, label


@pytest.mark.parametrize("D,tile", [(96, 3), (640, 22), (640, 19)])
def test_kept_tiles_and_pairs_follow_the_reference(D, tile):
    host = _host_jobs(D)
    params = _projection_net(D, 9)
    pl = P.plan(host, params, D, EPS)
    anchor_margin, label_margin = _margins(pl)
    assert anchor_margin > 0.05 and label_margin > 0.2, (anchor_margin, label_margin)

    net = E.Mlp(D, torch.from_numpy(_flat(params)))
    jobs = []
    for R, S, th, alias in host:
        Rd = torch.from_numpy(R).cuda()
        jobs.append((Rd, Rd if alias else torch.from_numpy(S).cuda(), th))
    caps = [max(1, R.shape[0] * S.shape[0]) for R, S, _, _ in host]
    res, st = E.batch(jobs, prec="bf16", tile=tile, prefilter=net, eps=EPS, capacities=caps)
    assert st["tile"] == tile

    sure = amb = 0
    checked_in = checked_out = 0
    for q, ((R, S, th, _), J, got) in enumerate(zip(host, pl["jobs"], res)):
        got = set(zip(got.r.cpu().tolist(), got.s.cpu().tolist()))
        if R.shape[0] == 0:
            assert not got
            continue
        cut = th - EPS
        keep_sure = J["bound"] >= cut + TOL
        prune_sure = J["bound"] < cut - TOL
        sure += int(keep_sure.sum())
        amb += int((~keep_sure & ~prune_sure).sum())
        ri, si, _, _ = O.threshold(R, S, th)
        exact = set(zip(ri.tolist(), si.tolist()))
        assert got <= exact, f"job {q}: pairs outside the exact join"
        pos_r = np.empty(R.shape[0], np.int64)
        pos_r[J["order_r"]] = np.arange(R.shape[0])
        pos_s = np.empty(S.shape[0], np.int64)
        pos_s[J["order_s"]] = np.arange(S.shape[0])
        tr, ts = pos_r[ri] // P.TILE, pos_s[si] // P.TILE
        must = keep_sure[tr, ts]
        never = prune_sure[tr, ts]
        for i, j, m, nv in zip(ri.tolist(), si.tolist(), must, never):
            if m:
                assert (i, j) in got, f"job {q}: pair {(i, j)} of a kept tile pair missing"
                checked_in += 1
            elif nv:
                assert (i, j) not in got, f"job {q}: pair {(i, j)} of a pruned tile pair returned"
                checked_out += 1
    assert sure <= st["tiles_kept"] <= sure + amb, (sure, amb, st["tiles_kept"])
    assert amb <= st["tiles_total"] // 50
    assert st["tiles_kept"] < st["tiles_total"]   # the prefilter prunes here
    assert checked_in > 1000
