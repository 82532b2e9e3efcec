"""FP64 reference of the learned prefilter's inference side (test
infrastructure only; the prefilter is not part of the paper's method).

Given a batch of threshold jobs and the network's weights, this predicts
which 128 x 128 tile pairs the approximate batch pass contracts, following
the steps of the mode in order:

  1. every relation's rows are prepared as the BF16 join prepares operands
     (L2-normalised, rounded to bfloat16) and coded by the network in its
     inference form (BF16 weights, hidden layer kept in BF16), u = z / ||z||;
  2. the relations are laid out one after another in the order the batch
     planner takes the jobs (most 128 x 128 tiles first, ties in caller
     order; R then S, S omitted for a self-join, empty jobs omitted);
  3. K = min(2048, real rows) anchor rows are drawn with SplitMix64 (seed
     0x5EED): draw q picks real row floor(x_q * n_real / 2^64) of the
     concatenated relations;
  4. the anchors' codes are grouped by leader clustering at cosine 0.6 and
     every row takes the label of its nearest anchor as its key;
  5. every relation is put in stable key order and cut into tiles of 128
     consecutive rows;
  6. each tile pair (T, U) of a job gets the smallest of four upper bounds
     of u_r . u_s over its rows: the centroid/radius bound, the angular
     bound, and the tile-to-rows bound from each side (with the library's
     margin on the largest dot); it is kept when that bound reaches
     theta - eps.

Every step calls the plain functions of oracle/mlp.py; the bounds are pinned
against brute force in tests/test_oracle_mlp.py and the generator against
its published reference outputs.

This module is test infrastructure: only the tests, the smoke check and the
benchmark's CPU baseline may import it.
"""
from __future__ import annotations

import numpy as np

from . import mlp as M

TILE = 128
N_ANCHORS = 2048
ANCHOR_TAU = 0.6
ANCHOR_SEED = 0x5EED
M_SLACK = 0.02          # the library's margin on the tile-to-rows dot (BF16 codes)

_M64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 (Steele, Lea and Flood, 2014): a Weyl sequence with
    increment 0x9E3779B97F4A7C15 passed through a MurmurHash3-style
    finaliser (shifts 30, 27, 31 with multipliers 0xBF58476D1CE4E5B9 and
    0x94D049BB133111EB)."""

    def __init__(self, seed: int):
        self.x = seed & _M64

    def next(self) -> int:
        self.x = (self.x + 0x9E3779B97F4A7C15) & _M64
        z = self.x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        return z ^ (z >> 31)

    def below(self, n: int) -> int:
        """A draw in [0, n): the high 64 bits of next() * n."""
        return (self.next() * n) >> 64


def prepared_bf16(X, d: int) -> np.ndarray:
    """Rows of X (first d columns) L2-normalised and rounded to bfloat16
    (float64 values); zero rows stay zero."""
    X = np.asarray(X, np.float64)[:, :d]
    n = np.sqrt(np.sum(X * X, axis=1))
    Y = np.where(n[:, None] > 0, X / np.where(n > 0, n, 1.0)[:, None], 0.0)
    return M.bf16_round(Y.astype(np.float32))


def codes(params: dict, X, d: int) -> np.ndarray:
    """Unit codes of the rows of X in the network's inference form."""
    W = M.forward_weights(params, round_bf16=True)
    return M.forward(W, prepared_bf16(X, d), round_h=True)["u"]


def job_order(shapes) -> list:
    """Order in which the batch planner takes jobs: most 128 x 128 tiles
    first, ties in caller order.  shapes: list of (|R|, |S|)."""
    tiles = [-(-nr // TILE) * -(-ns // TILE) for nr, ns in shapes]
    return sorted(range(len(shapes)), key=lambda i: -tiles[i])


def plan(jobs, params: dict, d: int, eps: float, tau: float = ANCHOR_TAU,
         n_anchors: int = N_ANCHORS, seed: int = ANCHOR_SEED, m_slack: float = M_SLACK):
    """Predict the prefilter's decisions for a batch.

    jobs: list of (R, S, theta, self_join) with R, S float32 arrays (rows x
    ld); self_join means S is R itself.  Returns a dict with, per job (in
    caller order), 'order_r' / 'order_s' (local row at every ordered
    position), 'bound' (tiles_m x tiles_n, float64) and 'keep'
    (bound >= theta - eps); and the intermediates 'anchors' (segment,
    local row), 'A' (anchor codes), 'labels', and per segment 'keys' and
    'U' (codes in input row order)."""
    shapes = [(R.shape[0], S.shape[0]) for R, S, _, _ in jobs]
    segs = []          # (job, side, X)
    for q in job_order(shapes):
        R, S, _, alias = jobs[q]
        if R.shape[0] == 0 or S.shape[0] == 0:
            continue
        segs.append((q, "r", R))
        if not alias:
            segs.append((q, "s", S))
    U = [codes(params, X, d) for _, _, X in segs]
    real = sum(X.shape[0] for _, _, X in segs)
    K = min(n_anchors, real)
    rng = SplitMix64(seed)
    anchors = []
    for _ in range(K):
        r = rng.below(real)
        i = 0
        while r >= segs[i][2].shape[0]:
            r -= segs[i][2].shape[0]
            i += 1
        anchors.append((i, r))
    A = np.array([U[i][r] for i, r in anchors]).reshape(K, -1)
    labels = M.leader_labels(A, tau)
    keys = [M.anchor_key(u, A, labels) for u in U]
    orders = [M.order_by_key(k) for k in keys]
    # tile statistics of every segment in key order
    stats = []
    for u, o in zip(U, orders):
        uo = u[o]
        C, rho = M.tile_stats(uo, TILE)
        alpha = M.tile_angles(uo, TILE)
        stats.append((uo, C, rho, alpha))
    seg_of = {(q, side): i for i, (q, side, _) in enumerate(segs)}
    out = []
    for q, (R, S, theta, alias) in enumerate(jobs):
        nr, ns = shapes[q]
        if nr == 0 or ns == 0:
            out.append({"order_r": np.arange(nr), "order_s": np.arange(ns),
                        "bound": np.zeros((0, 0)), "keep": np.zeros((0, 0), bool)})
            continue
        ir = seg_of[(q, "r")]
        is_ = seg_of[(q, "r")] if alias else seg_of[(q, "s")]
        ur, Cr, rr, ar = stats[ir]
        us, Cs, rs, as_ = stats[is_]
        tm, tn = Cr.shape[0], Cs.shape[0]
        B = np.empty((tm, tn))
        for a in range(tm):
            da = Cr[a] / np.linalg.norm(Cr[a])
            rows_a = ur[a * TILE:(a + 1) * TILE]
            for b in range(tn):
                db = Cs[b] / np.linalg.norm(Cs[b])
                rows_b = us[b * TILE:(b + 1) * TILE]
                B[a, b] = min(M.tile_pair_bound(Cr[a], rr[a], Cs[b], rs[b]),
                              M.tile_pair_bound_angular(Cr[a], ar[a], Cs[b], as_[b]),
                              M.tile_rows_bound(da, ar[a], rows_b, m_slack),
                              M.tile_rows_bound(db, as_[b], rows_a, m_slack))
        out.append({"order_r": orders[ir], "order_s": orders[is_], "bound": B,
                    "keep": B >= theta - eps})
    return {"jobs": out, "anchors": anchors, "A": A, "labels": labels, "keys": keys, "U": U,
            "segs": [(q, side) for q, side, _ in segs]}
