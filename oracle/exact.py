"""Exact-rational brute force for tiny inputs (test infrastructure only).

Decides the join predicate of the paper's cosine similarity (Section III.A)
over the Cartesian product (Section III.C) with no rounding at all: the float32
inputs and the float64 threshold are converted to exact rationals and the
comparison  cos(r, s) >= theta  is decided by signs and squares,

    theta >= 0:  dot >= 0  and  dot^2 >= theta^2 * |r|^2 * |s|^2
    theta <  0:  dot >= 0  or   dot^2 <= theta^2 * |r|^2 * |s|^2

with cos := 0 for a zero row (so such a pair matches iff theta <= 0).  It is
independent of the FP64 oracle (no shared code, different arithmetic) and pins
it: the two must agree on every pair except those the FP64 oracle reports as
ties (|sim64 - theta| below 1e-12).

Top-k order uses the exact monotone key  sign(dot) * dot^2 / (|r|^2 |s|^2),
ties broken by the smaller S index.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _rows(X, d):
    X = np.asarray(X, dtype=np.float32)
    return [[Fraction(float(v)) for v in row[:d]] for row in X]


def _dot(a, b):
    return sum((x * y for x, y in zip(a, b)), Fraction(0))


def matches(r, s, theta: float) -> bool:
    """Exact decision of cos(r, s) >= theta for rational vectors r, s."""
    th = Fraction(float(theta))
    nr = _dot(r, r)
    ns = _dot(s, s)
    if nr == 0 or ns == 0:
        return 0 >= th
    dot = _dot(r, s)
    lhs = dot * dot
    rhs = th * th * nr * ns
    if th >= 0:
        return dot >= 0 and lhs >= rhs
    return dot >= 0 or lhs <= rhs


def threshold(R, S, theta: float, d: int | None = None):
    """Set of (i, j) with cos(R_i, S_j) >= theta, decided exactly."""
    d = np.asarray(R).shape[1] if d is None else d
    Rq = _rows(R, d)
    Sq = _rows(S, d)
    return {(i, j) for i, r in enumerate(Rq) for j, s in enumerate(Sq)
            if matches(r, s, theta)}


def sim_key(r, s) -> Fraction:
    """Exact key that orders pairs like cos(r, s): sign(dot) dot^2/(|r|^2|s|^2)."""
    nr = _dot(r, r)
    ns = _dot(s, s)
    if nr == 0 or ns == 0:
        return Fraction(0)
    dot = _dot(r, s)
    key = dot * dot / (nr * ns)
    return key if dot >= 0 else -key


def topk(R, S, k: int, d: int | None = None):
    """Per R row, the first min(k, |S|) S indices by (cos desc, index asc);
    padded with -1."""
    d = np.asarray(R).shape[1] if d is None else d
    Rq = _rows(R, d)
    Sq = _rows(S, d)
    out = []
    for r in Rq:
        keys = [(-sim_key(r, s), j) for j, s in enumerate(Sq)]
        keys.sort()
        row = [j for _, j in keys[:k]]
        row += [-1] * (k - len(row))
        out.append(row)
    return np.array(out, dtype=np.int64).reshape(len(Rq), k)


def topk_range(R, S, k: int, theta: float, d: int | None = None):
    """The range predicate combined with the top-k condition: per R row the
    first min(k, m) of the m S indices with cos >= theta, by (cos desc, index
    asc), decided exactly; padded with -1."""
    d = np.asarray(R).shape[1] if d is None else d
    Rq = _rows(R, d)
    Sq = _rows(S, d)
    out = []
    for r in Rq:
        keys = [(-sim_key(r, s), j) for j, s in enumerate(Sq) if matches(r, s, theta)]
        keys.sort()
        row = [j for _, j in keys[:k]]
        row += [-1] * (k - len(row))
        out.append(row)
    return np.array(out, dtype=np.int64).reshape(len(Rq), k)
