"""FP64 reference of the learned prefilter (test infrastructure only).

The prefilter is not part of the paper's method: the paper names learned
indexes only among related work and index pre-filtering as a way to avoid
scanning all pairs.  What is computed here is the approximate mode built on
top of the exact tensor join:

  * a two-layer MLP f maps a normalised embedding row x (d values) to a
    64-d code: h = ReLU(x W1 + b1) (256 values), z = h W2 + b2,
    u = z / ||z||;
  * the predicted similarity of a pair is p = u_r . u_s;
  * it is trained on (pair, sim64) records drawn from the exact join with
    the loss  mean[(p - t)^2] + lambda * mean[max(0, t - p)^2 * 1{t >= theta_lo}]
    (the second term charges under-predicted true matches, which protects
    recall) and Adam (beta 0.9 / 0.999, eps 1e-8) on FP32 master weights
    whose BF16 copies feed the forward pass;
  * inference codes every row, orders the rows of each relation by a
    locality-sensitive key of u, and bounds the predicted similarity of all
    pairs of a tile pair (T, U) by
        c_T . c_U + rho_T ||c_U|| + rho_U ||c_T|| + rho_T rho_U
    with c the mean code of a tile and rho the largest distance of a code of
    the tile from c; tile pairs whose bound is below theta - eps are skipped.

Every function follows those definitions step by step in float64 with
numpy; nothing is blocked, fused or reordered.  Parity pins live in
tests/test_oracle_mlp.py (finite differences, Adam closed forms, the
scale invariance of the normalisation, brute-force tile bounds).

This module is test infrastructure: only the tests, the smoke check and the
benchmark's CPU baseline may import it.
"""
from __future__ import annotations

import numpy as np

HIDDEN = 256
OUT = 64


# ---------------------------------------------------------------------------
# BF16 copies of the weights
# ---------------------------------------------------------------------------

def bf16_round(a) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned
    as float64.  Written from the format's definition: keep the top 16 bits
    of the IEEE single pattern after adding half an ulp of the kept part
    (0x7FFF plus the lowest kept bit)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# forward / loss / backward
# ---------------------------------------------------------------------------

def forward_weights(params: dict, round_bf16: bool = True) -> dict:
    """The weights the forward pass uses: BF16 copies of the FP32 masters
    (or the masters themselves, for finite-difference checks)."""
    if not round_bf16:
        return {k: np.asarray(v, np.float64) for k, v in params.items()}
    return {k: bf16_round(v) for k, v in params.items()}


def forward(W: dict, X, round_h: bool = False) -> dict:
    """Codes of the rows of X (n x d, float64 values).  Returns the
    intermediates a1 = x W1 + b1, h = ReLU(a1), z = h W2 + b2, the norm of z
    and u = z / ||z||.  round_h stores h in BF16 before the second layer
    (the inference form, whose hidden layer is kept in BF16)."""
    X = np.asarray(X, np.float64)
    a1 = X @ W["W1"] + W["b1"]
    h = np.maximum(a1, 0.0)
    if round_h:
        h = bf16_round(h)
    z = h @ W["W2"] + W["b2"]
    nz = np.sqrt(np.sum(z * z, axis=1))
    u = z / nz[:, None]
    return {"X": X, "a1": a1, "h": h, "z": z, "nz": nz, "u": u}


def pair_loss(p, t, lam: float, theta_lo: float):
    """Loss of a batch of predicted similarities p against targets t, and
    its derivative with respect to every p."""
    p = np.asarray(p, np.float64)
    t = np.asarray(t, np.float64)
    B = p.shape[0]
    under = np.maximum(0.0, t - p) * (t >= theta_lo)
    loss = np.mean((p - t) ** 2) + lam * np.mean(under ** 2)
    dp = (2.0 / B) * (p - t) - lam * (2.0 / B) * under
    return loss, dp


def loss_and_grads(params: dict, X, pr, ps, t, lam: float = 4.0, theta_lo: float = 0.7,
                   round_bf16: bool = True):
    """Loss of the pair batch (rows pr[i], ps[i] of X, targets t[i]) and the
    gradients with respect to the master weights.  The BF16 rounding of the
    forward weights is passed straight through (the gradient of a copy is
    the gradient of its master)."""
    W = forward_weights(params, round_bf16)
    pr = np.asarray(pr, np.int64)
    ps = np.asarray(ps, np.int64)
    X = np.asarray(X, np.float64)
    # both rows of every pair go through the network as their own slot
    rows = np.concatenate([X[pr], X[ps]])
    f = forward(W, rows)
    B = pr.shape[0]
    ur, us = f["u"][:B], f["u"][B:]
    p = np.sum(ur * us, axis=1)
    loss, dp = pair_loss(p, t, lam, theta_lo)
    # p = u_r . u_s
    du = np.concatenate([dp[:, None] * us, dp[:, None] * ur])
    # u = z / ||z||:  dz = (du - u (u . du)) / ||z||
    u = f["u"]
    dz = (du - u * np.sum(u * du, axis=1, keepdims=True)) / f["nz"][:, None]
    # z = h W2 + b2
    gW2 = f["h"].T @ dz
    gb2 = dz.sum(axis=0)
    dh = dz @ W["W2"].T
    # h = ReLU(a1)
    da1 = dh * (f["a1"] > 0.0)
    # a1 = x W1 + b1
    gW1 = f["X"].T @ da1
    gb1 = da1.sum(axis=0)
    return loss, {"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2}, p


# ---------------------------------------------------------------------------
# Adam
# ---------------------------------------------------------------------------

def adam_step(params: dict, grads: dict, m: dict, v: dict, step: int, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step is 1 for the first update).  Returns new
    (params, m, v); inputs are not modified."""
    P, M, V = {}, {}, {}
    for k in params:
        g = np.asarray(grads[k], np.float64)
        M[k] = beta1 * np.asarray(m[k], np.float64) + (1.0 - beta1) * g
        V[k] = beta2 * np.asarray(v[k], np.float64) + (1.0 - beta2) * g * g
        mhat = M[k] / (1.0 - beta1 ** step)
        vhat = V[k] / (1.0 - beta2 ** step)
        P[k] = np.asarray(params[k], np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return P, M, V


# ---------------------------------------------------------------------------
# inference side: ordering key and tile bounds
# ---------------------------------------------------------------------------

def leader_labels(A, tau: float) -> np.ndarray:
    """Leader clustering of anchor codes A (K x 64) in order: an anchor joins
    the first earlier leader whose code has cosine >= tau with it, else it
    becomes a leader; returns each anchor's leader rank."""
    A = np.asarray(A, np.float64)
    leaders = []
    lab = np.zeros(A.shape[0], np.int64)
    for k in range(A.shape[0]):
        for rank, j in enumerate(leaders):
            if A[k] @ A[j] >= tau:
                lab[k] = rank
                break
        else:
            lab[k] = len(leaders)
            leaders.append(k)
    return lab


def anchor_key(U, A, labels) -> np.ndarray:
    """Ordering key of every code: the label of its nearest anchor (largest
    dot product, ties to the lower anchor index)."""
    d = np.asarray(U, np.float64) @ np.asarray(A, np.float64).T
    return np.asarray(labels)[np.argmax(d, axis=1)]


def order_by_key(keys) -> np.ndarray:
    """Stable ascending order of the keys (equal keys keep row order)."""
    return np.argsort(np.asarray(keys, np.int64), kind="stable")


def tile_stats(U, tile: int):
    """Centroid and radius of every block of `tile` consecutive rows of U."""
    U = np.asarray(U, np.float64)
    n = U.shape[0]
    nt = (n + tile - 1) // tile
    C = np.zeros((nt, U.shape[1]))
    rho = np.zeros(nt)
    for i in range(nt):
        blk = U[i * tile:(i + 1) * tile]
        C[i] = blk.mean(axis=0)
        rho[i] = np.sqrt(((blk - C[i]) ** 2).sum(axis=1)).max()
    return C, rho


def tile_pair_bound(cT, rT, cU, rU) -> float:
    """Upper bound of u . v over u within rT of cT and v within rU of cU."""
    cT = np.asarray(cT, np.float64)
    cU = np.asarray(cU, np.float64)
    return float(cT @ cU + rT * np.linalg.norm(cU) + rU * np.linalg.norm(cT) + rT * rU)


def tile_angles(U, tile: int):
    """Angular radius of every block of `tile` consecutive unit codes: the
    largest angle between a code of the block and the direction of the
    block's centroid (nan for a zero centroid)."""
    C, _ = tile_stats(U, tile)
    U = np.asarray(U, np.float64)
    out = np.zeros(C.shape[0])
    for i in range(C.shape[0]):
        n = np.linalg.norm(C[i])
        if n == 0.0:
            out[i] = np.nan
            continue
        cos = U[i * tile:(i + 1) * tile] @ (C[i] / n)
        out[i] = np.arccos(np.clip(cos.min(), -1.0, 1.0))
    return out


def tile_pair_bound_angular(cT, aT, cU, aU) -> float:
    """Upper bound of u . v for unit u within angle aT of the direction of cT
    and unit v within angle aU of the direction of cU: the angle between u
    and v is at least (angle between the directions) - aT - aU."""
    cT = np.asarray(cT, np.float64)
    cU = np.asarray(cU, np.float64)
    cphi = cT @ cU / (np.linalg.norm(cT) * np.linalg.norm(cU))
    gap = np.arccos(np.clip(cphi, -1.0, 1.0)) - aT - aU
    return float(np.cos(gap)) if gap > 0.0 else 1.0



def tile_rows_bound(dT, aT, V, slack: float = 0.0) -> float:
    """Upper bound of u . v over unit u within angle aT of the unit direction
    dT and every row v of V (unit codes): the angle between u and v is at
    least angle(dT, v) - aT, so u . v <= cos(max(0, acos(max_v dT . v) - aT)).
    `slack` widens the largest dot before the arccos (the library adds a
    margin there for its BF16 copies of the codes)."""
    dT = np.asarray(dT, np.float64)
    m = float(np.max(np.asarray(V, np.float64) @ dT)) + slack
    gap = np.arccos(np.clip(m, -1.0, 1.0)) - aT
    return float(np.cos(gap)) if gap > 0.0 else 1.0
