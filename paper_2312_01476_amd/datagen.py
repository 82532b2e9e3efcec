"""Seeded synthetic embedding generators shared by the tests, the bench and the
oracle checks.

This module holds only input generation: it contains none of the join's
arithmetic (no similarity, no threshold, no selection).  The paper evaluates on
FastText embeddings of Wikipedia strings (Section VI.A); that model and dataset
are not available, so clustered synthetic embeddings stand in for them:

* cluster centre  c = g / ||g||,  g ~ N(0, I_d)
* point           x = normalise(c + (sigma / sqrt(d)) * z),  z ~ N(0, I_d)

so that the noise vector has norm ~sigma.  R and S draw their points from the
same set of centres, each point picking its cluster uniformly at random; the
labels are returned so that tests can form the closed-form match count
sum_c |R_c| |S_c| when the within-cluster similarity clears the threshold and
the across-cluster similarity does not.

Rows are written into a row-major float32 buffer of leading dimension
``ld >= d``; columns ``d..ld-1`` are filled with ``pad_value`` (zero by default;
tests use NaN there to prove that nothing reads past ``d``).

Two back ends produce the same recipe: numpy ``Generator(PCG64(seed))`` on the
host (used for everything the oracle checks in full) and a torch generator on a
device for the large bench workloads (the oracle then checks copied-back
sub-blocks).  They draw different random streams for the same seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# host (numpy) generators
# --------------------------------------------------------------------------

def centres(d: int, n_clusters: int, seed: int) -> np.ndarray:
    """Unit-norm cluster centres, float64 (n_clusters, d)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal((n_clusters, d))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def _to_buffer(x: np.ndarray, ld: int | None, pad_value: float) -> np.ndarray:
    n, d = x.shape
    ld = d if ld is None else int(ld)
    if ld < d:
        raise ValueError("ld < d")
    out = np.empty((n, ld), dtype=np.float32)
    out[:, :d] = x.astype(np.float32)
    if ld > d:
        out[:, d:] = pad_value
    return out


def clustered_points(cent: np.ndarray, n: int, sigma: float, seed: int,
                     ld: int | None = None, pad_value: float = 0.0,
                     chunk: int = 1 << 16):
    """n points around the given centres.

    Returns (X float32 (n, ld), labels int64 (n,)).
    """
    k, d = cent.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    labels = rng.integers(0, k, size=n)
    ld_ = d if ld is None else int(ld)
    out = np.empty((n, ld_), dtype=np.float32)
    scale = sigma / math.sqrt(d)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        z = rng.standard_normal((hi - lo, d))
        x = cent[labels[lo:hi]] + scale * z
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[lo:hi] = _to_buffer(x, ld_, pad_value)
    return out, labels


def word_tuples(n_tuples: int, vocab: np.ndarray, vocab_labels: np.ndarray,
                seed: int, ld: int | None = None, pad_value: float = 0.0):
    """Tuples that each draw one word of the vocabulary uniformly, with
    replacement (so repeated words give bitwise-identical rows).

    ``vocab`` is float32 (n_words, d).  Returns (X float32 (n, ld), word ids,
    cluster labels)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ids = rng.integers(0, vocab.shape[0], size=n_tuples)
    out = _to_buffer(vocab[ids, :], ld, pad_value)
    return out, ids, vocab_labels[ids]


def uniform_sphere(n: int, d: int, seed: int, ld: int | None = None,
                   pad_value: float = 0.0) -> np.ndarray:
    """Unclustered unit vectors (no structure), float32 (n, ld)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal((n, d))
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    return _to_buffer(x, ld, pad_value)


def gaussian_raw(n: int, d: int, seed: int, scale: float = 1.0,
                 ld: int | None = None, pad_value: float = 0.0) -> np.ndarray:
    """Unnormalised Gaussian rows (the join must normalise them itself)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = scale * rng.standard_normal((n, d))
    return _to_buffer(x, ld, pad_value)


# --------------------------------------------------------------------------
# device (torch) generator for the large workloads
# --------------------------------------------------------------------------

def clustered_points_torch(n: int, d: int, n_clusters: int, sigma: float,
                           seed: int, centre_seed: int, ld: int | None = None,
                           device: str = "cuda", chunk: int = 1 << 18,
                           pad_value: float = 0.0):
    """Device-side counterpart of :func:`centres` + :func:`clustered_points`.

    Same recipe, torch's generator (so a different stream than numpy for the
    same seed).  Returns (X float32 tensor (n, ld) on ``device``, labels int64
    tensor (n,) on ``device``)."""
    import torch

    ld_ = d if ld is None else int(ld)
    gc = torch.Generator(device=device)
    gc.manual_seed(int(centre_seed))
    c = torch.randn((n_clusters, d), generator=gc, device=device,
                    dtype=torch.float64)
    c /= torch.linalg.vector_norm(c, dim=1, keepdim=True)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    labels = torch.randint(0, n_clusters, (n,), generator=g, device=device)
    out = torch.empty((n, ld_), dtype=torch.float32, device=device)
    if ld_ > d:
        out[:, d:] = pad_value
    scale = sigma / math.sqrt(d)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        z = torch.randn((hi - lo, d), generator=g, device=device,
                        dtype=torch.float32)
        x = c[labels[lo:hi]].to(torch.float32) + scale * z
        x /= torch.linalg.vector_norm(x, dim=1, keepdim=True)
        out[lo:hi, :d] = x
    return out, labels


# --------------------------------------------------------------------------
# named workloads (sizes and distributions of the paper-derived configs)
# --------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    n_r: int
    n_s: int
    d: int
    ld: int
    n_clusters: int
    sigma: float
    theta: float | None = None
    k: int | None = None
    prec: str = "fp32"
    band: float | None = None
    vocab: int | None = None
    seeds: tuple = (11, 12, 13)        # (centres, R, S)
    notes: str = ""
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    # 1k x 1k word tuples over a 5k-word vocabulary of 300-d vectors from 50
    # clusters (sigma 0.3); every pair with cosine >= 0.8.
    "words_1k": Workload("words_1k", 1000, 1000, 300, 320, 50, 0.3, theta=0.8,
                         vocab=5000, seeds=(101, 102, 103),
                         notes="1k x 1k word tuples, 300-d, fp32, theta 0.8"),
    # 100k x 100k, 300-d (row stride 320), 200 clusters sigma 0.25, theta 0.9.
    "fp32_100k": Workload("fp32_100k", 100_000, 100_000, 300, 320, 200, 0.25,
                          theta=0.9, seeds=(201, 202, 203),
                          notes="100k x 100k, 300-d (ld 320), fp32, theta 0.9"),
    # 1M x 1M, 384-d, 1000 clusters sigma 0.2, theta 0.85, bf16 + fp64 band 1e-2.
    "bf16_1m": Workload("bf16_1m", 1_000_000, 1_000_000, 384, 384, 1000, 0.2,
                        theta=0.85, prec="bf16", band=1e-2, seeds=(301, 302, 303),
                        notes="1M x 1M, 384-d, bf16 + fp64 band 1e-2, theta 0.85"),
    # 2M x 200k, 768-d, 2000 clusters sigma 0.3, top-10, fp8 e4m3 per-row scale.
    "fp8_topk_2m": Workload("fp8_topk_2m", 2_000_000, 200_000, 768, 768, 2000,
                            0.3, k=10, prec="fp8", seeds=(401, 402, 403),
                            notes="2M x 200k, 768-d, top-10, fp8 e4m3"),
    # 64 joins in one batch: |R| log-uniform 1k-500k, |S| log-uniform 1k-100k,
    # theta uniform in [0.75, 0.95], 768-d, 1000 shared clusters sigma 0.3
    # (job shapes from batch_jobs, seed 501; per-job R/S seeds from there).
    "batch64_fp32": Workload("batch64_fp32", 0, 0, 768, 768, 1000, 0.3, prec="fp32",
                             seeds=(500, 0, 0), extra={"batch": 64, "job_seed": 501},
                             notes="64 uneven joins, 768-d, fp32 + fp64 band, one batch pass"),
    "batch64_bf16": Workload("batch64_bf16", 0, 0, 768, 768, 1000, 0.3, prec="bf16",
                             seeds=(500, 0, 0), extra={"batch": 64, "job_seed": 501},
                             notes="64 uneven joins, 768-d, bf16 + fp64 band, one batch pass"),
    # the same 64 joins through the learned prefilter (approximate mode):
    # network 768-256-64 trained on pairs drawn from the exact batch output
    "batch64_learned": Workload("batch64_learned", 0, 0, 768, 768, 1000, 0.3, prec="bf16",
                                seeds=(500, 0, 0),
                                extra={"batch": 64, "job_seed": 501, "prefilter": True,
                                       "mlp_seed": 601, "train_steps": 300,
                                       "train_batch": 4096, "eps": 0.05},
                                notes="64 uneven joins, 768-d, learned prefilter (approximate)"),
    # the same 64 joins with exact tile pruning (certified bounds in the
    # original space; the result is the exact join)
    "batch64_exact": Workload("batch64_exact", 0, 0, 768, 768, 1000, 0.3, prec="bf16",
                              seeds=(500, 0, 0),
                              extra={"batch": 64, "job_seed": 501, "exact_prune": True},
                              notes="64 uneven joins, 768-d, bf16, exact tile pruning"),
    # the same job shapes and thresholds over 100 clusters (about ten times
    # more rows per cluster in every relation, so that 128-row tiles hold
    # one cluster): where tile pruning can pay; a different data
    # distribution from the 64-job workload above
    "batch64_exact_c100": Workload("batch64_exact_c100", 0, 0, 768, 768, 100, 0.3,
                                   prec="bf16", seeds=(500, 0, 0),
                                   extra={"batch": 64, "job_seed": 501, "exact_prune": True},
                                   notes="64 uneven joins, 768-d, 100 clusters, exact pruning"),
    "batch64_learned_c100": Workload("batch64_learned_c100", 0, 0, 768, 768, 100, 0.3,
                                     prec="bf16", seeds=(500, 0, 0),
                                     extra={"batch": 64, "job_seed": 501, "prefilter": True,
                                            "mlp_seed": 601, "train_steps": 300,
                                            "train_batch": 4096, "eps": 0.05},
                                     notes="64 uneven joins, 768-d, 100 clusters, learned "
                                           "prefilter (approximate)"),
    # the scan side of the scan-versus-probe study: 10k query tuples joined
    # with 1M data tuples after a relational pre-filter on the data side
    # (selectivity 1-100% of an attribute drawn uniformly in [0, 1)), range
    # predicate sim >= 0.9 and top-1 / top-32, 300-d (ld 320), fp32; 10k
    # clusters (sigma 0.25), so a query has ~100 same-cluster rows in all of S
    "sel_10k_1m": Workload("sel_10k_1m", 10_000, 1_000_000, 300, 320, 10_000, 0.25,
                           theta=0.9, seeds=(701, 702, 703), extra={"attr_seed": 704},
                           notes="10k x 1M, 300-d, fp32, pre-filter on S at 1-100%"),
}


def attribute_column_torch(n: int, seed: int, device: str = "cuda"):
    """A relational attribute drawn uniformly in [0, 1) (float32, on the
    device): a range predicate a < s on it keeps a fraction s of the rows."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.rand((n,), generator=g, device=device, dtype=torch.float32)


def micro_sweep_side(ops: int, dim: int) -> int:
    """Relation size for the paper's per-element micro sweep (Section VI.D):
    |R| = |S| = sqrt(#FP32-Ops / dim), where #FP32-Ops = |R| |S| dim."""
    return int(round(math.sqrt(ops / dim)))


def batch_jobs(n_jobs: int = 64, d: int = 768, seed: int = 501,
               r_range=(1_000, 500_000), s_range=(1_000, 100_000),
               theta_range=(0.75, 0.95)):
    """Job shapes of the batched workload: |R| and |S| log-uniform, theta
    uniform.  Returns a list of dicts (n_r, n_s, theta, seed_r, seed_s)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    jobs = []
    for j in range(n_jobs):
        nr = int(round(math.exp(rng.uniform(math.log(r_range[0]), math.log(r_range[1])))))
        ns = int(round(math.exp(rng.uniform(math.log(s_range[0]), math.log(s_range[1])))))
        th = float(rng.uniform(*theta_range))
        jobs.append(dict(n_r=nr, n_s=ns, theta=th, seed_r=seed * 1000 + 2 * j,
                         seed_s=seed * 1000 + 2 * j + 1))
    return jobs


def make_host(w: Workload, n_r: int | None = None, n_s: int | None = None,
              pad_value: float = 0.0):
    """Generate a workload (or a leading sub-block of it) on the host.

    Returns (R, S, labels_R, labels_S) with R, S float32 (n, ld)."""
    n_r = w.n_r if n_r is None else n_r
    n_s = w.n_s if n_s is None else n_s
    cs, rs, ss = w.seeds
    if w.vocab is not None:
        cent = centres(w.d, w.n_clusters, cs)
        vocab, vlab = clustered_points(cent, w.vocab, w.sigma, cs + 7)
        R, _, lr = word_tuples(n_r, vocab, vlab, rs, ld=w.ld, pad_value=pad_value)
        S, _, ls = word_tuples(n_s, vocab, vlab, ss, ld=w.ld, pad_value=pad_value)
        return R, S, lr, ls
    cent = centres(w.d, w.n_clusters, cs)
    R, lr = clustered_points(cent, n_r, w.sigma, rs, ld=w.ld, pad_value=pad_value)
    S, ls = clustered_points(cent, n_s, w.sigma, ss, ld=w.ld, pad_value=pad_value)
    return R, S, lr, ls


# --------------------------------------------------------------------------
# seeded initial state of the prefilter network (random draws only)
# --------------------------------------------------------------------------

def mlp_init(dim: int, seed: int, hidden: int = 256, out: int = 64, bias_scale: float = 0.0):
    """He-initialised flat parameters (W1 dim x hidden, b1, W2 hidden x out,
    b2; biases N(0, bias_scale^2)), float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.standard_normal((dim, hidden)) * math.sqrt(2.0 / dim)
    b1 = rng.standard_normal(hidden) * bias_scale
    W2 = rng.standard_normal((hidden, out)) * math.sqrt(2.0 / hidden)
    b2 = rng.standard_normal(out) * bias_scale
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2]).astype(np.float32)
