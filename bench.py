#!/usr/bin/env python3
"""Benchmark of the threshold E-join hot path on one MI355X.

One step = one full ``ejoin_threshold`` call through the C ABI over the
workload (prep + matrix-core tiles with the threshold epilogue + FP64 band
rescore + count read-back), inputs already resident in HBM.

Default workload: 100k x 100k tuples, 300-d float32 embeddings (row stride
320), 200 Gaussian clusters (sigma 0.25), theta 0.9, FP32 contraction with the
FP64 band recheck.  The printed JSON line carries the throughput
(Gpairs/s = |R| |S| / step time), the roofline position of the dominant
kernel (the MFMA tile kernel, timed with HIP events on the stream it runs on)
and the FP64 CPU oracle timed on a bounded sample of the same workload.  The
default line also carries, each measured in the same run: the nested-loop
comparator on the same inputs, the 1M x 1M BF16 join (and the plain FP32 join
on its inputs), the selectivity sweep, and the FP8 2M x 200k top-10, the
64-job BF16 batch and that batch's shapes over 100 clusters with exact tile
pruning (these three in child processes, each line as its own run prints it).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {  # MI355X published dense peaks
    "fp32": ("TFLOP/s", 157.3),
    "bf16": ("TFLOP/s", 2500.0),
    "fp8": ("TFLOP/s", 5000.0),
    "hbm": ("GB/s", 8000.0),
}
DTYPE = {"fp32": "f32", "bf16": "bf16", "fp8": "fp8_e4m3"}

# HBM bytes per launch of the dominant kernel from FETCH_SIZE / WRITE_SIZE
# counter runs scaled by a plain copy of known size (the commands and the raw
# figures are in profiles/threshold_fp32_100k_traffic.md and
# profiles/hbm_traffic_bf16_kernels.md); valid for the
# kernel as it was when the counters were taken, keyed by workload and tile
TRAFFIC = {("fp32_100k", "fp32:panel/2wg"): 2673670.375 * 1024 * 2.0 + 600664.40625 * 1024 * 1.0,
           ("bf16_1m", "bf16:panel"): 51713273.375 * 1024 * 2.0 + 11982635.28125 * 1024 * 1.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(w, torch):
    """Inputs on the device.  Host generation (numpy) for sizes the oracle
    checks in full; device generation (torch) for the largest workloads."""
    from paper_2312_01476_amd import datagen as G
    if w.n_r * w.ld <= 50_000_000:
        R, S, lr, ls = G.make_host(w)
        return (torch.from_numpy(R).cuda(), torch.from_numpy(S).cuda(), R, S,
                torch.from_numpy(lr), torch.from_numpy(ls))
    cs, rs, ss = w.seeds
    Rd, lr = G.clustered_points_torch(w.n_r, w.d, w.n_clusters, w.sigma, rs, cs, ld=w.ld)
    Sd, ls = G.clustered_points_torch(w.n_s, w.d, w.n_clusters, w.sigma, ss, cs, ld=w.ld)
    return Rd, Sd, None, None, lr.cpu(), ls.cpu()


def cpu_baseline(Rh, Sh, w, budget_s=15.0, threads=0):
    """FP64 oracle on a bounded row sample of the same workload (threads 0:
    every host core)."""
    from oracle import oracle as O
    threads = threads or O.max_threads()
    rows = 8 if threads > 1 else 1
    t = 0.0
    while True:
        t0 = time.perf_counter()
        O.threshold(Rh[:rows], Sh, w.theta, d=w.d, threads=threads)
        t = time.perf_counter() - t0
        if t >= budget_s / 4 or rows >= Rh.shape[0]:
            break
        rows = min(Rh.shape[0], int(rows * max(2.0, budget_s / 4 / max(t, 1e-3))))
    pairs = rows * Sh.shape[0]
    return {"value": pairs / t / 1e9, "unit": "Gpairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{rows} R rows x all {Sh.shape[0]} S rows of the workload "
                      f"({pairs:.3g} pairs, {t:.1f} s, FP64 sequential dots, "
                      f"{threads} OpenMP thread{'s' if threads > 1 else ''})"}


def _timed(fn):
    """Wall time of fn() in ms, with a device synchronisation on both sides."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, r


def extra_nlj(Rd, Sd, w, out, capacity, n_tensor, ms_tensor):
    """The nested-loop comparator (tile 23: one pair per wavefront, no
    tiling) on the same inputs and the same exact result rule."""
    from paper_2312_01476_amd import ejoin as E
    import torch
    ws = torch.empty(E.threshold_workspace(Rd, Sd, d=w.d, tile=23), dtype=torch.uint8,
                     device="cuda")
    E.threshold_raw(Rd[:512], Sd[:512], w.theta, out, capacity, ws, d=w.d, tile=23)  # load
    ms, (rc, n, st) = _timed(lambda: E.threshold_raw(Rd, Sd, w.theta, out, capacity, ws, d=w.d,
                                                     tile=23, flags=E.TIMING))
    if rc != E.OK:
        raise E.EjoinError(rc, "ejoin_threshold (nlj)")
    res = {"ms": round(ms, 2), "kernel_ms": round(st["ms_main"], 2), "pairs_out": n,
           "same_count_as_tensor": n == n_tensor,
           "time_ratio_nlj_over_tensor": round(ms / ms_tensor, 2),
           "form": "one pair per wavefront, lanes over the 300 dims, no tiling (tile 23)"}
    log(f"[bench] nlj comparator {res}")
    return res


def extra_bf16_1m(args):
    """The 1M x 1M 384-d workload: the BF16 join (bulk contraction in BF16,
    FP64 band recheck) with its roofline and sampled score error against the
    FP64 rule, and the plain FP32 join on the same inputs for the speedup."""
    import numpy as np
    import torch
    from oracle import oracle as O
    from paper_2312_01476_amd import datagen as G
    from paper_2312_01476_amd import ejoin as E
    w = G.WORKLOADS["bf16_1m"]
    cs, rs, ss = w.seeds
    Rd, lr = G.clustered_points_torch(w.n_r, w.d, w.n_clusters, w.sigma, rs, cs, ld=w.ld)
    Sd, ls = G.clustered_points_torch(w.n_s, w.d, w.n_clusters, w.sigma, ss, cs, ld=w.ld)
    cnt_r = torch.bincount(lr, minlength=w.n_clusters).double()
    cnt_s = torch.bincount(ls, minlength=w.n_clusters).double()
    expected = int((cnt_r * cnt_s).sum().item())
    capacity = int(expected * 1.05) + (1 << 20)
    out = torch.empty((capacity, 3), dtype=torch.int32, device="cuda")
    nb = max(E.threshold_workspace(Rd, Sd, d=w.d, prec="bf16", band=w.band),
             E.threshold_workspace(Rd, Sd, d=w.d, prec="fp32"))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    log(f"[bench] bf16_1m inputs resident, label count {expected}")

    def run(prec, flags=0, R=Rd, S=Sd):
        rc, n, st = E.threshold_raw(R, S, w.theta, out, capacity, ws, d=w.d, prec=prec,
                                    band=w.band if prec == "bf16" else None, flags=flags)
        if rc != E.OK:
            raise E.EjoinError(rc, f"ejoin_threshold ({prec})")
        return n, st

    run("bf16")
    steps = 2
    t = []
    mains = []
    for _ in range(steps):
        ms, (n, st) = _timed(lambda: run("bf16", E.TIMING))
        t.append(ms)
        mains.append(st["ms_main"])
    ms_bf16 = float(np.mean(t))
    flops = 2.0 * w.d * w.n_r * w.n_s
    k_ms = float(np.mean(mains))
    tile = E.lib().ejoin_tile_name(st["tile"]).decode()
    # sampled score error of the emitted scores against the FP64 rule
    res = out[:n]
    rng = np.random.Generator(np.random.PCG64(3))
    pick = torch.from_numpy(rng.integers(0, n, size=min(n, 20000))).cuda()
    pr = res[pick, 0].long()
    ps = res[pick, 1].long()
    sc = res[pick, 2].view(torch.float32).cpu().numpy().astype(np.float64)
    Rs = Rd[pr].cpu().numpy()
    Ss = Sd[ps].cpu().numpy()
    i = np.arange(Rs.shape[0])
    ref = O.sim64_pairs(Rs, Ss, i, i, d=w.d)
    err = np.abs(sc - ref)
    # exact set on a leading sub-block
    sub = 2000
    r_all = res[:, 0]
    s_all = res[:, 1]
    m = (r_all < sub) & (s_all < sub)
    got = set(zip(r_all[m].cpu().tolist(), s_all[m].cpu().tolist()))
    ori, osi, _, _ = O.threshold(Rd[:sub].cpu().numpy(), Sd[:sub].cpu().numpy(), w.theta, d=w.d)
    same = got == set(zip(ori.tolist(), osi.tolist()))
    n_bf16, band_pairs = n, st["n_band"]
    # the plain FP32 join on the same inputs (one call; its kernel loaded on a sub-block)
    run("fp32", 0, Rd[:1024], Sd[:1024])
    ms_fp32, (n32, st32) = _timed(lambda: run("fp32", E.TIMING))
    r = {"value": round(w.n_r * w.n_s / (ms_bf16 * 1e-3) / 1e9, 3), "unit": "Gpairs/s",
         "ms_per_step": round(ms_bf16, 2), "steps": steps, "warmup": 1, "dtype": "bf16",
         "config": {"workload": w.name, "n_r": w.n_r, "n_s": w.n_s, "dim": w.d,
                    "theta": w.theta, "band": w.band, "clusters": w.n_clusters,
                    "sigma": w.sigma, "tile": tile, "pairs_out": n_bf16,
                    "band_pairs": band_pairs},
         "roofline": {"bound": "mfma", "achieved": round(flops / (k_ms * 1e-3) / 1e12, 2),
                      "peak": PEAK["bf16"][1], "unit": "TFLOP/s",
                      "frac": round(flops / (k_ms * 1e-3) / 1e12 / PEAK["bf16"][1], 4),
                      "traffic": (round(TRAFFIC[(w.name, tile)])
                                  if (w.name, tile) in TRAFFIC else None),
                      "kernel": "panel_kernel<ThresholdEpi>",
                      "kernel_ms": round(k_ms, 3), "algorithmic_flops_per_launch": flops},
         "score_error_vs_fp64": {"sampled_pairs": int(err.size),
                                 "max_abs": float(err.max()) if err.size else 0.0,
                                 "rms": float(np.sqrt(np.mean(err ** 2))) if err.size else 0.0},
         "verify": {"count_equals_label_count": n_bf16 == expected,
                    "subblock": f"{sub}x{sub}", "subblock_set_equal": bool(same)},
         "fp32_same_inputs": {"ms": round(ms_fp32, 2), "kernel_ms": round(st32["ms_main"], 2),
                              "tile": E.lib().ejoin_tile_name(st32["tile"]).decode(),
                              "pairs_out": n32, "same_count": n32 == n_bf16},
         "speedup_vs_fp32_same_config": round(ms_fp32 / ms_bf16, 3)}
    log(f"[bench] bf16_1m {r}")
    del out, ws, Rd, Sd
    torch.cuda.empty_cache()
    return r


def extra_selectivity(args):
    """The paper's pre-filter sweep on the scan side: a range predicate on a
    relational attribute of S keeps 1-100% of its rows (evaluated on the
    device), then the FP32 E-join of 10k queries with the kept rows, for the
    range predicate sim >= 0.9, top-1, top-32 and the range predicate with a
    cap of k = 32."""
    import torch
    from paper_2312_01476_amd import datagen as G
    from paper_2312_01476_amd import ejoin as E
    w = G.WORKLOADS["sel_10k_1m"]
    cs, rs, ss = w.seeds
    Rd, _ = G.clustered_points_torch(w.n_r, w.d, w.n_clusters, w.sigma, rs, cs, ld=w.ld)
    Sd, _ = G.clustered_points_torch(w.n_s, w.d, w.n_clusters, w.sigma, ss, cs, ld=w.ld)
    attr = G.attribute_column_torch(w.n_s, w.extra["attr_seed"])
    points = []
    # kernels loaded once outside the timings
    ids = E.select_range(attr, 0.0, 0.01)
    E.threshold_sel(Rd, None, Sd, ids, w.theta, d=w.d)
    E.topk_sel(Rd, None, Sd, ids, 1, d=w.d, prec="fp32")
    E.topk_sel(Rd, None, Sd, ids, 32, d=w.d, prec="fp32")
    E.topk_sel(Rd, None, Sd, ids, 32, d=w.d, prec="fp32", min_sim=w.theta)
    for sel in (0.01, 0.1, 0.5, 1.0):
        ms_sel, ids = _timed(lambda: E.select_range(attr, 0.0, sel))
        kept = int(ids.numel())
        pairs = w.n_r * kept
        ms_range, res = _timed(lambda: E.threshold_sel(Rd, None, Sd, ids, w.theta, d=w.d))
        ms_t1, _ = _timed(lambda: E.topk_sel(Rd, None, Sd, ids, 1, d=w.d, prec="fp32"))
        ms_t32, _ = _timed(lambda: E.topk_sel(Rd, None, Sd, ids, 32, d=w.d, prec="fp32"))
        ms_rk, _ = _timed(lambda: E.topk_sel(Rd, None, Sd, ids, 32, d=w.d, prec="fp32",
                                             min_sim=w.theta))
        pt = {"selectivity": sel, "kept_rows": kept, "select_ms": round(ms_sel, 3),
              "range_ms": round(ms_range, 2), "range_pairs_out": len(res),
              "top1_ms": round(ms_t1, 2), "top32_ms": round(ms_t32, 2),
              "range_top32_ms": round(ms_rk, 2),
              "range_gpairs_s": round(pairs / (ms_range * 1e-3) / 1e9, 1)}
        points.append(pt)
        log(f"[bench] selectivity {pt}")
    ms_plain, res = _timed(lambda: E.threshold(Rd, Sd, w.theta, d=w.d))
    r = {"config": {"workload": w.name, "n_r": w.n_r, "n_s": w.n_s, "dim": w.d,
                    "prec": "fp32", "theta": w.theta, "predicate": "attr < selectivity on S"},
         "points": points, "no_selection_range_ms": round(ms_plain, 2),
         "no_selection_pairs_out": len(res)}
    del Rd, Sd, attr
    torch.cuda.empty_cache()
    return r


def extra_child(workload: str, steps: int = 3, warmup: int = 1):
    """One more workload measured by a child process of this script (its
    own seeded inputs, warm-up and timed steps, in HBM before its timed
    region); its progress goes to this process's stderr and its JSON line is
    embedded as printed."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", workload, "--steps",
           str(steps), "--warmup", str(warmup), "--no-cpu"]
    log(f"[bench] extra {workload}: {' '.join(cmd[1:])}")
    r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=900)
    lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"error": f"exit status {r.returncode}"}
    return json.loads(lines[-1])


def calibrate_gemm(torch):
    """Dense BF16 GEMM C = A B^T through torch.matmul (hipBLASLt) at square
    and join-shaped sizes: the practical matrix-core rate of this chip, with
    no epilogue, for comparison with the join's contraction."""
    points = []
    for m, n, k in [(16384, 16384, 16384), (16384, 16384, 4096), (65536, 65536, 384),
                    (32768, 32768, 768)]:
        a = torch.randn(m, k, device="cuda", dtype=torch.bfloat16)
        b = torch.randn(n, k, device="cuda", dtype=torch.bfloat16)
        c = torch.empty(m, n, device="cuda", dtype=torch.bfloat16)
        for _ in range(3):
            torch.matmul(a, b.t(), out=c)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        it = 10
        e0.record()
        for _ in range(it):
            torch.matmul(a, b.t(), out=c)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / it
        tf = 2.0 * m * n * k / (ms * 1e-3) / 1e12
        points.append({"m": m, "n": n, "k": k, "ms": round(ms, 3), "tflops": round(tf, 1),
                       "frac_of_dense_bf16_peak": round(tf / PEAK["bf16"][1], 4)})
        log(f"[bench] bf16 gemm {m}x{n}x{k}: {ms:.3f} ms, {tf:.1f} TF/s")
        del a, b, c
        torch.cuda.empty_cache()
    return {"calibration": "bf16 gemm, torch.matmul", "points": points}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fp32_100k")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy a BYTES-sized device buffer 3 times (reference kernel "
                         "for scaling the HBM traffic counters) and exit")
    ap.add_argument("--calibrate-gemm", action="store_true",
                    help="only time the vendor BF16 GEMM (torch.matmul) at a few shapes, "
                         "the practical matrix-core ceiling the join is compared with, and exit")
    ap.add_argument("--autotune", action="store_true",
                    help="batched workloads: time every tile first and use the fastest")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-verify", action="store_true", help="skip the sampled parity check")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: skip the nested-loop comparator, the 1M x 1M "
                         "BF16 line with its same-input FP32 speedup and the selectivity sweep")
    ap.add_argument("--theta", type=float, default=None,
                    help="threshold workloads, diagnostic: another theta (e.g. 0.999 for a "
                         "run without result pairs); the line then reports the changed config")
    ap.add_argument("--n-s", type=int, default=None,
                    help="threshold workloads, diagnostic: generate only this many S rows")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2312_01476_amd import datagen as G
    from paper_2312_01476_amd import ejoin as E

    if args.calibrate_copy:
        n = args.calibrate_copy // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"[bench] copied {n * 4} bytes 3 times")
        return

    if args.calibrate_gemm:
        print(json.dumps(calibrate_gemm(torch)), flush=True)
        return

    w = G.WORKLOADS[args.workload]
    if w.k is not None:
        return bench_topk(args, w)
    if w.extra.get("batch"):
        return bench_batch(args, w)
    prec = w.prec
    diagnostic = args.theta is not None or args.n_s is not None
    if diagnostic:
        import dataclasses
        w = dataclasses.replace(w, theta=args.theta if args.theta is not None else w.theta,
                                n_s=args.n_s if args.n_s is not None else w.n_s)
        log(f"[bench] diagnostic config: theta {w.theta}, |S| {w.n_s}")
    log(f"[bench] workload {w.name}: {w.notes}")
    Rd, Sd, Rh, Sh, lr, ls = make_inputs(w, torch)
    torch.cuda.synchronize()
    log("[bench] inputs resident")

    stream = torch.cuda.current_stream()
    ws_bytes = E.threshold_workspace(Rd, Sd, d=w.d, prec=prec, band=w.band, tile=args.tile)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
    # expected matches from the generator labels (same-cluster pairs)
    cnt_r = torch.bincount(lr, minlength=w.n_clusters).double()
    cnt_s = torch.bincount(ls, minlength=w.n_clusters).double()
    expected = int((cnt_r * cnt_s).sum().item())
    capacity = int(expected * 1.05) + (1 << 20)
    out = torch.empty((capacity, 3), dtype=torch.int32, device="cuda")

    def step(flags=0):
        rc, n, st = E.threshold_raw(Rd, Sd, w.theta, out, capacity, ws, d=w.d, prec=prec,
                                    band=w.band, tile=args.tile, flags=flags, stream=stream)
        if rc != E.OK:
            raise E.EjoinError(rc, "ejoin_threshold")
        return n, st

    for i in range(args.warmup):
        n, st = step()
        log(f"[bench] warmup {i}: {n} pairs")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mains = []
    for i in range(args.steps):
        n, st = step(E.TIMING)
        mains.append(st["ms_main"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    pairs = w.n_r * w.n_s
    value = pairs / (ms * 1e-3) / 1e9
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step, {value:.1f} Gpairs/s, {n} pairs "
        f"(label count {expected}), band {st['n_band']}")

    # roofline of the dominant kernel (MFMA tile kernel), event-timed on its stream
    ms_main = float(np.mean(mains))
    flops = 2.0 * w.d * pairs
    achieved = flops / (ms_main * 1e-3) / 1e12
    unit, peak = PEAK[prec]
    tile_name = E.lib().ejoin_tile_name(st["tile"]).decode()
    kname = "panel_kernel<ThresholdEpi>" if "panel" in tile_name else "threshold_tile"
    traffic = None if diagnostic else TRAFFIC.get((w.name, tile_name))
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4),
            "traffic": round(traffic) if traffic else None,
            "kernel": kname, "kernel_ms": round(ms_main, 4),
            "algorithmic_flops_per_launch": flops}

    verify = None
    if not args.no_verify:
        # exact set on a leading sub-block + sampled scores against the oracle
        from oracle import oracle as O
        sub = 2000
        res = out[:n]
        r = res[:, 0].cpu().numpy()
        s = res[:, 1].cpu().numpy()
        sc = res[:, 2].view(torch.float32).cpu().numpy()
        Rs = Rh[:sub] if Rh is not None else Rd[:sub].cpu().numpy()
        Ss = Sh[:sub] if Sh is not None else Sd[:sub].cpu().numpy()
        m = (r < sub) & (s < sub)
        ori, osi, _, _ = O.threshold(Rs, Ss, w.theta, d=w.d)
        same = set(zip(r[m].tolist(), s[m].tolist())) == set(zip(ori.tolist(), osi.tolist()))
        rng = np.random.Generator(np.random.PCG64(0))
        pick = rng.integers(0, n, size=min(n, 20000))
        Rfull = Rh if Rh is not None else None
        if Rfull is not None:
            ref = O.sim64_pairs(Rh, Sh, r[pick], s[pick], d=w.d)
            err = float(np.abs(sc[pick] - ref).max()) if len(pick) else 0.0
        else:
            err = None
        verify = {"subblock": f"{sub}x{sub}", "subblock_set_equal": bool(same),
                  "count_equals_label_count": None if diagnostic else bool(n == expected),
                  "sampled_max_abs_score_err": err}
        log(f"[bench] verify {verify}")

    cpu = cpu1 = None
    if not args.no_cpu:
        Rh_ = Rh if Rh is not None else Rd[:4096].cpu().numpy()
        Sh_ = Sh if Sh is not None else Sd.cpu().numpy()
        cpu = cpu_baseline(Rh_, Sh_, w)
        log(f"[bench] cpu baseline {cpu}")
        cpu1 = cpu_baseline(Rh_, Sh_, w, budget_s=8.0, threads=1)
        log(f"[bench] cpu baseline, one core {cpu1}")

    extras = {}
    if w.name == "fp32_100k" and not diagnostic and not args.no_extras:
        extras["nlj_comparator"] = extra_nlj(Rd, Sd, w, out, capacity, n, ms)
        del out
        torch.cuda.empty_cache()
        extras["bf16_1m"] = extra_bf16_1m(args)
        extras["selectivity_sweep"] = extra_selectivity(args)
        # the top-k and batch workloads, each in a child process
        for wl in ("fp8_topk_2m", "batch64_bf16", "batch64_exact_c100"):
            extras[wl] = extra_child(wl)

    line = {
        "metric": "Gpairs/s similarity-join throughput at exact result set",
        "value": round(value, 3),
        "unit": "Gpairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic (seeded clustered embeddings)",
        "config": {"workload": w.name, "n_r": w.n_r, "n_s": w.n_s, "dim": w.d, "ld": w.ld,
                   "theta": w.theta, "prec": prec, "clusters": w.n_clusters,
                   "sigma": w.sigma, "pairs_out": n, "band_pairs": st["n_band"],
                   "tile": E.lib().ejoin_tile_name(st["tile"]).decode(),
                   **({"diagnostic": True} if diagnostic else {})},
        "roofline": roof,
        "cpu_baseline": cpu,
        "cpu_baseline_1core": cpu1,
        "verify": verify,
        **extras,
    }
    print(json.dumps(line), flush=True)


def bench_topk(args, w):
    """Top-k workload: one step = one ejoin_topk call (prep, FP64 norms,
    pilot floor, candidate sweep, certified FP64 finalize, exact fallback)."""
    import numpy as np
    import torch
    from paper_2312_01476_amd import ejoin as E

    log(f"[bench] workload {w.name}: {w.notes}")
    Rd, Sd, Rh, Sh, lr, ls = make_inputs(w, torch)
    torch.cuda.synchronize()
    log("[bench] inputs resident")
    stream = torch.cuda.current_stream()
    ws = torch.empty(E.topk_workspace(Rd, Sd, w.k, d=w.d, prec=w.prec), dtype=torch.uint8,
                     device="cuda")
    idx = torch.empty((w.n_r, w.k), dtype=torch.int32, device="cuda")
    sc = torch.empty((w.n_r, w.k), dtype=torch.float32, device="cuda")

    def step(flags=0):
        rc, st = E.topk_raw(Rd, Sd, w.k, idx, sc, ws, d=w.d, prec=w.prec, flags=flags,
                            stream=stream)
        if rc != E.OK:
            raise E.EjoinError(rc, "ejoin_topk")
        return st

    for i in range(args.warmup):
        st = step()
        log(f"[bench] warmup {i}: fallback rows {st['n_fallback']}, floor {st['topk_floor']:.4f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mains = []
    for i in range(args.steps):
        st = step(E.TIMING)
        mains.append(st["ms_main"])
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    pairs = w.n_r * w.n_s
    value = pairs / (ms * 1e-3) / 1e9
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step, {value:.1f} Gpairs/s, phases "
        f"prep+pilot {st['ms_prep']:.2f} sweep {st['ms_main']:.2f} finalize {st['ms_rescore']:.2f} ms, "
        f"fallback rows {st['n_fallback']}")
    ms_main = float(np.mean(mains))
    flops = 2.0 * w.d * pairs
    unit, peak = PEAK[w.prec]
    roof = {"bound": "mfma", "achieved": round(flops / (ms_main * 1e-3) / 1e12, 2), "peak": peak,
            "unit": unit, "frac": round(flops / (ms_main * 1e-3) / 1e12 / peak, 4),
            "traffic": None, "kernel": "panel_kernel<CandEpi>", "kernel_ms": round(ms_main, 4),
            "algorithmic_flops_per_launch": flops}
    verify = None
    if not args.no_verify:
        from oracle import oracle as O
        rng = np.random.Generator(np.random.PCG64(1))
        rows = np.sort(rng.choice(w.n_r, size=64, replace=False))
        Rs = Rd[torch.from_numpy(rows).cuda()].cpu().numpy()
        Sh_ = Sh if Sh is not None else Sd.cpu().numpy()
        oi, osc = O.topk(Rs, Sh_, w.k, d=w.d)
        gi = idx[torch.from_numpy(rows).cuda()].cpu().numpy()
        gs = sc[torch.from_numpy(rows).cuda()].cpu().numpy()
        verify = {"sampled_rows": int(rows.size),
                  "idx_equal": bool(np.array_equal(gi, oi)),
                  "scores_equal_f32": bool(np.array_equal(gs, osc.astype(np.float32))),
                  "same_cluster": bool(np.all(np.asarray(ls)[gi] == np.asarray(lr)[rows][:, None]))}
        log(f"[bench] verify {verify}")
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        Sh_ = Sh if Sh is not None else Sd.cpu().numpy()
        Rs = Rd[:4096].cpu().numpy()
        threads = O.max_threads()
        rows = 4
        while True:
            t0 = time.perf_counter()
            O.topk(Rs[:rows], Sh_, w.k, d=w.d)
            t = time.perf_counter() - t0
            if t >= 4.0 or rows >= Rs.shape[0]:
                break
            rows = min(Rs.shape[0], int(rows * max(2.0, 4.0 / max(t, 1e-3))))
        cpu = {"value": rows * w.n_s / t / 1e9, "unit": "Gpairs/s", "cores": threads,
               "kind": "oracle", "sample": f"{rows} R rows x all {w.n_s} S rows, top-{w.k} "
                                            f"({t:.1f} s, {threads} OpenMP threads)"}
        log(f"[bench] cpu baseline {cpu}")
    line = {
        "metric": "Gpairs/s similarity-join throughput at exact result set",
        "value": round(value, 3), "unit": "Gpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[w.prec],
        "data": "synthetic (seeded clustered embeddings)",
        "config": {"workload": w.name, "n_r": w.n_r, "n_s": w.n_s, "dim": w.d, "k": w.k,
                   "prec": w.prec, "clusters": w.n_clusters, "sigma": w.sigma,
                   "fallback_rows": st["n_fallback"], "floor": st["topk_floor"],
                   "slots": st["topk_slots"]},
        "roofline": roof, "cpu_baseline": cpu, "verify": verify,
    }
    print(json.dumps(line), flush=True)


def bench_batch(args, w):
    """Batched workload: one step = one ejoin_batch pass over all jobs (table
    upload, batched prep, one persistent tile launch, batched FP64 rescore,
    counts), inputs resident.  The same pass replayed through the captured
    graph is timed afterwards and reported beside it."""
    import numpy as np
    import torch
    from paper_2312_01476_amd import datagen as G
    from paper_2312_01476_amd import ejoin as E

    log(f"[bench] workload {w.name}: {w.notes}")
    shapes = G.batch_jobs(n_jobs=w.extra["batch"], d=w.d, seed=w.extra["job_seed"])
    jobs, labels = [], []
    for j in shapes:
        Rd, lr = G.clustered_points_torch(j["n_r"], w.d, w.n_clusters, w.sigma, j["seed_r"],
                                          w.seeds[0], ld=w.ld)
        Sd, ls = G.clustered_points_torch(j["n_s"], w.d, w.n_clusters, w.sigma, j["seed_s"],
                                          w.seeds[0], ld=w.ld)
        jobs.append((Rd, Sd, j["theta"]))
        labels.append((lr, ls))
    torch.cuda.synchronize()
    pairs = sum(j["n_r"] * j["n_s"] for j in shapes)
    log(f"[bench] {len(jobs)} jobs resident, {pairs / 1e9:.2f} Gpairs")
    # capacities: same-cluster pairs (a bound for theta above the cross-cluster
    # similarities) plus slack
    caps = []
    for lr, ls in labels:
        cr = torch.bincount(lr, minlength=w.n_clusters).double()
        cs = torch.bincount(ls, minlength=w.n_clusters).double()
        caps.append(int((cr * cs).sum().item() * 1.05) + 4096)
    outs = [torch.empty((c, 3), dtype=torch.int32, device="cuda") for c in caps]
    stream = torch.cuda.current_stream()
    band_cap = 0
    ws = None
    n_out = torch.zeros(len(jobs), dtype=torch.int64)
    for attempt in range(3):
        ws_bytes = E.batch_workspace(jobs, d=w.d, prec=w.prec, tile=args.tile,
                                     band_capacity=band_cap)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device="cuda")
        rc, st = E.batch_raw(jobs, outs, caps, ws, n_out, d=w.d, prec=w.prec, tile=args.tile,
                             band_capacity=band_cap, stream=stream)
        if rc == E.E_WORKSPACE and st["band_needed"] > 0:
            band_cap = int(st["band_needed"] * 1.1) + 4096
            del ws
            continue
        if rc != E.OK:
            raise E.EjoinError(rc, "ejoin_batch")
        break
    log(f"[bench] ws {ws.numel() / 2**30:.2f} GiB, band list {band_cap or 'default'}")
    tuned = None
    if args.autotune and args.tile == 0:
        tuner = E.Tuner()
        best, tms = tuner.autotune(jobs, outs, caps, ws, d=w.d, prec=w.prec,
                                   band_capacity=band_cap, reps=1)
        tuned = {E.lib().ejoin_tile_name(t).decode(): round(v, 2) for t, v in tms.items()}
        log(f"[bench] autotune: {tuned} -> {best}")
        args.tile = best

    def step(flags=0):
        rc, st = E.batch_raw(jobs, outs, caps, ws, n_out, d=w.d, prec=w.prec, tile=args.tile,
                             band_capacity=band_cap, flags=flags, stream=stream)
        if rc != E.OK:
            raise E.EjoinError(rc, "ejoin_batch")
        return st

    for i in range(args.warmup):
        st = step()
        log(f"[bench] warmup {i}: {st['n_pairs']} pairs, band {st['n_band']}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mains, phases = [], []
    for i in range(args.steps):
        st = step(E.TIMING)
        mains.append(st["ms_main"])
        phases.append((st["ms_prep"], st["ms_main"], st["ms_rescore"]))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    value = pairs / (ms * 1e-3) / 1e9
    counts = n_out.tolist()
    ph = np.mean(np.array(phases), axis=0)
    log(f"[bench] {args.steps} steps: {ms:.3f} ms/step, {value:.1f} Gpairs/s; prep {ph[0]:.2f} "
        f"tiles {ph[1]:.2f} rescore {ph[2]:.2f} ms; {sum(counts)} pairs, band {st['n_band']}")

    # the same pass through the captured graph (device counts)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = E.BatchGraph(len(jobs), ws, prec=w.prec, tile=st["tile"], band_capacity=band_cap,
                     stream=side)
    n_dev = torch.zeros(len(jobs), dtype=torch.int64, device="cuda")
    g.launch(jobs, outs, caps, n_dev, d=w.d, stream=side)
    torch.cuda.synchronize()
    graph_same = n_dev.cpu().tolist() == counts
    t0 = time.perf_counter()
    for i in range(args.steps):
        g.launch(jobs, outs, caps, n_dev, d=w.d, stream=side)
    torch.cuda.synchronize()
    graph_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    g.close()
    log(f"[bench] graph replay {graph_ms:.3f} ms/step, counts equal eager: {graph_same}")

    ms_main = float(np.mean(mains))
    flops = 2.0 * w.d * pairs
    unit, peak = PEAK[w.prec]
    achieved = flops / (ms_main * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4),
            "traffic": TRAFFIC.get((w.name, E.lib().ejoin_tile_name(st["tile"]).decode())),
            "kernel": {19: "batch_panel", 22: "batch_panel2"}.get(st["tile"], "batch_tile"),
            "kernel_ms": round(ms_main, 4), "algorithmic_flops_per_launch": flops}

    verify = None
    if not args.no_verify:
        # exact set of every job on its leading sub-block against the oracle
        from oracle import oracle as O
        sub = 400
        ok = 0
        for q, ((Rd, Sd, th), o) in enumerate(zip(jobs, outs)):
            res = o[:counts[q]]
            m = (res[:, 0] < sub) & (res[:, 1] < sub)
            got = res[m][:, :2].cpu().numpy()
            Rs = Rd[:sub].cpu().numpy()
            Ss = Sd[:sub].cpu().numpy()
            ori, osi, _, _ = O.threshold(Rs, Ss, th, d=w.d)
            ok += set(map(tuple, got.tolist())) == set(zip(ori.tolist(), osi.tolist()))
        verify = {"jobs": len(jobs), "subblock": f"{sub}x{sub} per job",
                  "jobs_set_equal": ok, "graph_counts_equal_eager": graph_same}
        log(f"[bench] verify {verify}")

    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        threads = O.max_threads()
        big = max(range(len(jobs)), key=lambda q: shapes[q]["n_s"])
        Rd, Sd, th = jobs[big]
        Rh = Rd[:2048].cpu().numpy()
        Sh = Sd.cpu().numpy()
        rows = 2
        while True:
            t0 = time.perf_counter()
            O.threshold(Rh[:rows], Sh, th, d=w.d)
            t = time.perf_counter() - t0
            if t >= 4.0 or rows >= Rh.shape[0]:
                break
            rows = min(Rh.shape[0], int(rows * max(2.0, 4.0 / max(t, 1e-3))))
        cpu = {"value": rows * Sh.shape[0] / t / 1e9, "unit": "Gpairs/s", "cores": threads,
               "kind": "oracle",
               "sample": f"{rows} R rows x all {Sh.shape[0]} S rows of the job with the "
                         f"largest S ({t:.1f} s, {threads} OpenMP threads)"}
        log(f"[bench] cpu baseline {cpu}")

    if w.extra.get("prefilter"):
        return bench_prefilter(args, w, jobs, outs, caps, counts, pairs, ms, ph, roof, st,
                               verify, cpu, band_cap)
    if w.extra.get("exact_prune"):
        return bench_exact_prune(args, w, jobs, outs, caps, counts, pairs, ms, roof, st, verify,
                                 cpu, band_cap)
    line = {
        "metric": "Gpairs/s similarity-join throughput at exact result set",
        "value": round(value, 3), "unit": "Gpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[w.prec],
        "data": "synthetic (seeded clustered embeddings)",
        "config": {"workload": w.name, "jobs": len(jobs), "pairs": pairs, "dim": w.d,
                   "prec": w.prec, "clusters": w.n_clusters, "sigma": w.sigma,
                   "pairs_out": int(sum(counts)), "band_pairs": st["n_band"],
                   "tile": E.lib().ejoin_tile_name(st["tile"]).decode(),
                   "phase_ms": {"prep": round(ph[0], 3), "tiles": round(ph[1], 3),
                                "rescore": round(ph[2], 3)},
                   "graph_ms_per_step": round(graph_ms, 4), "autotune_ms": tuned},
        "roofline": roof, "cpu_baseline": cpu, "verify": verify,
    }
    print(json.dumps(line), flush=True)


def bench_exact_prune(args, w, jobs, outs, caps, counts, pairs, plain_ms, plain_roof, plain_st,
                      plain_verify, cpu, band_cap):
    """Exact tile pruning on the batched workload: the same jobs through the
    pruned pass (projection codes, ordering, certified tile-to-rows bounds in
    the original space).  value = pairs / pruned step time; every job's count
    and pair set must equal the plain pass just measured."""
    import numpy as np
    import torch
    from paper_2312_01476_amd import ejoin as E

    stream = torch.cuda.current_stream()
    pouts = [torch.empty((c, 3), dtype=torch.int32, device="cuda") for c in caps]
    pcount = torch.zeros(len(jobs), dtype=torch.int64)
    ws = torch.empty(E.batch_workspace(jobs, d=w.d, prec=w.prec, band_capacity=band_cap,
                                       flags=E.EXACT_PRUNE), dtype=torch.uint8, device="cuda")

    def step(flags=0):
        rc, st = E.batch_raw(jobs, pouts, caps, ws, pcount, d=w.d, prec=w.prec,
                             flags=flags | E.EXACT_PRUNE, stream=stream, band_capacity=band_cap)
        if rc != E.OK:
            raise E.EjoinError(rc, "ejoin_batch (exact pruning)")
        return st

    for _ in range(args.warmup):
        st = step()
    same_counts = [int(pcount[q]) for q in range(len(jobs))] == [int(c) for c in counts]
    same_sets = True
    for q in range(len(jobs)):
        c = int(counts[q])
        if c:
            a = torch.sort(outs[q][:c, 0].long() * (1 << 31) + outs[q][:c, 1].long()).values
            b = torch.sort(pouts[q][:c, 0].long() * (1 << 31) + pouts[q][:c, 1].long()).values
            same_sets &= bool(torch.equal(a, b))
    torch.cuda.synchronize()
    phases = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = step(E.TIMING)
        phases.append((st["ms_prep"], st["ms_main"], st["ms_rescore"]))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ph = np.mean(np.array(phases), axis=0)
    kept = st["tiles_kept"] / max(1, st["tiles_total"])
    value = pairs / (ms * 1e-3) / 1e9
    log(f"[bench] exact pruning: {ms:.2f} ms/step ({plain_ms / ms:.2f}x the plain batch), "
        f"{value:.1f} Gpairs/s, same counts {same_counts}, same sets {same_sets}, "
        f"tile pairs kept {kept:.4f}; codes+order+bounds {ph[0]:.2f} tiles {ph[1]:.2f} "
        f"rescore {ph[2]:.2f} ms")
    kms = float(ph[1])
    flops_kept = 2.0 * w.d * pairs * kept
    unit, peak = PEAK[w.prec]
    line = {
        "metric": "Gpairs/s similarity-join throughput at exact result set",
        "value": round(value, 3), "unit": "Gpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[w.prec],
        "data": "synthetic (seeded clustered embeddings)",
        "config": {"workload": w.name, "jobs": len(jobs), "pairs": pairs, "dim": w.d,
                   "prec": w.prec, "clusters": w.n_clusters, "sigma": w.sigma,
                   "pairs_out": int(sum(counts)),
                   "tile": E.lib().ejoin_tile_name(st["tile"]).decode(),
                   "tile_pairs_kept": round(kept, 4),
                   "phase_ms": {"codes_order_bounds": round(float(ph[0]), 3),
                                "tiles": round(kms, 3), "rescore": round(float(ph[2]), 3)},
                   "plain_batch_ms": round(plain_ms, 3),
                   "speedup_vs_plain_batch": round(plain_ms / ms, 3)},
        "roofline": {"bound": "mfma",
                     "achieved": round(flops_kept / (kms * 1e-3) / 1e12, 2), "peak": peak,
                     "unit": unit, "frac": round(flops_kept / (kms * 1e-3) / 1e12 / peak, 4),
                     "traffic": None, "kernel": "batch_panel2<true>", "kernel_ms": round(kms, 4),
                     "algorithmic_flops_per_launch": flops_kept},
        "cpu_baseline": cpu,
        "verify": {"counts_equal_plain": same_counts, "sets_equal_plain": same_sets,
                   "plain": plain_verify},
    }
    print(json.dumps(line), flush=True)


def bench_prefilter(args, w, jobs, outs, caps, counts, pairs, plain_ms, plain_ph, plain_roof,
                    plain_st, plain_verify, cpu, band_cap):
    """Learned prefilter on the batched workload: train the network on pairs
    drawn from the exact batch output just computed, then time the
    prefiltered pass.  value = pairs / prefiltered step time; the result is
    approximate and its recall against the exact output is reported, with
    the same pass through the untrained network as the ablation."""
    import numpy as np
    import torch
    from paper_2312_01476_amd import datagen as G
    from paper_2312_01476_amd import ejoin as E

    x = w.extra
    flat = G.mlp_init(w.d, x["mlp_seed"])
    net = E.Mlp(w.d, torch.from_numpy(flat))
    raw = E.Mlp(w.d, torch.from_numpy(flat))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = E.prefilter_train(net, jobs, outs, caps, counts, d=w.d, steps=x["train_steps"],
                               batch=x["train_batch"], seed=7, hp={"lr": 2e-3})
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    log(f"[bench] trained {x['train_steps']} steps x {x['train_batch']} pairs in {train_s:.2f} s;"
        f" loss {np.mean(losses[:5]):.4f} -> {np.mean(losses[-10:]):.4f}")
    # exact output keys per job, for recall and the subset check
    exact = []
    for q, o in enumerate(outs):
        c = counts[q]
        r = o[:c, 0].long()
        s = o[:c, 1].long()
        exact.append(torch.sort(r * (1 << 31) + s).values)
    eps = x["eps"]
    stream = torch.cuda.current_stream()
    pouts = [torch.empty((c, 3), dtype=torch.int32, device="cuda") for c in caps]
    pcount = torch.zeros(len(jobs), dtype=torch.int64)

    def run(model, flags=0):
        ws_b = E.batch_workspace(jobs, d=w.d, prec="bf16", prefilter=model, eps=eps,
                                 band_capacity=band_cap)
        ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
        rc, st = E.batch_raw(jobs, pouts, caps, ws, pcount, d=w.d, prec="bf16", flags=flags,
                             stream=stream, prefilter=model, eps=eps, band_capacity=band_cap)
        if rc != E.OK:
            raise E.EjoinError(rc, "ejoin_batch (prefiltered)")
        return ws, st

    def recall_of():
        got = 0
        subset = True
        for q in range(len(jobs)):
            c = int(pcount[q])
            got += c
            if c:
                k = pouts[q][:c, 0].long() * (1 << 31) + pouts[q][:c, 1].long()
                subset &= bool(torch.isin(k, exact[q]).all().item())
        return got / max(1, sum(counts)), subset

    ws, st = run(net)  # warm-up
    rec, subset = recall_of()
    del ws
    torch.cuda.synchronize()
    ws_b = E.batch_workspace(jobs, d=w.d, prec="bf16", prefilter=net, eps=eps,
                             band_capacity=band_cap)
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    phases = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        rc, st = E.batch_raw(jobs, pouts, caps, ws, pcount, d=w.d, prec="bf16", flags=E.TIMING,
                             stream=stream, prefilter=net, eps=eps, band_capacity=band_cap)
        if rc != E.OK:
            raise E.EjoinError(rc, "ejoin_batch (prefiltered)")
        phases.append((st["ms_prep"], st["ms_main"], st["ms_rescore"]))
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    del ws
    ph = np.mean(np.array(phases), axis=0)
    kept = st["tiles_kept"] / max(1, st["tiles_total"])
    value = pairs / (ms * 1e-3) / 1e9
    log(f"[bench] prefiltered: {ms:.2f} ms/step ({plain_ms / ms:.2f}x the plain batch), "
        f"{value:.1f} Gpairs/s, recall {rec:.5f}, subset {subset}, tile pairs kept {kept:.4f}; "
        f"codes+order+bounds {ph[0]:.2f} tiles {ph[1]:.2f} rescore {ph[2]:.2f} ms")
    # ablation: the untrained network
    torch.cuda.synchronize()
    ws0, st0 = run(raw, flags=E.TIMING)
    rec0, subset0 = recall_of()
    kept0 = st0["tiles_kept"] / max(1, st0["tiles_total"])
    log(f"[bench] untrained: {st0['ms_total']:.2f} ms, recall {rec0:.5f}, kept {kept0:.4f}")
    del ws0

    line = {
        "metric": "Gpairs/s similarity-join throughput, approximate (learned prefilter; "
                  "recall vs the exact join reported)",
        "value": round(value, 3), "unit": "Gpairs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic (seeded clustered embeddings)",
        "config": {"workload": w.name, "jobs": len(jobs), "pairs": pairs, "dim": w.d,
                   "clusters": w.n_clusters, "sigma": w.sigma, "eps": eps,
                   "recall": round(rec, 6), "precision_is_one": subset,
                   "tile_pairs_kept": round(kept, 5),
                   "plain_batched_ms": round(plain_ms, 3),
                   "speedup_vs_plain_batched": round(plain_ms / ms, 3),
                   "phase_ms": {"prep_codes_order_bounds": round(ph[0], 3),
                                "tiles": round(ph[1], 3), "rescore": round(ph[2], 3)},
                   "train": {"steps": x["train_steps"], "batch": x["train_batch"],
                             "seconds": round(train_s, 3),
                             "loss_first": round(float(np.mean(losses[:5])), 5),
                             "loss_last": round(float(np.mean(losses[-10:])), 5)},
                   "untrained": {"recall": round(rec0, 6), "tile_pairs_kept": round(kept0, 5),
                                 "ms": round(st0["ms_total"], 3), "precision_is_one": subset0}},
        "roofline": plain_roof | {"note": "plain batched pass (the prefiltered pass skips tiles)"},
        "cpu_baseline": cpu, "verify": plain_verify,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
