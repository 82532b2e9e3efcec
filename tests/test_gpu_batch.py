"""Parity of the batched threshold join (ejoin_batch, its captured graph and
the autotuner) with the FP64 oracle, through the C ABI.

Every job of a batch must return exactly the oracle's threshold set for its
own R, S and theta, whatever the job mix, tile shape, output capacity or
band-list capacity; scores obey the same bounds as the single join.
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


def _job_mix(d=96, seed=7):
    """Uneven jobs: clustered blocks, a self-join, empty and 1-row relations,
    ragged sizes; thresholds from each job's own similarity quantiles."""
    rng = np.random.default_rng(seed)
    cent = G.centres(d, 12, seed + 1)
    host = []
    shapes = [(700, 300), (1, 1), (0, 50), (129, 257), (300, 0), (513, 65), (64, 64),
              (1000, 1), (250, 250)]
    for i, (nr, ns) in enumerate(shapes):
        R = G.clustered_points(cent, nr, 0.35, seed * 100 + 2 * i)[0] if nr else \
            np.zeros((0, d), np.float32)
        S = G.clustered_points(cent, ns, 0.35, seed * 100 + 2 * i + 1)[0] if ns else \
            np.zeros((0, d), np.float32)
        if nr and ns:
            sims = O.sim_matrix(R, S)
            theta = float(np.quantile(sims, rng.uniform(0.6, 0.995)))
        else:
            theta = 0.5
        host.append((R, S, theta))
    # self-join (same device tensor for R and S)
    X = G.clustered_points(cent, 400, 0.35, seed * 100 + 99)[0]
    host.append((X, X, float(np.quantile(O.sim_matrix(X, X), 0.98))))
    return host


def _to_dev(host):
    jobs = []
    for R, S, th in host:
        Rd = _dev(R)
        Sd = Rd if S is R else _dev(S)
        jobs.append((Rd, Sd, th))
    return jobs


def _check_job(R, S, theta, res, prec, band, d=None):
    r = res.r.cpu().numpy().astype(np.int64)
    s = res.s.cpu().numpy().astype(np.int64)
    sc = res.score.cpu().numpy().astype(np.float64)
    if R.shape[0] == 0 or S.shape[0] == 0:
        assert len(r) == 0
        return
    ori, osi, _, _ = O.threshold(R, S, theta, d=d)
    got = set(zip(r.tolist(), s.tolist()))
    want = set(zip(ori.tolist(), osi.tolist()))
    assert len(got) == len(r), "duplicate pairs"
    assert got == want, (prec, len(want - got), len(got - want))
    if len(r):
        ref = O.sim64_pairs(R, S, r, s, d=d)
        tol = 1e-3 if prec == "fp32" else band
        assert np.abs(sc - ref).max() <= tol


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_batch_equals_oracle_per_job(prec):
    host = _job_mix()
    jobs = _to_dev(host)
    res, st = E.batch(jobs, prec=prec)
    assert len(res) == len(host)
    for (R, S, th), rr in zip(host, res):
        _check_job(R, S, th, rr, prec, st["band"])


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_equals_single_calls(prec):
    host = _job_mix(seed=11)
    jobs = _to_dev(host)
    res, _ = E.batch(jobs, prec=prec)
    for (Rd, Sd, th), rr in zip(jobs, res):
        one = E.threshold(Rd, Sd, th, prec=prec, tile=1 if prec == "fp32" else 3)
        a = set(zip(one.r.cpu().tolist(), one.s.cpu().tolist()))
        b = set(zip(rr.r.cpu().tolist(), rr.s.cpu().tolist()))
        assert a == b


@pytest.mark.parametrize("tile", [1, 2, 11, 18])
def test_batch_tile_invariance_fp32(tile):
    host = _job_mix(seed=13)
    jobs = _to_dev(host)
    res, st = E.batch(jobs, prec="fp32", tile=tile)
    assert st["tile"] == tile
    for (R, S, th), rr in zip(host, res):
        _check_job(R, S, th, rr, "fp32", st["band"])


@pytest.mark.parametrize("tile", [3, 4, 8, 16])
def test_batch_tile_invariance_bf16(tile):
    host = _job_mix(seed=17)
    jobs = _to_dev(host)
    res, st = E.batch(jobs, prec="bf16", tile=tile)
    assert st["tile"] == tile
    for (R, S, th), rr in zip(host, res):
        _check_job(R, S, th, rr, "bf16", st["band"])


def test_batch_panel_form_bf16():
    """Tiles 19 and 22 (register panels, 128-row panels swept over chunks of
    16 x 128 S columns; one or two workgroups per CU): jobs of 768-, 640-,
    560- and 500-d rows in one batch, one job with several panels and S
    chunks; one of them is the default for such a batch."""
    host = _job_mix(d=768, seed=23)[:4] + _job_mix(d=640, seed=29)[4:7] + \
        _job_mix(d=560, seed=31)[7:] + _job_mix(d=500, seed=33)[:3]
    cent = G.centres(768, 20, seed=37)
    R = G.clustered_points(cent, 300, 0.3, seed=38)[0]
    S = G.clustered_points(cent, 5000, 0.3, seed=39)[0]
    host.append((R, S, float(np.quantile(O.sim_matrix(R[:50], S), 0.99))))
    jobs = _to_dev(host)
    for tile in (19, 22, 0):
        res, st = E.batch(jobs, prec="bf16", tile=tile)
        assert st["tile"] == tile if tile else st["tile"] in (19, 22)
        for (R_, S_, th), rr in zip(host, res):
            _check_job(R_, S_, th, rr, "bf16", st["band"])


def test_batch_panel_form_rejects_other_depths():
    jobs = _to_dev(_job_mix(d=96, seed=41))
    with pytest.raises(E.EjoinError):
        E.batch(jobs, prec="bf16", tile=19)


@pytest.mark.parametrize("tile", [19, 22])
def test_batch_panel_form_retries_counts_nonfinite_and_graph(tile):
    """The batch panel form (640-d and 768-d jobs) through the raw call:
    overflow and band-list retries, device counts, a job with a NaN isolated,
    and a captured graph replayed for two batches with eager work between;
    a graph of the panel form refuses jobs of another depth."""
    host = _job_mix(d=640, seed=59)
    jobs = _to_dev(host)
    ref, st = E.batch(jobs, prec="bf16", tile=tile)
    assert st["tile"] == tile
    for (R, S, th), rr in zip(host, ref):
        _check_job(R, S, th, rr, "bf16", st["band"])
    want = [set(zip(r.r.cpu().tolist(), r.s.cpu().tolist())) for r in ref]
    # tiny outputs and band list: the raw call reports the true sizes
    caps = [3] * len(jobs)
    ws = torch.empty(E.batch_workspace(jobs, prec="bf16", tile=tile, band_capacity=16),
                     dtype=torch.uint8, device="cuda")
    outs = [torch.empty((c, 3), dtype=torch.int32, device="cuda") for c in caps]
    n_out = torch.zeros(len(jobs), dtype=torch.int64)
    rc, st = E.batch_raw(jobs, outs, caps, ws, n_out, prec="bf16", tile=tile, band_capacity=16)
    assert rc == E.E_WORKSPACE and st["band_needed"] > 16
    res, st = E.batch(jobs, prec="bf16", tile=tile, capacities=caps, band_capacity=16)
    assert [set(zip(r.r.cpu().tolist(), r.s.cpu().tolist())) for r in res] == want
    # device counts
    caps = [len(r) + 5 for r in ref]
    ws = torch.empty(E.batch_workspace(jobs, prec="bf16", tile=tile), dtype=torch.uint8,
                     device="cuda")
    outs = [torch.empty((max(c, 1), 3), dtype=torch.int32, device="cuda") for c in caps]
    n_dev = torch.full((len(jobs),), -99, dtype=torch.int64, device="cuda")
    rc, _ = E.batch_raw(jobs, outs, caps, ws, n_dev, prec="bf16", tile=tile, flags=E.NO_SYNC)
    assert rc == E.OK
    torch.cuda.synchronize()
    assert n_dev.cpu().tolist() == [len(r) for r in ref]
    # a NaN in one job's R: that job fails, the others are exact
    badh = list(host)
    bad = host[3][0].copy()
    bad[5, 3] = np.nan
    badh[3] = (bad, host[3][1], host[3][2])
    bjobs = _to_dev(badh)
    caps = [200_000] * len(bjobs)
    ws = torch.empty(E.batch_workspace(bjobs, prec="bf16", tile=tile), dtype=torch.uint8,
                     device="cuda")
    outs = [torch.empty((c, 3), dtype=torch.int32, device="cuda") for c in caps]
    n_out = torch.zeros(len(bjobs), dtype=torch.int64)
    rc, _ = E.batch_raw(bjobs, outs, caps, ws, n_out, prec="bf16", tile=tile)
    assert rc == E.E_NONFINITE
    assert int(n_out[3]) == 0
    for q in range(len(bjobs)):
        if q != 3:
            c = int(n_out[q])
            assert set(map(tuple, outs[q][:c, :2].cpu().tolist())) == want[q]
    # a graph of the panel form, replayed for two batches
    hostB = _job_mix(d=768, seed=61)[:6]
    jobsB = _to_dev(hostB)
    refB, _ = E.batch(jobsB, prec="bf16")
    wantB = [set(zip(r.r.cpu().tolist(), r.s.cpu().tolist())) for r in refB]
    ws_bytes = max(E.batch_workspace(jobs, prec="bf16", tile=tile, band_capacity=1 << 20),
                   E.batch_workspace(jobsB, prec="bf16", tile=tile, band_capacity=1 << 20))
    ws = torch.empty(ws_bytes + (1 << 16), dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = E.BatchGraph(len(jobs), ws, prec="bf16", tile=tile, band_capacity=1 << 20, stream=side)
    try:
        for js, rf, w in ((jobs, ref, want), (jobsB, refB, wantB), (jobs, ref, want)):
            n, got = _graph_run(g, js, [len(r) + 8 for r in rf], side)
            assert n == [len(x) for x in w]
            assert got == w
            E.batch(jobsB[:2], prec="bf16")
            torch.cuda.synchronize()
        small = _to_dev(_job_mix(d=96, seed=67)[:3])
        outs = [torch.empty((8, 3), dtype=torch.int32, device="cuda") for _ in small]
        n_dev = torch.zeros(len(small), dtype=torch.int64, device="cuda")
        with pytest.raises(E.EjoinError):
            g.launch(small, outs, [8] * len(small), n_dev, stream=side)
        torch.cuda.synchronize()
    finally:
        g.close()


def test_batch_fp8_tiles():
    host = _job_mix(seed=19)
    jobs = _to_dev(host)
    for tile in (5, 6, 10, 17):
        res, st = E.batch(jobs, prec="fp8", tile=tile)
        for (R, S, th), rr in zip(host, res):
            _check_job(R, S, th, rr, "fp8", st["band"])


def test_batch_overflow_and_band_retry():
    """Tiny output capacities and a tiny shared band list: the raw call
    reports overflow / workspace with the true sizes, the binding's retries
    reach the exact sets."""
    host = _job_mix(seed=23)
    jobs = _to_dev(host)
    caps = [3] * len(jobs)
    ws = torch.empty(E.batch_workspace(jobs, prec="bf16", band_capacity=16), dtype=torch.uint8,
                     device="cuda")
    outs = [torch.empty((c, 3), dtype=torch.int32, device="cuda") for c in caps]
    n_out = torch.zeros(len(jobs), dtype=torch.int64)
    rc, st = E.batch_raw(jobs, outs, caps, ws, n_out, prec="bf16", band_capacity=16)
    assert rc == E.E_WORKSPACE and st["band_needed"] > 16
    res, st = E.batch(jobs, prec="bf16", capacities=caps, band_capacity=16)
    for (R, S, th), rr in zip(host, res):
        _check_job(R, S, th, rr, "bf16", st["band"])


def test_batch_overflow_counts_exact():
    host = _job_mix(seed=29)
    jobs = _to_dev(host)
    ref, _ = E.batch(jobs, prec="fp32")
    caps = [max(0, len(r) // 2) for r in ref]
    ws = torch.empty(E.batch_workspace(jobs, prec="fp32"), dtype=torch.uint8, device="cuda")
    outs = [torch.empty((max(c, 1), 3), dtype=torch.int32, device="cuda") for c in caps]
    n_out = torch.zeros(len(jobs), dtype=torch.int64)
    rc, _ = E.batch_raw(jobs, outs, caps, ws, n_out, prec="fp32")
    assert rc == (E.E_OVERFLOW if any(len(r) > c for r, c in zip(ref, caps)) else E.OK)
    assert n_out.tolist() == [len(r) for r in ref]
    # the stored subset of an overflowing job is still a subset of the result
    for o, c, r in zip(outs, caps, ref):
        if c == 0:
            continue
        sub = set(map(tuple, o[:c, :2].cpu().tolist()))
        full = set(zip(r.r.cpu().tolist(), r.s.cpu().tolist()))
        assert sub <= full


def test_batch_no_sync_device_counts():
    host = _job_mix(seed=31)
    jobs = _to_dev(host)
    ref, _ = E.batch(jobs, prec="bf16")
    caps = [len(r) + 5 for r in ref]
    ws = torch.empty(E.batch_workspace(jobs, prec="bf16"), dtype=torch.uint8, device="cuda")
    outs = [torch.empty((max(c, 1), 3), dtype=torch.int32, device="cuda") for c in caps]
    n_dev = torch.full((len(jobs),), -99, dtype=torch.int64, device="cuda")
    rc, _ = E.batch_raw(jobs, outs, caps, ws, n_dev, prec="bf16", flags=E.NO_SYNC)
    assert rc == E.OK
    torch.cuda.synchronize()
    assert n_dev.cpu().tolist() == [len(r) for r in ref]


def test_batch_nonfinite_job_isolated():
    host = _job_mix(seed=37)
    bad = host[3][0].copy()
    bad[5, 3] = np.nan
    host[3] = (bad, host[3][1], host[3][2])
    jobs = _to_dev(host)
    caps = [200_000] * len(jobs)
    ws = torch.empty(E.batch_workspace(jobs, prec="fp32"), dtype=torch.uint8, device="cuda")
    outs = [torch.empty((c, 3), dtype=torch.int32, device="cuda") for c in caps]
    n_out = torch.zeros(len(jobs), dtype=torch.int64)
    rc, _ = E.batch_raw(jobs, outs, caps, ws, n_out, prec="fp32")
    assert rc == E.E_NONFINITE
    assert int(n_out[3]) == 0
    for q, (R, S, th) in enumerate(host):
        if q == 3:
            continue
        c = int(n_out[q])
        o = outs[q][:c].cpu().numpy()
        want = O.threshold(R, S, th)[0].shape[0] if R.shape[0] and S.shape[0] else 0
        assert c == want


def test_batch_rejects_panel_tile_and_bad_theta():
    host = _job_mix(seed=41)[:3]
    jobs = _to_dev(host)
    with pytest.raises(E.EjoinError) as ei:
        E.batch(jobs, prec="bf16", tile=14)
    assert ei.value.status in (E.E_INVAL,)
    bad = [(jobs[0][0], jobs[0][1], float("nan"))]
    with pytest.raises(E.EjoinError):
        E.batch(bad, prec="fp32")


def _graph_run(g, jobs, caps, stream):
    outs = [torch.empty((max(c, 1), 3), dtype=torch.int32, device="cuda") for c in caps]
    n_dev = torch.full((len(jobs),), -99, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    g.launch(jobs, outs, caps, n_dev, stream=stream)
    torch.cuda.synchronize()
    n = n_dev.cpu().tolist()
    res = []
    for o, c in zip(outs, n):
        assert 0 <= c
        t = o[:c].cpu()
        res.append(set(map(tuple, t[:, :2].tolist())))
    return n, res


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_graph_replays_match_eager(prec):
    """One captured graph replayed for three different batches (and the first
    again), with eager library work and synchronisations between replays;
    every replay equals the eager batch call."""
    hostA = _job_mix(seed=43)
    hostB = _job_mix(d=96, seed=47)[2:7]
    jobsA, jobsB = _to_dev(hostA), _to_dev(hostB)
    refA, _ = E.batch(jobsA, prec=prec)
    refB, _ = E.batch(jobsB, prec=prec)
    setA = [set(zip(r.r.cpu().tolist(), r.s.cpu().tolist())) for r in refA]
    setB = [set(zip(r.r.cpu().tolist(), r.s.cpu().tolist())) for r in refB]
    ws_bytes = max(E.batch_workspace(jobsA, prec=prec, band_capacity=1 << 20),
                   E.batch_workspace(jobsB, prec=prec, band_capacity=1 << 20))
    ws = torch.empty(ws_bytes + (1 << 16), dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()   # capture needs a stream other than the legacy default
    torch.cuda.synchronize()
    g = E.BatchGraph(len(jobsA), ws, prec=prec, band_capacity=1 << 20, stream=side)
    try:
        capsA = [len(r) + 8 for r in refA]
        capsB = [len(r) + 8 for r in refB]
        for jobs, caps, want in ((jobsA, capsA, setA), (jobsB, capsB, setB),
                                 (jobsA, capsA, setA)):
            n, got = _graph_run(g, jobs, caps, side)
            assert n == [len(w) for w in want]
            assert got == want
            # eager work on the same stream between replays
            E.batch(jobsB[:2], prec=prec)
            torch.cuda.synchronize()
    finally:
        g.close()


def test_autotune_records_and_tuner_roundtrip(tmp_path):
    host = _job_mix(seed=53)
    jobs = _to_dev(host)
    ref, _ = E.batch(jobs, prec="fp32")
    caps = [len(r) + 8 for r in ref]
    ws = torch.empty(E.batch_workspace(jobs, prec="fp32"), dtype=torch.uint8, device="cuda")
    outs = [torch.empty((c, 3), dtype=torch.int32, device="cuda") for c in caps]
    t = E.Tuner()
    best, ms = t.autotune(jobs, outs, caps, ws, prec="fp32", reps=2)
    assert best in (1, 2, 11, 18) and set(ms) == {1, 2, 11, 18}
    assert ms[best] == min(ms.values())
    pairs = sum(R.shape[0] * S.shape[0] for R, S, _ in jobs)
    assert t.lookup(True, "fp32", 96, pairs) == best
    p = tmp_path / "tune.txt"
    t.save(p)
    t2 = E.Tuner()
    t2.load(p)
    assert t2.lookup(True, "fp32", 96, pairs) == best
    res, st = E.batch(jobs, prec="fp32", tuner=t2)
    assert st["tile"] == best
    for (R, S, th), rr in zip(host, res):
        _check_job(R, S, th, rr, "fp32", st["band"])
    # single-join tuning includes the register-panel tiles
    R, S, th = host[0]
    one = [(jobs[0][0], jobs[0][1], th)]
    ws1 = torch.empty(E.threshold_workspace(jobs[0][0], jobs[0][1], prec="bf16"),
                      dtype=torch.uint8, device="cuda")
    out1 = [torch.empty((len(ref[0]) + 8, 3), dtype=torch.int32, device="cuda")]
    best1, ms1 = t.autotune(one, out1, [len(ref[0]) + 8], ws1, prec="bf16", reps=2)
    assert {12, 14, 16} <= set(ms1) and best1 in ms1
    got = E.threshold(jobs[0][0], jobs[0][1], th, prec="bf16", tuner=t)
    assert got.stats["tile"] == best1
