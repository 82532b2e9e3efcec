"""The allocation-free threshold join (ejoin_threshold_noalloc) against the
workspace entry point it is a variant of: same pair set, same scores, same
counts, on two calls in a row (the second on a smaller input, so stale
contents of the shared scratch array would show), and the size limit
refused with EJOIN_E_WORKSPACE."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _sorted_pairs(out, n):
    a = out[:n].cpu().numpy()
    r, s = a[:, 0].astype(np.int64), a[:, 1].astype(np.int64)
    sc = a[:, 2].view(np.float32)
    o = np.lexsort((s, r))
    return r[o], s[o], sc[o]


def _both(E, Rd, Sd, theta, d, prec):
    cap = 1 << 20
    out_a = torch.empty((cap, 3), dtype=torch.int32, device="cuda")
    out_b = torch.full((cap, 3), -7, dtype=torch.int32, device="cuda")
    # FP8's band is wide: room for every within-cluster pair of the word data
    bc = 1 << 20
    ws = torch.empty(E.threshold_workspace(Rd, Sd, d=d, prec=prec, band_capacity=bc),
                     dtype=torch.uint8, device="cuda")
    rc_a, n_a, st_a = E.threshold_raw(Rd, Sd, theta, out_a, cap, ws, d=d, prec=prec,
                                      band_capacity=bc)
    rc_b, n_b, st_b = E.threshold_noalloc_raw(Rd, Sd, theta, out_b, cap, d=d, prec=prec,
                                              band_capacity=bc)
    assert rc_a == E.OK and rc_b == E.OK, (rc_a, rc_b)
    assert n_a == n_b and st_a["n_band"] == st_b["n_band"]
    ra, sa, ca = _sorted_pairs(out_a, n_a)
    rb, sb, cb = _sorted_pairs(out_b, n_b)
    assert np.array_equal(ra, rb) and np.array_equal(sa, sb)
    assert np.array_equal(ca, cb)
    return n_b


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_noalloc_equals_workspace_call_twice(prec):
    from oracle import oracle as O
    from paper_2312_01476_amd import datagen as G
    from paper_2312_01476_amd import ejoin as E
    w = G.WORKLOADS["words_1k"]
    R, S, _, _ = G.make_host(w, n_r=3000, n_s=2500)
    # first call: 3000 x 2500; second call: a smaller, ragged input
    for nr, ns in ((3000, 2500), (517, 389)):
        Rd = torch.from_numpy(R[:nr]).cuda()
        Sd = torch.from_numpy(S[:ns]).cuda()
        n = _both(E, Rd, Sd, w.theta, w.d, prec)
        ri, si, _, _ = O.threshold(R[:nr], S[:ns], w.theta, d=w.d)
        assert n == len(ri)


def test_noalloc_self_join_and_size_limit():
    from paper_2312_01476_amd import datagen as G
    from paper_2312_01476_amd import ejoin as E
    w = G.WORKLOADS["words_1k"]
    R, _, _, _ = G.make_host(w, n_r=1000, n_s=1)
    Rd = torch.from_numpy(R).cuda()
    _both(E, Rd, Rd, 0.8, w.d, "bf16")
    # a join whose workspace exceeds the scratch array is refused
    big = torch.zeros((60000, 320), dtype=torch.float32, device="cuda")
    need = E.threshold_workspace(big, big[:1], d=300)
    assert need > E.noalloc_scratch_bytes()
    out = torch.empty((16, 3), dtype=torch.int32, device="cuda")
    rc, n, st = E.threshold_noalloc_raw(big, big[:1], 0.5, out, 16, d=300)
    assert rc == E.E_WORKSPACE and st["ws_needed"] == need
