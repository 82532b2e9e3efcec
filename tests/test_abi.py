"""The C-ABI library builds for gfx950, loads on a host without a GPU and
exports every symbol that include/ejoin.h declares; host-only helpers behave
as documented (no device work is started here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ejoin.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ejoin_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("ejoin_threshold", "ejoin_threshold_workspace", "ejoin_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2312_01476_amd import ejoin as E
    L = E.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_helpers():
    from paper_2312_01476_amd import ejoin as E
    assert E.version().startswith("ejoin-gfx950")
    # rigorous bands grow with the dimension and with coarser formats
    assert 0 < E.band_default("fp32", 300) < 1e-4
    assert E.band_default("fp32", 300) < E.band_default("fp32", 768)
    assert 0.0078 < E.band_default("bf16", 384) < 1e-2   # 1e-2 (the bf16 workload's band) is admissible
    assert E.band_default("bf16", 384) < E.band_default("fp8", 768) < 0.2
    names = E.tiles()
    assert names[1].startswith("fp32:") and any(v.startswith("bf16:") for v in names.values())
    L = E.lib()
    assert L.ejoin_strerror(2).decode().startswith("output capacity")
    assert L.ejoin_tile_name(0).decode() == "auto"
    assert names[20] == "fp32:panel" and names[21] == "fp32:panel/2wg"
    assert names[19] == "bf16:panel/batch" and names[22] == "bf16:panel/batch/2wg"


def test_workspace_query_is_bounded_not_dense():
    """Section V.B: a 100k x 100k join would materialise ~40 GB of FP32
    similarities; the library's workspace holds only the padded operand
    copies, per-row data and the band list."""
    from paper_2312_01476_amd import ejoin as E
    L = E.lib()
    R = E.Rel(0x1000, 100_000, 300, 320)
    o = E._opts("fp32", None, 0, 0, 0)
    ws = L.ejoin_threshold_workspace(C.byref(R), C.byref(R), C.byref(o))
    assert 0 < ws < 0.01 * 100_000 * 100_000 * 4
    bad = E.Rel(0x1000, 10, 300, 200)     # ld < dim
    assert L.ejoin_threshold_workspace(C.byref(bad), C.byref(R), C.byref(o)) == 0


def _job(E, nr, ns, d=768, theta=0.8, cap=0, alias=False):
    j = E.Job()
    j.R = E.Rel(0x1000, nr, d, d)
    j.S = E.Rel(0x1000 if alias else 0x2000, ns, d, d)
    j.theta = theta
    j.out = 0x3000 if cap else None
    j.capacity = cap
    return j


def test_batch_workspace_query():
    """The batch workspace holds the prepared operands of every job, one
    counter block per job and the shared band list; never a dense block of
    similarities.  A self-join prepares its relation once."""
    from paper_2312_01476_amd import ejoin as E
    L = E.lib()
    arr = (E.Job * 3)(_job(E, 500_000, 100_000), _job(E, 1000, 1000), _job(E, 0, 50))
    o = E._opts("bf16", None, 0, 0, 0)
    ws = L.ejoin_batch_workspace(arr, 3, C.byref(o))
    ops = (500_096 + 100_096 + 1024 * 2) * 768 * 2
    assert ops < ws < ops * 1.2
    # aliasing: one copy of the relation
    a1 = (E.Job * 1)(_job(E, 10_000, 10_000, alias=True))
    a2 = (E.Job * 1)(_job(E, 10_000, 10_000))
    o.band_capacity = 1
    assert L.ejoin_batch_workspace(a1, 1, C.byref(o)) < L.ejoin_batch_workspace(a2, 1, C.byref(o))
    # invalid: theta not finite, capacity without buffer, panel tile, wrong-precision tile
    bad = (E.Job * 1)(_job(E, 10, 10, theta=float("nan")))
    assert L.ejoin_batch_workspace(bad, 1, C.byref(o)) == 0
    bad = (E.Job * 1)(_job(E, 10, 10))
    bad[0].capacity = 5
    assert L.ejoin_batch_workspace(bad, 1, C.byref(o)) == 0
    ok = (E.Job * 1)(_job(E, 10, 10))
    for tile in (14, 12, 1):
        ot = E._opts("bf16", None, tile, 0, 0)
        assert L.ejoin_batch_workspace(ok, 1, C.byref(ot)) == 0
    assert L.ejoin_batch_workspace(ok, 1, C.byref(E._opts("bf16", None, 8, 0, 0))) > 0
    # the batch panel form takes only depths it has a register panel for
    # (BF16 rows of 8, 9, 10 or 12 K slices); empty jobs do not count
    o19 = E._opts("bf16", None, 19, 0, 0)
    assert L.ejoin_batch_workspace(ok, 1, C.byref(o19)) > 0
    mixed = (E.Job * 3)(_job(E, 10, 10), _job(E, 10, 10, d=500), _job(E, 0, 10, d=96))
    assert L.ejoin_batch_workspace(mixed, 3, C.byref(o19)) > 0
    for d in (96, 384, 1024):
        assert L.ejoin_batch_workspace((E.Job * 1)(_job(E, 10, 10, d=d)), 1, C.byref(o19)) == 0
    assert L.ejoin_batch_workspace(ok, 1, C.byref(E._opts("fp32", None, 19, 0, 0))) == 0
    o22 = E._opts("bf16", None, 22, 0, 0)
    assert L.ejoin_batch_workspace(mixed, 3, C.byref(o22)) > 0
    assert L.ejoin_batch_workspace((E.Job * 1)(_job(E, 10, 10, d=96)), 1, C.byref(o22)) == 0
    # empty batch is valid
    assert L.ejoin_batch_workspace(ok, 0, C.byref(o)) > 0


def test_tuner_file_roundtrip_and_nearest_bucket(tmp_path):
    from paper_2312_01476_amd import ejoin as E
    p = tmp_path / "t.txt"
    # batch prec Kp bucket tile
    p.write_text("# hand-written\n1 1 768 17 4 bf16:256x128x64\n1 1 768 12 3 x\n"
                 "0 1 384 15 14 bf16:panel/2wg\n0 0 320 16 11 fp32:256x128x32\n")
    t = E.Tuner()
    t.load(p)
    assert t.lookup(True, "bf16", 768, 4.0 ** 17) == 4
    assert t.lookup(True, "bf16", 768, 4.0 ** 18 + 5) == 4      # nearest bucket
    assert t.lookup(True, "bf16", 768, 4.0 ** 12) == 3
    assert t.lookup(True, "bf16", 720, 4.0 ** 12) == 3          # same padded depth (768)
    assert t.lookup(True, "bf16", 700, 4.0 ** 12) == 0          # padded depth 704
    assert t.lookup(False, "bf16", 384, 1e9) == 14
    assert t.lookup(False, "fp32", 300, 1e10) == 11
    assert t.lookup(True, "fp8", 768, 1e10) == 0                 # nothing recorded
    q = tmp_path / "u.txt"
    t.save(q)
    t2 = E.Tuner()
    t2.load(q)
    for args in ((True, "bf16", 768, 4.0 ** 17), (False, "fp32", 300, 1e10)):
        assert t2.lookup(*args) == t.lookup(*args)
    # a panel tile has no batch form; a tile of another precision is rejected
    for line in ("1 1 384 15 14 x\n", "0 0 320 16 3 x\n", "garbage\n"):
        r = tmp_path / "bad.txt"
        r.write_text(line)
        with pytest.raises(E.EjoinError):
            E.Tuner().load(r)


def test_prefilter_load_refuses_bad_files_before_touching_the_device(tmp_path):
    """The checkpoint file is validated on the host: a missing file, a wrong
    magic, another dim or a truncated file are EJOIN_E_INVAL without any
    device call (the state pointer here is not device memory)."""
    import struct
    from paper_2312_01476_amd import ejoin as E
    L = E.lib()
    E._ckpt_sigs(L)
    fake = C.c_void_p(0x1000)
    n_params = 96 * 256 + 256 + 256 * 64 + 64

    def load(path, dim=96):
        return L.ejoin_prefilter_load(fake, dim, str(path).encode(), None, None, None)

    assert load(tmp_path / "missing") == E.E_INVAL
    head = lambda magic, dim, n: magic + struct.pack("<iiqqfIQ", dim, 0, n, 3, 0.05, 0, 7)
    body = b"\0" * (3 * n_params * 4)
    bad_magic = tmp_path / "m"
    bad_magic.write_bytes(head(b"EJPFNETX", 96, n_params) + body)
    other_dim = tmp_path / "d"
    other_dim.write_bytes(head(b"EJPFNET1", 128, 128 * 256 + 256 + 256 * 64 + 64) + body)
    short = tmp_path / "s"
    short.write_bytes(head(b"EJPFNET1", 96, n_params) + body[:-4])
    longer = tmp_path / "l"
    longer.write_bytes(head(b"EJPFNET1", 96, n_params) + body + b"\0")
    for p in (bad_magic, other_dim, short, longer):
        assert load(p) == E.E_INVAL, p
    assert L.ejoin_prefilter_load(fake, 2000, str(short).encode(), None, None, None) == E.E_INVAL
