"""Python binding of ``libejoin.so`` (argument marshalling only).

Every step of the join runs in the library's HIP kernels; this module only
allocates device buffers through PyTorch, passes raw pointers and the current
HIP stream across the C ABI (``include/ejoin.h``) and turns status codes into
exceptions.  There is no CPU fallback: if the library is missing or fails to
load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libejoin.so")

OK, E_INVAL, E_OVERFLOW, E_WORKSPACE, E_NONFINITE, E_HIP, E_UNSUPPORTED, E_RANGE = range(8)
PREC = {"fp32": 0, "bf16": 1, "fp8": 2, "fp8_e4m3": 2}
NO_SYNC = 0x1
TIMING = 0x2
APPROX_PREFILTER = 0x4
TOPK_MIN_SIM = 0x8
EXACT_PRUNE = 0x10
FP64_SCORES = 0x20


class Rel(C.Structure):
    _fields_ = [("data", C.c_void_p), ("rows", C.c_int64), ("dim", C.c_int32), ("ld", C.c_int64)]


class Opts(C.Structure):
    _fields_ = [("prec", C.c_int32), ("tile", C.c_int32), ("band", C.c_double),
                ("band_capacity", C.c_int64), ("flags", C.c_uint32), ("topk_cand", C.c_int32),
                ("tuner", C.c_void_p), ("prefilter", C.c_void_p), ("prefilter_eps", C.c_float),
                ("topk_min_sim", C.c_double)]


class Sel(C.Structure):
    _fields_ = [("ids", C.c_void_p), ("n", C.c_int64)]


class Job(C.Structure):
    _fields_ = [("R", Rel), ("S", Rel), ("theta", C.c_double), ("out", C.c_void_p),
                ("capacity", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("n_pairs", C.c_int64), ("n_certain", C.c_int64), ("n_band", C.c_int64),
                ("n_band_accepted", C.c_int64), ("band_needed", C.c_int64),
                ("ws_needed", C.c_size_t), ("band", C.c_double), ("tile", C.c_int32),
                ("n_fallback", C.c_int32), ("ms_prep", C.c_float), ("ms_main", C.c_float),
                ("ms_rescore", C.c_float), ("ms_total", C.c_float),
                ("topk_floor", C.c_double), ("topk_slots", C.c_int32),
                ("tiles_total", C.c_int64), ("tiles_kept", C.c_int64),
                ("topk_refined", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class EjoinError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().ejoin_strerror(status).decode()
        super().__init__(f"{where}: {msg} (status {status})")


_lib = None


def lib():
    """Load libejoin.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2312_01476_amd.build` (no fallback exists)")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.ejoin_version.restype = C.c_char_p
        L.ejoin_strerror.restype = C.c_char_p
        L.ejoin_strerror.argtypes = [C.c_int]
        L.ejoin_opts_default.argtypes = [P(Opts)]
        L.ejoin_opts_default.restype = None
        L.ejoin_band_default.restype = C.c_double
        L.ejoin_band_default.argtypes = [C.c_int32, C.c_int32]
        L.ejoin_tile_count.restype = C.c_int32
        L.ejoin_tile_name.restype = C.c_char_p
        L.ejoin_tile_name.argtypes = [C.c_int32]
        L.ejoin_tile_occupancy.restype = C.c_int
        L.ejoin_tile_occupancy.argtypes = [C.c_int32, C.c_int32, P(C.c_int32), P(C.c_int32)]
        L.ejoin_threshold_workspace.restype = C.c_size_t
        L.ejoin_threshold_workspace.argtypes = [P(Rel), P(Rel), P(Opts)]
        L.ejoin_threshold.restype = C.c_int
        L.ejoin_threshold.argtypes = [P(Rel), P(Rel), C.c_double, P(Opts), C.c_void_p,
                                      C.c_int64, P(C.c_int64), C.c_void_p, C.c_size_t,
                                      C.c_void_p, P(Stats)]
        L.ejoin_threshold_noalloc.restype = C.c_int
        L.ejoin_threshold_noalloc.argtypes = [P(Rel), P(Rel), C.c_double, P(Opts), C.c_void_p,
                                              C.c_int64, P(C.c_int64), C.c_void_p, P(Stats)]
        L.ejoin_noalloc_scratch_bytes.restype = C.c_size_t
        L.ejoin_noalloc_scratch_bytes.argtypes = []
        L.ejoin_select_workspace.restype = C.c_size_t
        L.ejoin_select_workspace.argtypes = []
        L.ejoin_select_range.restype = C.c_int
        L.ejoin_select_range.argtypes = [C.c_void_p, C.c_int64, C.c_float, C.c_float, C.c_void_p,
                                         C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
        L.ejoin_threshold_sel_workspace.restype = C.c_size_t
        L.ejoin_threshold_sel_workspace.argtypes = [P(Rel), P(Sel), P(Rel), P(Sel), P(Opts)]
        L.ejoin_threshold_sel.restype = C.c_int
        L.ejoin_threshold_sel.argtypes = [P(Rel), P(Sel), P(Rel), P(Sel), C.c_double, P(Opts),
                                          C.c_void_p, C.c_int64, P(C.c_int64), C.c_void_p,
                                          C.c_size_t, C.c_void_p, P(Stats)]
        L.ejoin_topk_sel_workspace.restype = C.c_size_t
        L.ejoin_topk_sel_workspace.argtypes = [P(Rel), P(Sel), P(Rel), P(Sel), C.c_int32,
                                               P(Opts)]
        L.ejoin_topk_sel.restype = C.c_int
        L.ejoin_topk_sel.argtypes = [P(Rel), P(Sel), P(Rel), P(Sel), C.c_int32, P(Opts),
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                                     P(Stats)]
        L.ejoin_topk_workspace.restype = C.c_size_t
        L.ejoin_topk_workspace.argtypes = [P(Rel), P(Rel), C.c_int32, P(Opts)]
        L.ejoin_topk.restype = C.c_int
        L.ejoin_topk.argtypes = [P(Rel), P(Rel), C.c_int32, P(Opts), C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_size_t, C.c_void_p, P(Stats)]
        L.ejoin_batch_workspace.restype = C.c_size_t
        L.ejoin_batch_workspace.argtypes = [P(Job), C.c_int32, P(Opts)]
        L.ejoin_batch.restype = C.c_int
        L.ejoin_batch.argtypes = [P(Job), C.c_int32, P(Opts), C.c_void_p, C.c_void_p,
                                  C.c_size_t, C.c_void_p, P(Stats)]
        L.ejoin_batch_graph_create.restype = C.c_int
        L.ejoin_batch_graph_create.argtypes = [C.c_int32, P(Opts), C.c_void_p, C.c_size_t,
                                               C.c_void_p, P(C.c_void_p)]
        L.ejoin_batch_graph_launch.restype = C.c_int
        L.ejoin_batch_graph_launch.argtypes = [C.c_void_p, P(Job), C.c_int32, C.c_void_p,
                                               C.c_void_p]
        L.ejoin_batch_graph_destroy.restype = C.c_int
        L.ejoin_batch_graph_destroy.argtypes = [C.c_void_p]
        L.ejoin_tuner_create.restype = C.c_void_p
        L.ejoin_tuner_create.argtypes = []
        L.ejoin_tuner_destroy.restype = None
        L.ejoin_tuner_destroy.argtypes = [C.c_void_p]
        L.ejoin_tuner_lookup.restype = C.c_int32
        L.ejoin_tuner_lookup.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double]
        L.ejoin_tuner_save.restype = C.c_int
        L.ejoin_tuner_save.argtypes = [C.c_void_p, C.c_char_p]
        L.ejoin_tuner_load.restype = C.c_int
        L.ejoin_tuner_load.argtypes = [C.c_void_p, C.c_char_p]
        L.ejoin_autotune.restype = C.c_int
        L.ejoin_autotune.argtypes = [C.c_void_p, P(Job), C.c_int32, P(Opts), C.c_void_p,
                                     C.c_size_t, C.c_void_p, C.c_int32, P(C.c_int32),
                                     P(C.c_float)]
        _lib = L
    return _lib


def version() -> str:
    return lib().ejoin_version().decode()


def band_default(prec: str, dim: int) -> float:
    return float(lib().ejoin_band_default(PREC[prec], int(dim)))


def tiles():
    L = lib()
    return {i: L.ejoin_tile_name(i).decode() for i in range(1, L.ejoin_tile_count() + 1)}


def tile_occupancy(tile: int, dim: int):
    """(designed, resident) workgroups per CU of the panel kernel of `tile`
    for rows of `dim` elements (ejoin_tile_occupancy); None if the tile does
    not take that depth."""
    d, r = C.c_int32(0), C.c_int32(0)
    rc = lib().ejoin_tile_occupancy(int(tile), int(dim), C.byref(d), C.byref(r))
    if rc == E_INVAL:
        return None
    if rc != OK:
        raise EjoinError(rc, "ejoin_tile_occupancy")
    return d.value, r.value


def _rel(X, d):
    import torch
    if not isinstance(X, torch.Tensor) or X.device.type != "cuda":
        raise TypeError("relations must be CUDA (HIP) tensors")
    if X.dtype != torch.float32 or X.dim() != 2:
        raise TypeError("relations must be float32 2-D tensors")
    n, ld = X.shape
    if n > 0 and ld > 1 and X.stride(1) != 1:
        raise TypeError("relations must have unit column stride")
    dim = ld if d is None else int(d)
    return Rel(X.data_ptr() if n > 0 else 0, n, dim, X.stride(0) if n > 1 else max(ld, dim))


def _opts(prec, band, tile, band_capacity, flags, topk_cand=0, tuner=None, prefilter=None,
          eps=0.0, min_sim=None):
    o = Opts()
    lib().ejoin_opts_default(C.byref(o))
    o.prec = PREC[prec]
    o.tile = int(tile)
    o.band = -1.0 if band is None else float(band)
    o.band_capacity = int(band_capacity)
    o.flags = int(flags)
    o.topk_cand = int(topk_cand)
    o.tuner = tuner.handle if tuner is not None else None
    if prefilter is not None:
        o.flags |= APPROX_PREFILTER
        o.prefilter = prefilter.state.data_ptr()
        o.prefilter_eps = float(eps)
    if min_sim is not None:
        o.flags |= TOPK_MIN_SIM
        o.topk_min_sim = float(min_sim)
    return o


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


@dataclass
class Pairs:
    """Result of a threshold join: int32 offsets and float32 scores (device)."""
    r: "object"
    s: "object"
    score: "object"
    stats: dict

    def __len__(self):
        return int(self.r.shape[0])


def threshold_workspace(R, S, *, d=None, prec="fp32", band=None, tile=0, band_capacity=0,
                        tuner=None):
    r, s = _rel(R, d), _rel(S, d)
    o = _opts(prec, band, tile, band_capacity, 0, tuner=tuner)
    n = lib().ejoin_threshold_workspace(C.byref(r), C.byref(s), C.byref(o))
    if n == 0:
        raise EjoinError(E_INVAL, "ejoin_threshold_workspace")
    return int(n)


def threshold_raw(R, S, theta, out, capacity, ws, *, d=None, prec="fp32", band=None, tile=0,
                  band_capacity=0, flags=0, stream=None, n_out_dev=None, tuner=None):
    """One ejoin_threshold call on caller-provided buffers (``out``: int32
    tensor (capacity, 3); ``ws``: uint8 tensor).  Returns (status, n_out,
    stats dict).  With NO_SYNC, ``n_out_dev`` (int64 device tensor) receives
    the count."""
    r, s = _rel(R, d), _rel(S, d)
    o = _opts(prec, band, tile, band_capacity, flags, tuner=tuner)
    st = Stats()
    n = C.c_int64(0)
    if flags & NO_SYNC:
        nptr = C.cast(C.c_void_p(n_out_dev.data_ptr()), C.POINTER(C.c_int64))
    else:
        nptr = C.byref(n)
    rc = lib().ejoin_threshold(C.byref(r), C.byref(s), float(theta), C.byref(o),
                               C.c_void_p(out.data_ptr() if capacity > 0 else 0),
                               int(capacity), nptr, C.c_void_p(ws.data_ptr()),
                               int(ws.numel()), _stream(stream), C.byref(st))
    return rc, int(n.value), st.as_dict()


def threshold_noalloc_raw(R, S, theta, out, capacity, *, d=None, prec="fp32", band=None, tile=0,
                          band_capacity=0, flags=0, stream=None, n_out_dev=None):
    """One ejoin_threshold_noalloc call (no workspace: the library's own
    scratch array).  Returns (status, n_out, stats dict)."""
    r, s = _rel(R, d), _rel(S, d)
    o = _opts(prec, band, tile, band_capacity, flags)
    st = Stats()
    n = C.c_int64(0)
    if flags & NO_SYNC:
        nptr = C.cast(C.c_void_p(n_out_dev.data_ptr()), C.POINTER(C.c_int64))
    else:
        nptr = C.byref(n)
    rc = lib().ejoin_threshold_noalloc(C.byref(r), C.byref(s), float(theta), C.byref(o),
                                       C.c_void_p(out.data_ptr() if capacity > 0 else 0),
                                       int(capacity), nptr, _stream(stream), C.byref(st))
    return rc, int(n.value), st.as_dict()


def noalloc_scratch_bytes() -> int:
    return int(lib().ejoin_noalloc_scratch_bytes())


def threshold(R, S, theta: float, *, d=None, prec="fp32", band=None, tile=0, capacity=None,
              band_capacity=0, timing=False, stream=None, tuner=None,
              fp64_scores=False) -> Pairs:
    """Threshold E-join on the GPU: all (i, j) with sim64(R_i, S_j) >= theta.

    R, S: float32 CUDA tensors (n, ld) with unit column stride; ``d`` is the
    embedding dimension (default: all columns).  Grows the output and band
    buffers and retries when the library reports they were too small.
    ``fp64_scores``: every returned score is float(sim64) (EJOIN_FP64_SCORES)."""
    import torch
    dev = R.device
    nR, nS = R.shape[0], S.shape[0]
    if capacity is None:
        capacity = max(1 << 16, min(nR * nS, (nR + nS) * 64))
    flags = (TIMING if timing else 0) | (FP64_SCORES if fp64_scores else 0)
    for _ in range(4):
        ws_bytes = threshold_workspace(R, S, d=d, prec=prec, band=band, tile=tile,
                                       band_capacity=band_capacity, tuner=tuner)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        out = torch.empty((max(capacity, 1), 3), dtype=torch.int32, device=dev)
        rc, n, st = threshold_raw(R, S, theta, out, capacity, ws, d=d, prec=prec, band=band,
                                  tile=tile, band_capacity=band_capacity, flags=flags,
                                  stream=stream, tuner=tuner)
        if rc == OK:
            o = out[:n]
            return Pairs(o[:, 0], o[:, 1], o[:, 2].view(torch.float32), st)
        if rc == E_OVERFLOW:
            capacity = n
            continue
        if rc == E_WORKSPACE and st["band_needed"] > 0:
            band_capacity = int(st["band_needed"] * 1.25) + 1024
            continue
        raise EjoinError(rc, "ejoin_threshold")
    raise EjoinError(rc, "ejoin_threshold (retries exhausted)")


def topk_workspace(R, S, k, *, d=None, prec="bf16", topk_cand=0, tile=0, min_sim=None):
    r, s = _rel(R, d), _rel(S, d)
    o = _opts(prec, None, tile, 0, 0, topk_cand, min_sim=min_sim)
    n = lib().ejoin_topk_workspace(C.byref(r), C.byref(s), int(k), C.byref(o))
    if n == 0:
        raise EjoinError(E_INVAL, "ejoin_topk_workspace")
    return int(n)


def topk_raw(R, S, k, out_idx, out_score, ws, *, d=None, prec="bf16", topk_cand=0, flags=0,
             stream=None, tile=0, min_sim=None):
    """One ejoin_topk call on caller buffers.  Returns (status, stats dict)."""
    r, s = _rel(R, d), _rel(S, d)
    o = _opts(prec, None, tile, 0, flags, topk_cand, min_sim=min_sim)
    st = Stats()
    rc = lib().ejoin_topk(C.byref(r), C.byref(s), int(k), C.byref(o),
                          C.c_void_p(out_idx.data_ptr() if out_idx.numel() else 0),
                          C.c_void_p(out_score.data_ptr() if out_score.numel() else 0),
                          C.c_void_p(ws.data_ptr()), int(ws.numel()), _stream(stream),
                          C.byref(st))
    return rc, st.as_dict()


def topk(R, S, k: int, *, d=None, prec="bf16", topk_cand=0, timing=False, stream=None, tile=0,
         min_sim=None):
    """Top-k E-join on the GPU: per R row the k most similar S rows, ordered by
    (sim64 desc, index asc).  Returns (idx int32 (|R|, k), score float32
    (|R|, k), stats); empty slots hold (-1, -inf)."""
    import torch
    dev = R.device
    nR = R.shape[0]
    ws = torch.empty(topk_workspace(R, S, k, d=d, prec=prec, topk_cand=topk_cand, tile=tile,
                                    min_sim=min_sim), dtype=torch.uint8, device=dev)
    idx = torch.empty((nR, k), dtype=torch.int32, device=dev)
    sc = torch.empty((nR, k), dtype=torch.float32, device=dev)
    rc, st = topk_raw(R, S, k, idx, sc, ws, d=d, prec=prec, topk_cand=topk_cand,
                      flags=TIMING if timing else 0, stream=stream, tile=tile, min_sim=min_sim)
    if rc != OK:
        raise EjoinError(rc, "ejoin_topk")
    return idx, sc, st


# ---------------------------------------------------------------------------
# relational selections pushed below the join
# ---------------------------------------------------------------------------

def _sel(ids):
    """ids: None (every row) or an int32 CUDA tensor of ascending row ids."""
    import torch
    if ids is None:
        return None
    if not isinstance(ids, torch.Tensor) or ids.device.type != "cuda" or \
            ids.dtype != torch.int32 or ids.dim() != 1 or (ids.numel() > 1 and ids.stride(0) != 1):
        raise TypeError("a selection is a contiguous 1-D int32 CUDA tensor of row ids")
    return Sel(ids.data_ptr() if ids.numel() else None, ids.numel())


def _ref(x):
    return C.byref(x) if x is not None else None


def select_range(col, lo, hi, *, stream=None):
    """Row ids i (ascending) with lo <= col[i] < hi, computed on the device.
    Returns an int32 CUDA tensor."""
    import torch
    if col.dtype != torch.float32 or col.dim() != 1 or col.device.type != "cuda":
        raise TypeError("col must be a 1-D float32 CUDA tensor")
    col = col.contiguous()
    n = col.numel()
    ids = torch.empty(max(n, 1), dtype=torch.int32, device=col.device)
    n_sel = torch.zeros(1, dtype=torch.int64, device=col.device)
    ws = torch.empty(lib().ejoin_select_workspace(), dtype=torch.uint8, device=col.device)
    rc = lib().ejoin_select_range(C.c_void_p(col.data_ptr() if n else 0), n, float(lo),
                                  float(hi), C.c_void_p(ids.data_ptr()),
                                  C.c_void_p(n_sel.data_ptr()), C.c_void_p(ws.data_ptr()),
                                  ws.numel(), _stream(stream))
    if rc != OK:
        raise EjoinError(rc, "ejoin_select_range")
    return ids[:int(n_sel.item())]


def threshold_sel_raw(R, sel_r, S, sel_s, theta, out, capacity, ws, *, d=None, prec="fp32",
                      band=None, tile=0, band_capacity=0, flags=0, stream=None, n_out_dev=None):
    """One ejoin_threshold_sel call on caller buffers.  Returns (status,
    n_out, stats dict)."""
    r, s = _rel(R, d), _rel(S, d)
    a, b = _sel(sel_r), _sel(sel_s)
    o = _opts(prec, band, tile, band_capacity, flags)
    st = Stats()
    n = C.c_int64(0)
    if flags & NO_SYNC:
        nptr = C.cast(C.c_void_p(n_out_dev.data_ptr()), C.POINTER(C.c_int64))
    else:
        nptr = C.byref(n)
    rc = lib().ejoin_threshold_sel(C.byref(r), _ref(a), C.byref(s), _ref(b), float(theta),
                                   C.byref(o), C.c_void_p(out.data_ptr() if capacity > 0 else 0),
                                   int(capacity), nptr, C.c_void_p(ws.data_ptr()),
                                   int(ws.numel()), _stream(stream), C.byref(st))
    return rc, int(n.value), st.as_dict()


def threshold_sel_workspace(R, sel_r, S, sel_s, *, d=None, prec="fp32", band=None, tile=0,
                            band_capacity=0):
    r, s = _rel(R, d), _rel(S, d)
    a, b = _sel(sel_r), _sel(sel_s)
    o = _opts(prec, band, tile, band_capacity, 0)
    n = lib().ejoin_threshold_sel_workspace(C.byref(r), _ref(a), C.byref(s), _ref(b),
                                            C.byref(o))
    if n == 0:
        raise EjoinError(E_INVAL, "ejoin_threshold_sel_workspace")
    return int(n)


def threshold_sel(R, sel_r, S, sel_s, theta: float, *, d=None, prec="fp32", band=None, tile=0,
                  capacity=None, band_capacity=0, timing=False, stream=None,
                  fp64_scores=False) -> Pairs:
    """Threshold join restricted to the selected rows (row ids in the
    result); grows buffers and retries like ``threshold``."""
    import torch
    dev = R.device
    nR = R.shape[0] if sel_r is None else sel_r.numel()
    nS = S.shape[0] if sel_s is None else sel_s.numel()
    if capacity is None:
        capacity = max(1 << 16, min(nR * nS, (nR + nS) * 64))
    flags = (TIMING if timing else 0) | (FP64_SCORES if fp64_scores else 0)
    for _ in range(4):
        ws = torch.empty(threshold_sel_workspace(R, sel_r, S, sel_s, d=d, prec=prec, band=band,
                                                 tile=tile, band_capacity=band_capacity),
                         dtype=torch.uint8, device=dev)
        out = torch.empty((max(capacity, 1), 3), dtype=torch.int32, device=dev)
        rc, n, st = threshold_sel_raw(R, sel_r, S, sel_s, theta, out, capacity, ws, d=d,
                                      prec=prec, band=band, tile=tile,
                                      band_capacity=band_capacity, flags=flags, stream=stream)
        if rc == OK:
            o = out[:n]
            return Pairs(o[:, 0], o[:, 1], o[:, 2].view(torch.float32), st)
        if rc == E_OVERFLOW:
            capacity = n
            continue
        if rc == E_WORKSPACE and st["band_needed"] > 0:
            band_capacity = int(st["band_needed"] * 1.25) + 1024
            continue
        raise EjoinError(rc, "ejoin_threshold_sel")
    raise EjoinError(rc, "ejoin_threshold_sel (retries exhausted)")


def topk_sel(R, sel_r, S, sel_s, k: int, *, d=None, prec="bf16", topk_cand=0, timing=False,
             flags=0, stream=None, tile=0, min_sim=None):
    """Top-k over the selected rows: output row i is the i-th selected R row;
    indices are S row ids.  Returns (idx, score, stats)."""
    import torch
    dev = R.device
    r, s = _rel(R, d), _rel(S, d)
    a, b = _sel(sel_r), _sel(sel_s)
    o = _opts(prec, None, tile, 0, flags | (TIMING if timing else 0), topk_cand, min_sim=min_sim)
    L = lib()
    need = L.ejoin_topk_sel_workspace(C.byref(r), _ref(a), C.byref(s), _ref(b), int(k),
                                      C.byref(o))
    if need == 0:
        raise EjoinError(E_INVAL, "ejoin_topk_sel_workspace")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    nR = R.shape[0] if sel_r is None else sel_r.numel()
    idx = torch.empty((nR, k), dtype=torch.int32, device=dev)
    sc = torch.empty((nR, k), dtype=torch.float32, device=dev)
    st = Stats()
    rc = L.ejoin_topk_sel(C.byref(r), _ref(a), C.byref(s), _ref(b), int(k), C.byref(o),
                          C.c_void_p(idx.data_ptr() if idx.numel() else 0),
                          C.c_void_p(sc.data_ptr() if sc.numel() else 0),
                          C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream), C.byref(st))
    if rc != OK:
        raise EjoinError(rc, "ejoin_topk_sel")
    return idx, sc, st.as_dict()


# ---------------------------------------------------------------------------
# batched threshold joins
# ---------------------------------------------------------------------------

def _jobs(jobs, outs, caps, d):
    arr = (Job * max(1, len(jobs)))()
    for i, (R, S, theta) in enumerate(jobs):
        arr[i].R = _rel(R, d)
        arr[i].S = _rel(S, d)
        arr[i].theta = float(theta)
        arr[i].out = outs[i].data_ptr() if (outs is not None and caps[i] > 0) else None
        arr[i].capacity = int(caps[i]) if caps is not None else 0
    return arr


def batch_workspace(jobs, *, d=None, prec="fp32", band=None, tile=0, band_capacity=0,
                    tuner=None, prefilter=None, eps=0.0, flags=0):
    """Workspace bytes for ejoin_batch; ``jobs`` is a list of (R, S, theta)."""
    arr = _jobs(jobs, None, [0] * len(jobs), d)
    o = _opts(prec, band, tile, band_capacity, flags, tuner=tuner, prefilter=prefilter, eps=eps)
    n = lib().ejoin_batch_workspace(arr, len(jobs), C.byref(o))
    if n == 0:
        raise EjoinError(E_INVAL, "ejoin_batch_workspace")
    return int(n)


def batch_raw(jobs, outs, caps, ws, n_out, *, d=None, prec="fp32", band=None, tile=0,
              band_capacity=0, flags=0, stream=None, tuner=None, prefilter=None, eps=0.0):
    """One ejoin_batch call on caller buffers.  ``outs[i]``: int32 (cap_i, 3)
    tensors; ``n_out``: int64 CPU tensor (sync) or CUDA tensor (NO_SYNC).
    Returns (status, stats dict)."""
    arr = _jobs(jobs, outs, caps, d)
    o = _opts(prec, band, tile, band_capacity, flags, tuner=tuner, prefilter=prefilter, eps=eps)
    st = Stats()
    rc = lib().ejoin_batch(arr, len(jobs), C.byref(o), C.c_void_p(n_out.data_ptr()),
                           C.c_void_p(ws.data_ptr()), int(ws.numel()), _stream(stream),
                           C.byref(st))
    return rc, st.as_dict()


def batch(jobs, *, d=None, prec="fp32", band=None, tile=0, capacities=None, band_capacity=0,
          timing=False, stream=None, tuner=None, prefilter=None, eps=0.0, exact_prune=False,
          fp64_scores=False):
    """Run many threshold joins as one batch pass.  ``jobs``: list of
    (R, S, theta).  Returns (list of Pairs, stats dict).  Jobs whose output
    overflowed are run again (as a smaller batch) with exactly enough room."""
    import torch
    n = len(jobs)
    if n == 0:
        return [], {}
    dev = jobs[0][0].device
    caps = list(capacities) if capacities is not None else [
        max(1 << 16, min(R.shape[0] * S.shape[0], (R.shape[0] + S.shape[0]) * 64))
        for R, S, _ in jobs]
    results = [None] * n
    todo = list(range(n))
    stats = {}
    flags = (TIMING if timing else 0) | (EXACT_PRUNE if exact_prune else 0) | \
        (FP64_SCORES if fp64_scores else 0)
    for _ in range(6):
        sub = [jobs[i] for i in todo]
        sub_caps = [caps[i] for i in todo]
        ws = torch.empty(batch_workspace(sub, d=d, prec=prec, band=band, tile=tile,
                                         band_capacity=band_capacity, tuner=tuner,
                                         prefilter=prefilter, eps=eps,
                                         flags=flags & EXACT_PRUNE),
                         dtype=torch.uint8, device=dev)
        outs = [torch.empty((max(c, 1), 3), dtype=torch.int32, device=dev) for c in sub_caps]
        n_out = torch.zeros(len(sub), dtype=torch.int64)
        rc, st = batch_raw(sub, outs, sub_caps, ws, n_out, d=d, prec=prec, band=band, tile=tile,
                           band_capacity=band_capacity, flags=flags, stream=stream, tuner=tuner,
                           prefilter=prefilter, eps=eps)
        if not stats:
            stats = st
        if rc == E_WORKSPACE and st["band_needed"] > 0:
            band_capacity = int(st["band_needed"] * 1.25) + 1024
            continue
        if rc not in (OK, E_OVERFLOW):
            raise EjoinError(rc, "ejoin_batch")
        again = []
        for q, i in enumerate(todo):
            c = int(n_out[q])
            if c > sub_caps[q]:
                caps[i] = c
                again.append(i)
            else:
                o = outs[q][:c]
                results[i] = Pairs(o[:, 0], o[:, 1], o[:, 2].view(torch.float32), {})
        todo = again
        if not todo:
            return results, stats
    raise EjoinError(E_OVERFLOW, "ejoin_batch (retries exhausted)")


class BatchGraph:
    """A captured graph of the batch pass (ejoin_batch_graph_*), replayable
    for new batches of at most ``max_jobs`` jobs within the workspace ``ws``."""

    def __init__(self, max_jobs, ws, *, prec="fp32", band=None, tile=0, band_capacity=0,
                 stream=None):
        self.ws = ws
        self.handle = C.c_void_p()
        o = _opts(prec, band, tile, band_capacity, NO_SYNC)
        rc = lib().ejoin_batch_graph_create(int(max_jobs), C.byref(o), C.c_void_p(ws.data_ptr()),
                                            int(ws.numel()), _stream(stream),
                                            C.byref(self.handle))
        if rc != OK:
            raise EjoinError(rc, "ejoin_batch_graph_create")
        self.d = None

    def launch(self, jobs, outs, caps, n_out_dev, *, d=None, stream=None):
        arr = _jobs(jobs, outs, caps, d)
        rc = lib().ejoin_batch_graph_launch(self.handle, arr, len(jobs),
                                            C.c_void_p(n_out_dev.data_ptr()), _stream(stream))
        if rc != OK:
            raise EjoinError(rc, "ejoin_batch_graph_launch")

    def close(self):
        if self.handle:
            rc = lib().ejoin_batch_graph_destroy(self.handle)
            self.handle = C.c_void_p()
            if rc != OK:
                raise EjoinError(rc, "ejoin_batch_graph_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tuner:
    """Caller-owned table of measured tile choices (ejoin_tuner_*)."""

    def __init__(self):
        self.handle = lib().ejoin_tuner_create()
        if not self.handle:
            raise EjoinError(E_INVAL, "ejoin_tuner_create")

    def lookup(self, batch, prec, dim, pairs):
        return int(lib().ejoin_tuner_lookup(self.handle, int(bool(batch)), PREC[prec],
                                            int(dim), float(pairs)))

    def save(self, path):
        rc = lib().ejoin_tuner_save(self.handle, str(path).encode())
        if rc != OK:
            raise EjoinError(rc, "ejoin_tuner_save")

    def load(self, path):
        rc = lib().ejoin_tuner_load(self.handle, str(path).encode())
        if rc != OK:
            raise EjoinError(rc, "ejoin_tuner_load")

    def autotune(self, jobs, outs, caps, ws, *, d=None, prec="fp32", band=None,
                 band_capacity=0, reps=3, stream=None):
        """Time every tile that can run ``jobs`` and record the fastest.
        Returns (best tile id, {tile id: median ms})."""
        arr = _jobs(jobs, outs, caps, d)
        o = _opts(prec, band, 0, band_capacity, 0)
        best = C.c_int32(0)
        nt = lib().ejoin_tile_count()
        ms = (C.c_float * (nt + 1))()
        rc = lib().ejoin_autotune(self.handle, arr, len(jobs), C.byref(o),
                                  C.c_void_p(ws.data_ptr()), int(ws.numel()), _stream(stream),
                                  int(reps), C.byref(best), ms)
        if rc != OK:
            raise EjoinError(rc, "ejoin_autotune")
        return int(best.value), {i: float(ms[i]) for i in range(1, nt + 1) if ms[i] >= 0}

    def __del__(self):
        try:
            if self.handle:
                lib().ejoin_tuner_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


# ---------------------------------------------------------------------------
# prefilter network
# ---------------------------------------------------------------------------

MLP_HIDDEN, MLP_OUT = 256, 64
MLP_GRAD_ONLY = 0x1


class MlpLayout(C.Structure):
    _fields_ = [("dim", C.c_int32), ("dim_pad", C.c_int32), ("n_params", C.c_int64),
                ("off_params", C.c_size_t), ("off_grads", C.c_size_t), ("off_m", C.c_size_t),
                ("off_v", C.c_size_t), ("off_w1t", C.c_size_t), ("off_w2t", C.c_size_t),
                ("off_step", C.c_size_t), ("total", C.c_size_t)]


class MlpHparams(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("lambda_", C.c_float), ("theta_lo", C.c_float),
                ("flags", C.c_uint32)]


def _mlp_sigs(L):
    P = C.POINTER
    L.ejoin_mlp_layout_get.restype = C.c_int
    L.ejoin_mlp_layout_get.argtypes = [C.c_int32, P(MlpLayout)]
    L.ejoin_mlp_hparams_default.restype = None
    L.ejoin_mlp_hparams_default.argtypes = [P(MlpHparams)]
    L.ejoin_mlp_init.restype = C.c_int
    L.ejoin_mlp_init.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
    L.ejoin_mlp_train_workspace.restype = C.c_size_t
    L.ejoin_mlp_train_workspace.argtypes = [C.c_int32, C.c_int32]
    L.ejoin_mlp_train_step.restype = C.c_int
    L.ejoin_mlp_train_step.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_int64,
                                       C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                       P(MlpHparams), C.c_void_p, C.c_size_t, C.c_void_p,
                                       C.c_void_p]
    L.ejoin_mlp_forward_workspace.restype = C.c_size_t
    L.ejoin_mlp_forward_workspace.argtypes = [C.c_int32, C.c_int64]
    L.ejoin_mlp_forward.restype = C.c_int
    L.ejoin_mlp_forward.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                    C.c_void_p, C.c_size_t, C.c_void_p]


def _ckpt_sigs(L):
    if hasattr(L, "_ckpt_sigs"):
        return
    L.ejoin_prefilter_save.restype = C.c_int
    L.ejoin_prefilter_save.argtypes = [C.c_void_p, C.c_int32, C.c_float, C.c_uint64, C.c_char_p,
                                       C.c_void_p]
    L.ejoin_prefilter_load.restype = C.c_int
    L.ejoin_prefilter_load.argtypes = [C.c_void_p, C.c_int32, C.c_char_p,
                                       C.POINTER(C.c_float), C.POINTER(C.c_uint64), C.c_void_p]
    L._ckpt_sigs = True


def prefilter_save(net, path, *, eps=0.0, seed=0, stream=None):
    """Write the network's masters, Adam moments and step to a host file."""
    L = lib()
    _ckpt_sigs(L)
    rc = L.ejoin_prefilter_save(C.c_void_p(net.state.data_ptr()), net.dim, float(eps), int(seed),
                                str(path).encode(), _stream(stream))
    if rc != OK:
        raise EjoinError(rc, "ejoin_prefilter_save")


def prefilter_load(net, path, *, stream=None):
    """Restore a checkpoint into ``net`` (same dim).  Returns (eps, seed)."""
    L = lib()
    _ckpt_sigs(L)
    eps = C.c_float(0.0)
    seed = C.c_uint64(0)
    rc = L.ejoin_prefilter_load(C.c_void_p(net.state.data_ptr()) if net is not None else None,
                                net.dim if net is not None else 1, str(path).encode(),
                                C.byref(eps), C.byref(seed), _stream(stream))
    if rc != OK:
        raise EjoinError(rc, "ejoin_prefilter_load")
    return float(eps.value), int(seed.value)


def mlp_layout(dim):
    L = lib()
    if not hasattr(L, "_mlp_sigs"):
        _mlp_sigs(L)
        L._mlp_sigs = True
    lay = MlpLayout()
    rc = L.ejoin_mlp_layout_get(int(dim), C.byref(lay))
    if rc != OK:
        raise EjoinError(rc, "ejoin_mlp_layout_get")
    return lay


class Mlp:
    """The prefilter network's state block (one device tensor) and views of
    its regions.  ``params``: flat FP32 initial weights (W1 dim x 256, b1,
    W2 256 x 64, b2)."""

    def __init__(self, dim, params, stream=None):
        import torch
        self.dim = int(dim)
        self.lay = mlp_layout(dim)
        self.state = torch.zeros(self.lay.total, dtype=torch.uint8, device="cuda")
        p = params.to(device="cuda", dtype=torch.float32).contiguous()
        if p.numel() != self.lay.n_params:
            raise ValueError("params have the wrong size")
        rc = lib().ejoin_mlp_init(C.c_void_p(self.state.data_ptr()), self.dim,
                                  C.c_void_p(p.data_ptr()), _stream(stream))
        if rc != OK:
            raise EjoinError(rc, "ejoin_mlp_init")
        self._ws = None

    def _f32(self, off, n):
        return self.state[off:off + 4 * n].view(__import__("torch").float32)

    def params(self):
        return self._f32(self.lay.off_params, self.lay.n_params)

    def grads(self):
        return self._f32(self.lay.off_grads, self.lay.n_params)

    def moments(self):
        return (self._f32(self.lay.off_m, self.lay.n_params),
                self._f32(self.lay.off_v, self.lay.n_params))

    def split(self, flat):
        """Views W1, b1, W2, b2 of a flat parameter-shaped vector."""
        d, H, O = self.dim, MLP_HIDDEN, MLP_OUT
        a = d * H
        return {"W1": flat[:a].view(d, H), "b1": flat[a:a + H],
                "W2": flat[a + H:a + H + H * O].view(H, O), "b2": flat[a + H + H * O:]}

    def train_step(self, X, pr, ps, target, loss, *, hp=None, grad_only=False, stream=None):
        """One step on pairs (pr, ps) of the BF16 rows X with targets."""
        import torch
        L = lib()
        h = MlpHparams()
        L.ejoin_mlp_hparams_default(C.byref(h))
        for k, v in (hp or {}).items():
            setattr(h, "lambda_" if k == "lambda" else k, v)
        if grad_only:
            h.flags |= MLP_GRAD_ONLY
        B = int(pr.numel())
        need = L.ejoin_mlp_train_workspace(self.dim, B)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device="cuda")
        rc = L.ejoin_mlp_train_step(C.c_void_p(self.state.data_ptr()), self.dim,
                                    C.c_void_p(X.data_ptr()), X.stride(0), X.shape[0],
                                    C.c_void_p(pr.data_ptr()), C.c_void_p(ps.data_ptr()),
                                    C.c_void_p(target.data_ptr()), B, C.byref(h),
                                    C.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                    C.c_void_p(loss.data_ptr()), _stream(stream))
        if rc != OK:
            raise EjoinError(rc, "ejoin_mlp_train_step")

    def forward(self, X, n, U, stream=None):
        """Codes of the first n rows of X (dim_pad BF16 values per row,
        round_up(n, 128) rows) into U (n x 64 FP32)."""
        import torch
        L = lib()
        need = L.ejoin_mlp_forward_workspace(self.dim, int(n))
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
        rc = L.ejoin_mlp_forward(C.c_void_p(self.state.data_ptr()), self.dim,
                                 C.c_void_p(X.data_ptr()), int(n), C.c_void_p(U.data_ptr()),
                                 C.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream))
        if rc != OK:
            raise EjoinError(rc, "ejoin_mlp_forward")


class TrainOpts(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("seed", C.c_uint64),
                ("pos_frac", C.c_float), ("hp", MlpHparams)]


def prefilter_train(net, jobs, outs, caps, n_out, *, d=None, steps=300, batch=4096, seed=1,
                    pos_frac=0.5, hp=None, losses=True, stream=None):
    """Train ``net`` (an Mlp) on the batch ``jobs`` whose exact outputs are
    in ``outs`` (``n_out``: per-job counts).  Returns the per-step losses."""
    import torch
    L = lib()
    if not hasattr(L, "_pf_sigs"):
        P = C.POINTER
        L.ejoin_prefilter_train_opts_default.restype = None
        L.ejoin_prefilter_train_opts_default.argtypes = [P(TrainOpts)]
        L.ejoin_prefilter_train_workspace.restype = C.c_size_t
        L.ejoin_prefilter_train_workspace.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.ejoin_prefilter_train.restype = C.c_int
        L.ejoin_prefilter_train.argtypes = [C.c_void_p, P(Job), C.c_int32, P(C.c_int64),
                                            P(TrainOpts), C.c_void_p, C.c_size_t,
                                            P(C.c_float), C.c_void_p]
        L._pf_sigs = True
    arr = _jobs(jobs, outs, caps, d)
    to = TrainOpts()
    L.ejoin_prefilter_train_opts_default(C.byref(to))
    to.steps, to.batch, to.seed, to.pos_frac = int(steps), int(batch), int(seed), float(pos_frac)
    for k, v in (hp or {}).items():
        setattr(to.hp, "lambda_" if k == "lambda" else k, v)
    need = L.ejoin_prefilter_train_workspace(len(jobs), net.dim, int(batch))
    if need == 0:
        raise EjoinError(E_INVAL, "ejoin_prefilter_train_workspace")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    cnt = (C.c_int64 * len(jobs))(*[int(x) for x in n_out])
    ls = (C.c_float * max(1, int(steps)))() if losses else None
    rc = L.ejoin_prefilter_train(C.c_void_p(net.state.data_ptr()), arr, len(jobs), cnt,
                                 C.byref(to), C.c_void_p(ws.data_ptr()), ws.numel(),
                                 ls, _stream(stream))
    if rc != OK:
        raise EjoinError(rc, "ejoin_prefilter_train")
    return [float(x) for x in ls[:int(steps)]] if losses else None
