"""Python binding of libcompass.so (ctypes; argument marshalling only).

Every step of the hot path runs in the library's HIP kernels; this module
only turns torch tensors into device pointers, numpy seed arrays into host
pointers, and status codes into exceptions.  It fails loudly when the
library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcompass.so")

I32, F32, I64 = 0, 1, 2
PRED_KIND = {"point": 0, "range": 1, "subset": 2}
FLAG_EXACT = 1
FLAG_UNSUPPORTED = 2

STATUS = {0: "OK", 1: "E_ARG", 2: "E_RANGE", 3: "E_GRAPH", 4: "E_HIP",
          5: "E_UNSUPPORTED"}


class CompassError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Scalar(ctypes.Union):
    _fields_ = [("i", ctypes.c_int32), ("f", ctypes.c_float)]


class Pred(ctypes.Structure):
    _fields_ = [("col", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("lo", Scalar), ("hi", Scalar),
                ("bitmap", ctypes.c_void_p), ("domain", ctypes.c_int64)]


class SketchSpec(ctypes.Structure):
    _fields_ = [("key_col", ctypes.c_void_p), ("key_dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("seeds", ctypes.POINTER(ctypes.c_uint64)),
                ("counters", ctypes.c_void_p)]


class JoinGraph(ctypes.Structure):
    _fields_ = [("n_tables", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("d", ctypes.c_int32), ("w", ctypes.c_int32),
                ("counter_bits", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("edge_u", ctypes.POINTER(ctypes.c_int32)),
                ("edge_v", ctypes.POINTER(ctypes.c_int32)),
                ("n_selected", ctypes.c_void_p),
                ("sketch", ctypes.POINTER(ctypes.c_void_p))]


_lib = None


def lib():
    """The loaded library; raises if it was never built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libcompass.so is not built (run __graft_entry__.build() or "
                "python -m paper_2102_02440_amd.build); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.compass_sketch_build.argtypes = [
            ctypes.c_int64, ctypes.POINTER(vp), ctypes.c_int32,
            ctypes.POINTER(Pred), ctypes.c_int32, ctypes.POINTER(SketchSpec),
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_int32, vp, vp]
        L.compass_sketch_build.restype = ctypes.c_int32
        L.compass_estimate.argtypes = [
            ctypes.POINTER(JoinGraph), ctypes.POINTER(ctypes.c_uint64),
            ctypes.c_int32, vp, vp, vp, vp]
        L.compass_estimate.restype = ctypes.c_int32
        L.compass_release.argtypes = []
        L.compass_release.restype = ctypes.c_int32
        L.compass_last_error.argtypes = []
        L.compass_last_error.restype = ctypes.c_char_p
        L.compass_version.argtypes = []
        L.compass_version.restype = ctypes.c_char_p
        L.compass_profile_enable.argtypes = [ctypes.c_int32]
        L.compass_profile_enable.restype = ctypes.c_int32
        L.compass_profile_take.argtypes = [ctypes.c_char_p,
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_double)]
        L.compass_profile_take.restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise CompassError(status, lib().compass_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.int32:
        return I32
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.int64:
        return I64
    raise TypeError("unsupported dtype %s" % t.dtype)


def version() -> str:
    return lib().compass_version().decode()


def release():
    _check(lib().compass_release())


def profile_enable(on: bool = True):
    _check(lib().compass_profile_enable(1 if on else 0))


def profile_take(name: str):
    """(launch count, total ms) of kernel `name` since the last take."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(lib().compass_profile_take(name.encode(), ctypes.byref(n),
                                      ctypes.byref(ms)))
    return n.value, ms.value


# --------------------------------------------------------------------------
# compass_sketch_build
# --------------------------------------------------------------------------
def sketch_build(n_rows: int, pred_cols, preds, keys, seeds, counters,
                 n_selected: torch.Tensor, d: int, w: int,
                 counter_bits: int = 32, accumulate: bool = False,
                 stream=None):
    """One fused selection scan + sketch build (see include/compass.h).

    pred_cols: list of device column tensors; preds: list of dicts
    {col, kind, lo, hi, bitmap (device uint64 tensor), domain};
    keys/seeds/counters: one entry per sketch (device key tensor, (d, 6)
    uint64 numpy seeds, device (d, w) counter tensor).
    """
    ncol = len(pred_cols)
    cols = (ctypes.c_void_p * max(1, ncol))(*[c.data_ptr() for c in pred_cols])
    np_ = len(preds)
    parr = (Pred * max(1, np_))()
    for i, p in enumerate(preds):
        col = pred_cols[p["col"]]
        q = parr[i]
        q.col = p["col"]
        q.kind = PRED_KIND[p["kind"]]
        q.dtype = _dtype_code(col)
        if q.dtype == F32:
            q.lo.f = float(p.get("lo", 0))
            q.hi.f = float(p.get("hi", 0))
        else:
            q.lo.i = int(p.get("lo", 0))
            q.hi.i = int(p.get("hi", 0))
        bm = p.get("bitmap")
        q.bitmap = bm.data_ptr() if bm is not None else None
        q.domain = int(p.get("domain", 0))
    ns = len(keys)
    sarr = (SketchSpec * ns)()
    keep = []
    for i in range(ns):
        sd = np.ascontiguousarray(np.asarray(seeds[i], dtype=np.uint64).reshape(-1))
        keep.append(sd)
        sarr[i].key_col = keys[i].data_ptr()
        sarr[i].key_dtype = _dtype_code(keys[i])
        sarr[i].seeds = sd.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        sarr[i].counters = counters[i].data_ptr()
    _check(lib().compass_sketch_build(
        int(n_rows), cols, ncol, parr, np_, sarr, ns, int(d), int(w),
        int(counter_bits), 1 if accumulate else 0,
        ctypes.c_void_p(n_selected.data_ptr()), _stream(stream)))


# --------------------------------------------------------------------------
# compass_estimate
# --------------------------------------------------------------------------
def estimate(n_tables: int, edge_u, edge_v, d: int, w: int, counter_bits: int,
             n_selected: torch.Tensor, sketches, masks, row_est=None,
             est=None, flags=None, stream=None):
    """Estimates every sub-plan mask; returns (row_est, est, flags) device
    tensors: row_est int64 (n, d, 2) = (lo, hi) of the 128-bit row values."""
    ne = len(edge_u)
    eu = (ctypes.c_int32 * max(1, ne))(*[int(x) for x in edge_u])
    ev = (ctypes.c_int32 * max(1, ne))(*[int(x) for x in edge_v])
    sk = (ctypes.c_void_p * max(1, 2 * ne))(*[s.data_ptr() for s in sketches])
    g = JoinGraph(int(n_tables), ne, int(d), int(w), int(counter_bits), 0,
                  eu, ev, n_selected.data_ptr(), sk)
    ms = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    n = ms.size
    dev = n_selected.device
    if row_est is None:
        row_est = torch.empty((n, d, 2), dtype=torch.int64, device=dev)
    if est is None:
        est = torch.empty(n, dtype=torch.float64, device=dev)
    if flags is None:
        flags = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib().compass_estimate(
        ctypes.byref(g), ms.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
        n, ctypes.c_void_p(row_est.data_ptr() if row_est is not None else 0),
        ctypes.c_void_p(est.data_ptr()), ctypes.c_void_p(flags.data_ptr()),
        _stream(stream)))
    return row_est, est, flags


def row_values(row_est: torch.Tensor):
    """Unsigned 128-bit Python ints (value mod 2^128) of the (n, d, 2)
    int64 (lo, hi) pairs."""
    a = row_est.cpu().numpy().astype(np.int64)
    out = []
    for m in range(a.shape[0]):
        r = []
        for i in range(a.shape[1]):
            lo = int(a[m, i, 0]) & ((1 << 64) - 1)
            hi = int(a[m, i, 1]) & ((1 << 64) - 1)
            r.append((hi << 64) | lo)
        out.append(r)
    return out


# --------------------------------------------------------------------------
# A query resident on the device: tables, predicates, sketches
# --------------------------------------------------------------------------
class DeviceQuery:
    """Uploads a workloads.Query to device memory once and runs the hot path
    on it: one fused build per table (all its attribute sketches in one
    scan), then the estimates of any set of sub-plans."""

    def __init__(self, q, device="cuda"):
        self.q = q
        self.device = device
        self.d, self.w, self.bits = q.d, q.w, q.counter_bits
        cdt = torch.int32 if self.bits == 32 else torch.int64
        self.tables = []
        self.sketch_of_side = [None] * (2 * len(q.edges))
        for t, tb in enumerate(q.tables):
            cols = {c: torch.from_numpy(np.ascontiguousarray(v)).to(device)
                    for c, v in tb.cols.items()}
            pred_names = []
            preds = []
            for p in tb.preds:
                if p.col not in pred_names:
                    pred_names.append(p.col)
                pd = {"col": pred_names.index(p.col), "kind": p.kind,
                      "lo": p.lo, "hi": p.hi, "domain": p.domain}
                if p.kind == "subset":
                    pd["bitmap"] = torch.from_numpy(
                        np.asarray(p.bitmap, dtype=np.uint64).view(np.int64)).to(device)
                preds.append(pd)
            inc = q.incident(t)
            keys, seeds, counters = [], [], []
            for (e, side, col) in inc:
                c = torch.zeros((self.d, self.w), dtype=cdt, device=device)
                keys.append(cols[col])
                seeds.append(q.seeds[e])
                counters.append(c)
                self.sketch_of_side[2 * e + side] = c
            self.tables.append({
                "n": tb.n_rows, "cols": cols,
                "pred_cols": [cols[c] for c in pred_names], "preds": preds,
                "keys": keys, "seeds": seeds, "counters": counters})
        self.n_selected = torch.zeros(len(q.tables), dtype=torch.int64,
                                      device=device)

    def build(self, stream=None):
        for t, tb in enumerate(self.tables):
            if not tb["keys"]:
                continue
            sketch_build(tb["n"], tb["pred_cols"], tb["preds"], tb["keys"],
                         tb["seeds"], tb["counters"], self.n_selected[t:t + 1],
                         self.d, self.w, self.bits, stream=stream)

    def estimate(self, masks, stream=None):
        return estimate(len(self.q.tables), self.q.edge_u, self.q.edge_v,
                        self.d, self.w, self.bits, self.n_selected,
                        self.sketch_of_side, masks, stream=stream)
