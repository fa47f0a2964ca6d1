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
# COMPASS_LIB selects another build of the same library (a sanitizer build)
LIB_PATH = os.environ.get("COMPASS_LIB") or os.path.join(_PKG, "libcompass.so")

I32, F32, I64 = 0, 1, 2
PRED_KIND = {"point": 0, "range": 1, "subset": 2}
FLAG_EXACT = 1
FLAG_UNSUPPORTED = 2
FLAG_APPROX = 4

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


class TensorGraph(ctypes.Structure):
    _fields_ = [("n_tables", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("d", ctypes.c_int32), ("counter_bits", ctypes.c_int32),
                ("edge_u", ctypes.POINTER(ctypes.c_int32)),
                ("edge_v", ctypes.POINTER(ctypes.c_int32)),
                ("width", ctypes.POINTER(ctypes.c_int32)),
                ("tensor", ctypes.POINTER(ctypes.c_void_p)),
                ("n_selected", ctypes.c_void_p)]


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
        L.compass_sketch_build_noalloc.argtypes = L.compass_sketch_build.argtypes
        L.compass_sketch_build_noalloc.restype = ctypes.c_int32
        L.compass_estimate.argtypes = [
            ctypes.POINTER(JoinGraph), ctypes.POINTER(ctypes.c_uint64),
            ctypes.c_int32, vp, vp, vp, vp]
        L.compass_estimate.restype = ctypes.c_int32
        L.compass_profile_select.argtypes = [ctypes.c_char_p]
        L.compass_profile_select.restype = ctypes.c_int32
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
        L.compass_sketch_build_2d.argtypes = [
            ctypes.c_int64, ctypes.POINTER(vp), ctypes.c_int32,
            ctypes.POINTER(Pred), ctypes.c_int32, ctypes.POINTER(SketchSpec),
            ctypes.POINTER(SketchSpec), ctypes.c_int32, ctypes.c_int32,
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.compass_sketch_build_2d.restype = ctypes.c_int32
        L.compass_sketch_build_kd.argtypes = [
            ctypes.c_int64, ctypes.POINTER(vp), ctypes.c_int32,
            ctypes.POINTER(Pred), ctypes.c_int32, ctypes.POINTER(SketchSpec),
            ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
            ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.compass_sketch_build_kd.restype = ctypes.c_int32
        L.compass_estimate_partitioned.argtypes = [
            ctypes.POINTER(TensorGraph), vp, vp, vp, vp]
        L.compass_estimate_partitioned.restype = ctypes.c_int32
        L.compass_estimate_chain3.argtypes = [
            vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp]
        L.compass_estimate_chain3.restype = ctypes.c_int32
        L.compass_sketch_build_select.argtypes = [
            ctypes.c_int64, ctypes.POINTER(vp), ctypes.c_int32,
            ctypes.POINTER(Pred), ctypes.c_int32, ctypes.POINTER(SketchSpec),
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_int32, vp, vp, ctypes.c_int64, vp, ctypes.c_int64, vp]
        L.compass_sketch_build_select.restype = ctypes.c_int32
        L.compass_agms_build.argtypes = [
            ctypes.c_int64, ctypes.POINTER(vp), ctypes.c_int32,
            ctypes.POINTER(Pred), ctypes.c_int32, ctypes.POINTER(SketchSpec),
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.compass_agms_build.restype = ctypes.c_int32
        L.compass_agms_estimate.argtypes = [
            ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32,
            ctypes.c_int32, vp, vp, vp, vp]
        L.compass_agms_estimate.restype = ctypes.c_int32
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


def profile_select(names=None):
    """Records only the kernels named (a list of names; None: every kernel)."""
    arg = None if not names else ",".join(names).encode()
    _check(lib().compass_profile_select(arg))


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
                 stream=None, noalloc: bool = False):
    """One fused selection scan + sketch build (see include/compass.h).

    pred_cols: list of device column tensors; preds: list of dicts
    {col, kind, lo, hi, bitmap (device uint64 tensor), domain};
    keys/seeds/counters: one entry per sketch (device key tensor, (d, 6)
    uint64 numpy seeds, device (d, w) counter tensor).  noalloc: call
    compass_sketch_build_noalloc (fixed scratch region, allocates nothing).
    """
    cols, ncol, parr, np_ = _marshal_preds(pred_cols, preds)
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
    fn = lib().compass_sketch_build_noalloc if noalloc else lib().compass_sketch_build
    _check(fn(int(n_rows), cols, ncol, parr, np_, sarr, ns, int(d), int(w),
              int(counter_bits), 1 if accumulate else 0,
              ctypes.c_void_p(n_selected.data_ptr()), _stream(stream)))


def sketch_build_select(n_rows: int, pred_cols, preds, keys, seeds, counters,
                        n_selected: torch.Tensor, d: int, w: int, rows_out,
                        rows_count: torch.Tensor, row_base: int = 0,
                        counter_bits: int = 32, accumulate: bool = False,
                        stream=None):
    """sketch_build that also writes the qualifying row indices (plus
    row_base) to rows_out (device int64, its length is the capacity) and
    counts them in rows_count (device int64)."""
    cols, ncol, parr, np_ = _marshal_preds(pred_cols, preds)
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
    cap = rows_out.numel() if rows_out is not None else 0
    _check(lib().compass_sketch_build_select(
        int(n_rows), cols, ncol, parr, np_, sarr, ns, int(d), int(w),
        int(counter_bits), 1 if accumulate else 0,
        ctypes.c_void_p(n_selected.data_ptr()),
        ctypes.c_void_p(rows_out.data_ptr() if cap else 0), int(cap),
        ctypes.c_void_p(rows_count.data_ptr()), int(row_base), _stream(stream)))


def _marshal_preds(pred_cols, preds):
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
    return cols, ncol, parr, np_


def sketch_build_2d(n_rows: int, pred_cols, preds, key1, seeds1, key2, seeds2,
                    counters, n_selected: torch.Tensor, d: int, w1: int, w2: int,
                    counter_bits: int = 32, accumulate: bool = False,
                    stream=None):
    """Partitioned sketch of one table over two join keys (device
    (d, w1, w2) counters); see compass_sketch_build_2d."""
    cols, ncol, parr, np_ = _marshal_preds(pred_cols, preds)
    specs = []
    keep = []
    for k, sd in ((key1, seeds1), (key2, seeds2)):
        a = np.ascontiguousarray(np.asarray(sd, dtype=np.uint64).reshape(-1))
        keep.append(a)
        sp = SketchSpec()
        sp.key_col = k.data_ptr()
        sp.key_dtype = _dtype_code(k)
        sp.seeds = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        sp.counters = None
        specs.append(sp)
    _check(lib().compass_sketch_build_2d(
        int(n_rows), cols, ncol, parr, np_, ctypes.byref(specs[0]),
        ctypes.byref(specs[1]), int(d), int(w1), int(w2), int(counter_bits),
        1 if accumulate else 0, ctypes.c_void_p(counters.data_ptr()),
        ctypes.c_void_p(n_selected.data_ptr()), _stream(stream)))


def sketch_build_kd(n_rows: int, pred_cols, preds, keys, seeds, counters,
                    n_selected: torch.Tensor, d: int, widths,
                    counter_bits: int = 32, accumulate: bool = False,
                    stream=None):
    """Partitioned sketch of one table over k = 2 .. 4 join keys (device
    (d, w_1, .., w_k) counters); see compass_sketch_build_kd."""
    cols, ncol, parr, np_ = _marshal_preds(pred_cols, preds)
    k = len(keys)
    specs = (SketchSpec * k)()
    keep = []
    for m in range(k):
        a = np.ascontiguousarray(np.asarray(seeds[m], dtype=np.uint64).reshape(-1))
        keep.append(a)
        specs[m].key_col = keys[m].data_ptr()
        specs[m].key_dtype = _dtype_code(keys[m])
        specs[m].seeds = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        specs[m].counters = None
    w = (ctypes.c_int32 * k)(*[int(x) for x in widths])
    _check(lib().compass_sketch_build_kd(
        int(n_rows), cols, ncol, parr, np_, specs, k, int(d), w, int(counter_bits),
        1 if accumulate else 0, ctypes.c_void_p(counters.data_ptr()),
        ctypes.c_void_p(n_selected.data_ptr()), _stream(stream)))


def estimate_partitioned(edge_u, edge_v, d: int, widths, tensors,
                         n_selected: torch.Tensor, counter_bits: int = 32,
                         stream=None):
    """Join size estimate of a tree of tables from partitioned sketches
    (tensors[t]: device counters with one dimension per incident edge, in
    increasing edge id).  Returns (row_est (d, 2) int64, est, flag) device
    tensors."""
    nt = len(tensors)
    ne = len(edge_u)
    eu = (ctypes.c_int32 * max(1, ne))(*[int(x) for x in edge_u])
    ev = (ctypes.c_int32 * max(1, ne))(*[int(x) for x in edge_v])
    wd = (ctypes.c_int32 * max(1, ne))(*[int(x) for x in widths])
    tp = (ctypes.c_void_p * nt)(*[t.data_ptr() for t in tensors])
    g = TensorGraph(nt, ne, int(d), int(counter_bits), eu, ev, wd, tp,
                    n_selected.data_ptr())
    dev = n_selected.device
    row_est = torch.empty((d, 2), dtype=torch.int64, device=dev)
    est = torch.empty(1, dtype=torch.float64, device=dev)
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().compass_estimate_partitioned(
        ctypes.byref(g), ctypes.c_void_p(row_est.data_ptr()),
        ctypes.c_void_p(est.data_ptr()), ctypes.c_void_p(flag.data_ptr()),
        _stream(stream)))
    return row_est, est, flag


def agms_build(n_rows: int, pred_cols, preds, keys, seeds, counters,
               n_selected: torch.Tensor, r: int, b: int, accumulate: bool = False,
               stream=None):
    """AGMS sketch (Section 4.1) of one table: keys/seeds one entry per join
    (device key tensor, (r*b, 6) uint64 seeds); counters device (r, b) int64."""
    cols, ncol, parr, np_ = _marshal_preds(pred_cols, preds)
    nj = len(keys)
    sarr = (SketchSpec * nj)()
    keep = []
    for e in range(nj):
        a = np.ascontiguousarray(np.asarray(seeds[e], dtype=np.uint64).reshape(-1))
        keep.append(a)
        sarr[e].key_col = keys[e].data_ptr()
        sarr[e].key_dtype = _dtype_code(keys[e])
        sarr[e].seeds = a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        sarr[e].counters = None
    _check(lib().compass_agms_build(
        int(n_rows), cols, ncol, parr, np_, sarr, nj, int(r), int(b),
        1 if accumulate else 0, ctypes.c_void_p(counters.data_ptr()),
        ctypes.c_void_p(n_selected.data_ptr()), _stream(stream)))


def agms_estimate(sketches, n_selected, stream=None):
    """AGMS estimate from the tables' (r, b) int64 sketches and their device
    selected counts; returns device (row_sums (r, 2) int64, est (1,), flag (1,))."""
    r, b = sketches[0].shape
    nt = len(sketches)
    dev = sketches[0].device
    sk = (ctypes.c_void_p * nt)(*[x.data_ptr() for x in sketches])
    ns = (ctypes.c_void_p * nt)(*[x.data_ptr() for x in n_selected])
    rows = torch.empty((r, 2), dtype=torch.int64, device=dev)
    est = torch.empty(1, dtype=torch.float64, device=dev)
    flag = torch.empty(1, dtype=torch.int32, device=dev)
    vp = ctypes.c_void_p
    _check(lib().compass_agms_estimate(sk, ns, nt, int(r), int(b), vp(rows.data_ptr()),
                                       vp(est.data_ptr()), vp(flag.data_ptr()),
                                       _stream(stream)))
    return rows, est, flag


def estimate_chain3(a, p, b, n_a, n_p, n_b, counter_bits: int = 32,
                    stream=None):
    """Three-table chain estimate from sketches a (d, w1), p (d, w1, w2)
    and b (d, w2); n_* are device int64 scalars.  Returns device tensors
    (row_est (d, 2) int64 = lo, hi; est (1,) float64; flags (1,) int32)."""
    d, w1, w2 = p.shape
    dev = p.device
    row_est = torch.empty((d, 2), dtype=torch.int64, device=dev)
    est = torch.empty(1, dtype=torch.float64, device=dev)
    flags = torch.empty(1, dtype=torch.int32, device=dev)
    vp = ctypes.c_void_p
    _check(lib().compass_estimate_chain3(
        vp(a.data_ptr()), vp(p.data_ptr()), vp(b.data_ptr()),
        int(counter_bits), int(d), int(w1), int(w2), vp(n_a.data_ptr()),
        vp(n_p.data_ptr()), vp(n_b.data_ptr()), vp(row_est.data_ptr()),
        vp(est.data_ptr()), vp(flags.data_ptr()), _stream(stream)))
    return row_est, est, flags


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

    def _build_table(self, t, stream):
        tb = self.tables[t]
        sketch_build(tb["n"], tb["pred_cols"], tb["preds"], tb["keys"],
                     tb["seeds"], tb["counters"], self.n_selected[t:t + 1],
                     self.d, self.w, self.bits, stream=stream)

    def build(self, stream=None, overlap=True):
        """Builds every table's sketches on `stream` (the current stream
        by default); the work is complete on that stream when it returns.

        overlap: tables with predicates (compaction, then hashing of the
        survivors: short launches bound by their latency) are built on a
        second stream of the device while the tables without predicates
        (one fused scan each, bound by the hashing) run on `stream`; the
        tables share no buffers and the library keeps its scratch per
        stream.  `stream` then waits for the second stream."""
        todo = [t for t, tb in enumerate(self.tables) if tb["keys"]]
        main = stream if stream is not None else torch.cuda.current_stream()
        side_tabs = [t for t in todo if self.tables[t]["preds"]]
        if not overlap or not side_tabs or len(side_tabs) == len(todo):
            for t in todo:
                self._build_table(t, main)
            return
        if getattr(self, "_side", None) is None:
            self._side = torch.cuda.Stream(device=main.device)  # default priority
        side = self._side
        side.wait_stream(main)
        for t in side_tabs:
            self._build_table(t, side)
        for t in todo:
            if t not in side_tabs:
                self._build_table(t, main)
        main.wait_stream(side)

    def estimate(self, masks, stream=None):
        return estimate(len(self.q.tables), self.q.edge_u, self.q.edge_v,
                        self.d, self.w, self.bits, self.n_selected,
                        self.sketch_of_side, masks, stream=stream)


# --------------------------------------------------------------------------
# Batched build (one persistent graph-captured launch for many tables)
# --------------------------------------------------------------------------
class BuildJob(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("pred_cols", ctypes.POINTER(ctypes.c_void_p)),
                ("n_pred_cols", ctypes.c_int32), ("n_preds", ctypes.c_int32),
                ("preds", ctypes.POINTER(Pred)), ("sketches", ctypes.POINTER(SketchSpec)),
                ("n_sketches", ctypes.c_int32), ("d", ctypes.c_int32),
                ("w", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("n_selected", ctypes.c_void_p)]


class Tune(ctypes.Structure):
    _fields_ = [("rows_per_item", ctypes.c_int64), ("lds_budget", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32)]


def _bind_batch(L):
    if getattr(L, "_batch_bound", False):
        return
    vp = ctypes.c_void_p
    L.compass_batch_plan_create.argtypes = [ctypes.POINTER(BuildJob), ctypes.c_int32,
                                            ctypes.c_int32, ctypes.POINTER(Tune), vp,
                                            ctypes.POINTER(vp)]
    L.compass_batch_plan_create.restype = ctypes.c_int32
    L.compass_batch_plan_launch.argtypes = [vp, vp]
    L.compass_batch_plan_launch.restype = ctypes.c_int32
    L.compass_batch_plan_info.argtypes = [vp, ctypes.POINTER(Tune),
                                          ctypes.POINTER(ctypes.c_int32),
                                          ctypes.POINTER(ctypes.c_int32)]
    L.compass_batch_plan_info.restype = ctypes.c_int32
    L.compass_batch_plan_destroy.argtypes = [vp]
    L.compass_batch_plan_destroy.restype = ctypes.c_int32
    L._batch_bound = True


def _marshal_build(n_rows, pred_cols, preds, keys, seeds, counters):
    """ctypes arrays for one table build; returns (arrays, keepalive)."""
    ncol = len(pred_cols)
    cols = (ctypes.c_void_p * max(1, ncol))(*[c.data_ptr() for c in pred_cols])
    parr = (Pred * max(1, len(preds)))()
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
    sarr = (SketchSpec * len(keys))()
    keep = [cols, parr, sarr]
    for i in range(len(keys)):
        sd = np.ascontiguousarray(np.asarray(seeds[i], dtype=np.uint64).reshape(-1))
        keep.append(sd)
        sarr[i].key_col = keys[i].data_ptr()
        sarr[i].key_dtype = _dtype_code(keys[i])
        sarr[i].seeds = sd.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
        sarr[i].counters = counters[i].data_ptr()
    return cols, parr, sarr, keep


class BatchPlan:
    """A graph-captured persistent build of many tables' sketches.

    jobs: list of dicts with the arguments of sketch_build (n_rows,
    pred_cols, preds, keys, seeds, counters, n_selected, d, w).  tune: None
    (autotune, cached) or (rows_per_item, lds_budget, blocks_per_cu)."""

    def __init__(self, jobs, counter_bits=32, tune=None, stream=None):
        L = lib()
        _bind_batch(L)
        self._keep = []
        arr = (BuildJob * max(1, len(jobs)))()
        for i, j in enumerate(jobs):
            cols, parr, sarr, keep = _marshal_build(j["n_rows"], j["pred_cols"],
                                                    j["preds"], j["keys"], j["seeds"],
                                                    j["counters"])
            self._keep.append(keep)
            b = arr[i]
            b.n_rows = int(j["n_rows"])
            b.pred_cols = cols
            b.n_pred_cols = len(j["pred_cols"])
            b.n_preds = len(j["preds"])
            b.preds = parr
            b.sketches = sarr
            b.n_sketches = len(j["keys"])
            b.d = int(j["d"])
            b.w = int(j["w"])
            b.n_selected = j["n_selected"].data_ptr()
        t = None
        if tune is not None:
            t = Tune(int(tune[0]), int(tune[1]), int(tune[2]))
        h = ctypes.c_void_p()
        _check(L.compass_batch_plan_create(arr, len(jobs), int(counter_bits),
                                           ctypes.byref(t) if t is not None else None,
                                           _stream(stream), ctypes.byref(h)))
        self.h = h
        self._keep.append(arr)

    def launch(self, stream=None):
        _check(lib().compass_batch_plan_launch(self.h, _stream(stream)))

    def info(self):
        t = Tune()
        n = ctypes.c_int32()
        g = ctypes.c_int32()
        _check(lib().compass_batch_plan_info(self.h, ctypes.byref(t), ctypes.byref(n),
                                             ctypes.byref(g)))
        return {"rows_per_item": t.rows_per_item, "lds_budget": t.lds_budget,
                "blocks_per_cu": t.blocks_per_cu, "n_items": n.value, "grid": g.value}

    def close(self):
        if self.h:
            lib().compass_batch_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def upload_pool(pool, device="cuda"):
    """Device copies of every column of a table pool."""
    return [{c: torch.from_numpy(np.ascontiguousarray(v)).to(device)
             for c, v in pt.cols.items()} for pt in pool]


class DeviceBatch:
    """A pool of tables resident on the device and a batch of queries over
    it: per (query, table) one build job with the query's selections and
    one sketch per incident edge (d, w and seeds of the query)."""

    def __init__(self, pool, queries, device="cuda", counter_bits=32,
                 pool_cols=None):
        self.pool, self.queries, self.device = pool, queries, device
        self.bits = counter_bits
        cdt = torch.int32 if counter_bits == 32 else torch.int64
        self.cols = pool_cols if pool_cols is not None else upload_pool(pool, device)
        self.jobs = []
        self.sides = []       # per query: list of counters per side (2 * n_edges)
        self.n_selected = []  # per query: int64 tensor (n_tables,)
        for qi, pq in enumerate(queries):
            nsel = torch.zeros(len(pq.tables), dtype=torch.int64, device=device)
            sides = [None] * (2 * len(pq.edges))
            for t, ptab in enumerate(pq.tables):
                cols = self.cols[ptab]
                inc = pq.incident(t)
                if not inc:
                    continue
                names, preds = [], []
                for p in pq.preds[t]:
                    if p.col not in names:
                        names.append(p.col)
                    pd = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo,
                          "hi": p.hi, "domain": p.domain}
                    if p.kind == "subset":
                        pd["bitmap"] = torch.from_numpy(
                            np.asarray(p.bitmap, dtype=np.uint64).view(np.int64)).to(device)
                    preds.append(pd)
                keys, seeds, counters = [], [], []
                for (e, side, c) in inc:
                    cnt = torch.zeros((pq.d, pq.w), dtype=cdt, device=device)
                    sides[2 * e + side] = cnt
                    keys.append(cols[c])
                    seeds.append(pq.seeds[e])
                    counters.append(cnt)
                self.jobs.append({"n_rows": len(cols["id"]),
                                  "pred_cols": [cols[c] for c in names],
                                  "preds": preds, "keys": keys, "seeds": seeds,
                                  "counters": counters,
                                  "n_selected": nsel[t:t + 1], "d": pq.d, "w": pq.w,
                                  "query": qi, "table": t})
            self.sides.append(sides)
            self.n_selected.append(nsel)

    def plan(self, tune=None, stream=None):
        return BatchPlan(self.jobs, self.bits, tune=tune, stream=stream)

    def build_per_table(self, stream=None):
        """One compass_sketch_build per (query, table): all its sketches."""
        for j in self.jobs:
            sketch_build(j["n_rows"], j["pred_cols"], j["preds"], j["keys"],
                         j["seeds"], j["counters"], j["n_selected"], j["d"],
                         j["w"], self.bits, stream=stream)

    def build_per_sketch(self, stream=None):
        """The plain path: one compass_sketch_build launch per sketch."""
        for j in self.jobs:
            for k in range(len(j["keys"])):
                sketch_build(j["n_rows"], j["pred_cols"], j["preds"], [j["keys"][k]],
                             [j["seeds"][k]], [j["counters"][k]], j["n_selected"],
                             j["d"], j["w"], self.bits, stream=stream)

    def estimate(self, qi, masks, stream=None):
        pq = self.queries[qi]
        return estimate(len(pq.tables), [e.u for e in pq.edges],
                        [e.v for e in pq.edges], pq.d, pq.w, self.bits,
                        self.n_selected[qi], self.sides[qi], masks, stream=stream)


# --------------------------------------------------------------------------
# Learned correction network
# --------------------------------------------------------------------------
def _bind_mlp(L):
    if getattr(L, "_mlp_bound", False):
        return
    vp = ctypes.c_void_p
    fp = ctypes.POINTER(ctypes.c_float)
    L.compass_mlp_create.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                     fp, ctypes.POINTER(vp)]
    L.compass_mlp_create.restype = ctypes.c_int32
    L.compass_mlp_n_params.argtypes = [vp]
    L.compass_mlp_n_params.restype = ctypes.c_int64
    L.compass_mlp_adam_steps.argtypes = [vp]
    L.compass_mlp_adam_steps.restype = ctypes.c_int64
    L.compass_mlp_forward.argtypes = [vp, vp, vp, ctypes.c_int32, vp, vp]
    L.compass_mlp_forward.restype = ctypes.c_int32
    L.compass_mlp_train_step.argtypes = [vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float,
                                         vp, vp]
    L.compass_mlp_train_step.restype = ctypes.c_int32
    L.compass_mlp_train_epoch.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_float, vp, vp]
    L.compass_mlp_train_epoch.restype = ctypes.c_int32
    L.compass_mlp_read.argtypes = [vp, ctypes.c_int32, fp]
    L.compass_mlp_read.restype = ctypes.c_int32
    L.compass_mlp_write.argtypes = [vp, fp, fp, fp, ctypes.c_int64]
    L.compass_mlp_write.restype = ctypes.c_int32
    L.compass_mlp_destroy.argtypes = [vp]
    L.compass_mlp_destroy.restype = ctypes.c_int32
    L.compass_mlp_features.argtypes = [vp, ctypes.c_int32, vp, vp, vp, ctypes.c_int32,
                                       ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp,
                                       vp]
    L.compass_mlp_features.restype = ctypes.c_int32
    L._mlp_bound = True


def mlp_n_params(n_in=20, hidden=64, layers=3):
    dims = [n_in] + [hidden] * layers + [1]
    return sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(len(dims) - 1))


class MLP:
    """The learned correction network on the device (fp32 master weights,
    bfloat16 copy, Adam state), driven by the library's HIP kernels."""

    def __init__(self, init_params, n_in=20, hidden=64, layers=3):
        L = lib()
        _bind_mlp(L)
        p = np.ascontiguousarray(np.asarray(init_params, dtype=np.float32))
        assert p.size == mlp_n_params(n_in, hidden, layers)
        h = ctypes.c_void_p()
        _check(L.compass_mlp_create(n_in, hidden, layers,
                                    p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    ctypes.byref(h)))
        self.h = h
        self.n_in = n_in
        self.hidden = hidden
        self.layers = layers
        self.n_params = int(L.compass_mlp_n_params(h))
        self._loss = None

    def forward(self, x, base, out=None, stream=None):
        n = x.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(lib().compass_mlp_forward(self.h, x.data_ptr(), base.data_ptr(), n,
                                         out.data_ptr(), _stream(stream)))
        return out

    def train_step(self, x, base, target, lr, stream=None):
        """One Adam step; returns the device scalar holding the batch MSE."""
        if self._loss is None or self._loss.device != x.device:
            self._loss = torch.zeros(1, dtype=torch.float32, device=x.device)
        _check(lib().compass_mlp_train_step(self.h, x.data_ptr(), base.data_ptr(),
                                            target.data_ptr(), x.shape[0],
                                            float(lr), self._loss.data_ptr(),
                                            _stream(stream)))
        return self._loss

    def train_epoch(self, x, base, target, idx, batch, lr, stream=None):
        """Adam steps on the batches idx[k * batch:(k + 1) * batch] (device
        int32 row indices); returns the device tensor of the batches' MSEs."""
        assert idx.dtype == torch.int32 and idx.is_contiguous()
        nb = idx.numel() // batch
        losses = torch.empty(max(1, nb), dtype=torch.float32, device=x.device)
        _check(lib().compass_mlp_train_epoch(self.h, x.data_ptr(), base.data_ptr(),
                                             target.data_ptr(), idx.data_ptr(), nb,
                                             int(batch), float(lr), losses.data_ptr(),
                                             _stream(stream)))
        return losses[:nb]

    def read(self, what=0):
        out = np.empty(self.n_params, dtype=np.float32)
        _check(lib().compass_mlp_read(self.h, int(what),
                                      out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return out

    def write(self, params, m=None, v=None, step=0):
        fp = ctypes.POINTER(ctypes.c_float)
        arrs = [None if a is None else np.ascontiguousarray(np.asarray(a, np.float32))
                for a in (params, m, v)]
        ptrs = [None if a is None else a.ctypes.data_as(fp) for a in arrs]
        _check(lib().compass_mlp_write(self.h, ptrs[0], ptrs[1], ptrs[2], int(step)))

    def adam_steps(self):
        return int(lib().compass_mlp_adam_steps(self.h))

    def save(self, path):
        """Checkpoint: parameters, Adam moments and step count (npz)."""
        np.savez(path, params=self.read(0), adam_m=self.read(2), adam_v=self.read(3),
                 step=np.int64(self.adam_steps()), n_in=np.int32(self.n_in),
                 hidden=np.int32(self.hidden), layers=np.int32(self.layers))

    @classmethod
    def load(cls, path):
        """A network restored from save(): the same parameters and Adam
        state, so training continues exactly where it stopped."""
        z = np.load(path)
        m = cls(z["params"], int(z["n_in"]), int(z["hidden"]), int(z["layers"]))
        m.write(z["params"], z["adam_m"], z["adam_v"], int(z["step"]))
        return m

    def close(self):
        if self.h:
            lib().compass_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def features(row_est, est, masks_dev, n_selected, n_tables, edge_u, edge_v,
             stream=None):
    """(x n x 20, base n) device float32 features of n sub-plans of one
    query (join graph edge_u/edge_v; the kernel computes every feature)."""
    L = lib()
    _bind_mlp(L)
    n, d = row_est.shape[0], row_est.shape[1]
    dev = row_est.device
    x = torch.empty((n, 20), dtype=torch.float32, device=dev)
    base = torch.empty(n, dtype=torch.float32, device=dev)
    eu = np.ascontiguousarray(np.asarray(edge_u, dtype=np.int32))
    ev = np.ascontiguousarray(np.asarray(edge_v, dtype=np.int32))
    _check(L.compass_mlp_features(row_est.data_ptr(), d, est.data_ptr(),
                                  masks_dev.data_ptr(), n_selected.data_ptr(),
                                  int(n_tables), int(eu.size), eu.ctypes.data,
                                  ev.ctypes.data, n, x.data_ptr(), base.data_ptr(),
                                  _stream(stream)))
    return x, base


def enumerate_plan(n_tables, edge_u, edge_v, masks, est, card, max_plans=10,
                   alpha=0.5, beta=0.5):
    """Algorithm 1 join-order search over host estimates; returns (order,
    cost, complete plans reached)."""
    L = lib()
    if not getattr(L, "_enum_bound", False):
        vp = ctypes.c_void_p
        L.compass_enumerate.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp,
                                        ctypes.c_int32, vp, ctypes.c_int32,
                                        ctypes.c_double, ctypes.c_double, vp, vp, vp]
        L.compass_enumerate.restype = ctypes.c_int32
        L._enum_bound = True
    ne = len(edge_u)
    eu = np.ascontiguousarray(np.asarray(edge_u, dtype=np.int32))
    ev = np.ascontiguousarray(np.asarray(edge_v, dtype=np.int32))
    ms = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    es = np.ascontiguousarray(np.asarray(est, dtype=np.float64))
    cd = np.ascontiguousarray(np.asarray(card, dtype=np.float64))
    order = np.zeros(n_tables, dtype=np.int32)
    cost = np.zeros(1, dtype=np.float64)
    npl = np.zeros(1, dtype=np.int64)
    _check(L.compass_enumerate(int(n_tables), ne, eu.ctypes.data, ev.ctypes.data,
                               ms.ctypes.data, es.ctypes.data, int(ms.size),
                               cd.ctypes.data, int(max_plans), float(alpha),
                               float(beta), order.ctypes.data, cost.ctypes.data,
                               npl.ctypes.data))
    return order.tolist(), float(cost[0]), int(npl[0])


def enumerate_greedy(n_tables, edge_u, edge_v, masks, est, card):
    """The greedy variant (one source: the smaller table of the two-table
    sub-plan with the smallest estimate); returns (order, cost)."""
    L = lib()
    if not getattr(L, "_greedy_bound", False):
        vp = ctypes.c_void_p
        L.compass_enumerate_greedy.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp,
                                               vp, vp, ctypes.c_int32, vp, vp, vp]
        L.compass_enumerate_greedy.restype = ctypes.c_int32
        L._greedy_bound = True
    ne = len(edge_u)
    eu = np.ascontiguousarray(np.asarray(edge_u, dtype=np.int32))
    ev = np.ascontiguousarray(np.asarray(edge_v, dtype=np.int32))
    ms = np.ascontiguousarray(np.asarray(masks, dtype=np.uint64))
    es = np.ascontiguousarray(np.asarray(est, dtype=np.float64))
    cd = np.ascontiguousarray(np.asarray(card, dtype=np.float64))
    order = np.zeros(n_tables, dtype=np.int32)
    cost = np.zeros(1, dtype=np.float64)
    _check(L.compass_enumerate_greedy(int(n_tables), ne, eu.ctypes.data, ev.ctypes.data,
                                      ms.ctypes.data, es.ctypes.data, int(ms.size),
                                      cd.ctypes.data, order.ctypes.data,
                                      cost.ctypes.data))
    return order.tolist(), float(cost[0])


# The four search spaces of the paper's plan-enumeration experiment
# (Section 7.2.8): name -> max_plans of Algorithm 1 (greedy: one source).
ENUM_VARIANTS = (("greedy", None), ("full-greedy", 1), ("limit-10", 10),
                 ("exhaustive", 0))


def enumerate_variant(name, n_tables, edge_u, edge_v, masks, est, card):
    """(order, estimated cost) of one of ENUM_VARIANTS."""
    mp = dict(ENUM_VARIANTS)[name]
    if mp is None:
        return enumerate_greedy(n_tables, edge_u, edge_v, masks, est, card)
    order, cost, _ = enumerate_plan(n_tables, edge_u, edge_v, masks, est, card,
                                    max_plans=mp)
    return order, cost
