"""The C ABI library loads and exports every declared entry point, and its
argument validation answers before any GPU work (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "compass.h")).read()
    return sorted(set(re.findall(r"\b(compass_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def C():
    from paper_2102_02440_amd import compass
    return compass


def test_exports_every_declared_symbol(C):
    names = declared_functions()
    assert "compass_sketch_build" in names and "compass_estimate" in names
    lib = ctypes.CDLL(C.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n


def test_version(C):
    assert C.version().startswith("compass-gfx950")


def _spec(C, d, seeds):
    s = (C.SketchSpec * 1)()
    arr = np.ascontiguousarray(seeds.reshape(-1).astype(np.uint64))
    s[0].key_col = 16
    s[0].key_dtype = C.I32
    s[0].seeds = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    s[0].counters = 32
    return s, arr


@pytest.mark.parametrize("kw,status", [
    (dict(d=0), 1), (dict(d=33), 1), (dict(w=0), 1), (dict(counter_bits=16), 1),
    (dict(n_rows=-1), 2), (dict(n_rows=2**31), 2), (dict(n_rows=2**47, counter_bits=64), 2),
    (dict(w=(1 << 20) + 1), 1), (dict(bad_seed=True), 1), (dict(n_sketches=0), 1),
])
def test_build_validation(C, kw, status):
    L = C.lib()
    d = kw.get("d", 3)
    seeds = np.zeros((max(d, 1), 6), np.uint64)
    if kw.get("bad_seed"):
        seeds[0, 2] = (1 << 61) - 1
    s, keep = _spec(C, d, seeds)
    r = L.compass_sketch_build(kw.get("n_rows", 10), None, 0, None, 0, s,
                               kw.get("n_sketches", 1), d, kw.get("w", 64),
                               kw.get("counter_bits", 32), 0,
                               ctypes.c_void_p(64), ctypes.c_void_p(0))
    assert r == status
    assert L.compass_last_error().decode() != ""


def test_estimate_rejects_disconnected(C):
    L = C.lib()
    eu = (ctypes.c_int32 * 1)(0)
    ev = (ctypes.c_int32 * 1)(1)
    sk = (ctypes.c_void_p * 2)(16, 32)
    g = C.JoinGraph(3, 1, 3, 64, 32, 0, eu, ev, 64, sk)
    masks = np.array([0b101], dtype=np.uint64)
    r = L.compass_estimate(ctypes.byref(g), masks.ctypes.data_as(
        ctypes.POINTER(ctypes.c_uint64)), 1, None, ctypes.c_void_p(8),
        ctypes.c_void_p(8), ctypes.c_void_p(0))
    assert r == 3
    assert "not connected" in L.compass_last_error().decode()
    masks = np.array([0b1000], dtype=np.uint64)
    r = L.compass_estimate(ctypes.byref(g), masks.ctypes.data_as(
        ctypes.POINTER(ctypes.c_uint64)), 1, None, ctypes.c_void_p(8),
        ctypes.c_void_p(8), ctypes.c_void_p(0))
    assert r == 3


@pytest.mark.parametrize("kw,status", [
    (dict(d=0), 1), (dict(d=25), 1), (dict(w1=0), 1), (dict(w2=0), 1),
    (dict(w1=1 << 15, w2=1 << 14), 1), (dict(counter_bits=8), 1),
    (dict(n_rows=-1), 2), (dict(n_rows=2**31), 2), (dict(bad_seed=True), 1),
    (dict(null_counters=True), 1),
])
def test_build_2d_validation(C, kw, status):
    L = C.lib()
    d = kw.get("d", 3)
    seeds = np.zeros((max(d, 1), 6), np.uint64)
    if kw.get("bad_seed"):
        seeds[-1, 5] = (1 << 61) + 7
    s1, k1 = _spec(C, d, seeds)
    s2, k2 = _spec(C, d, np.zeros((max(d, 1), 6), np.uint64))
    r = L.compass_sketch_build_2d(
        kw.get("n_rows", 10), None, 0, None, 0, s1, s2, d, kw.get("w1", 64),
        kw.get("w2", 32), kw.get("counter_bits", 32), 0,
        ctypes.c_void_p(0 if kw.get("null_counters") else 48),
        ctypes.c_void_p(64), ctypes.c_void_p(0))
    assert r == status
    assert L.compass_last_error().decode() != ""


@pytest.mark.parametrize("kw,status", [
    (dict(d=0), 1), (dict(d=33), 1), (dict(w2=16385), 1), (dict(w1=0), 1),
    (dict(counter_bits=16), 1), (dict(null_a=True), 1),
])
def test_chain3_validation(C, kw, status):
    L = C.lib()
    v = ctypes.c_void_p
    r = L.compass_estimate_chain3(
        v(0 if kw.get("null_a") else 16), v(32), v(48), kw.get("counter_bits", 32),
        kw.get("d", 3), kw.get("w1", 64), kw.get("w2", 64), v(8), v(8), v(8),
        None, v(8), v(8), v(0))
    assert r == status
    assert L.compass_last_error().decode() != ""


@pytest.mark.parametrize("kw,status", [
    (dict(r=0), 1), (dict(r=65), 1), (dict(b=0), 1), (dict(r=32, b=33), 1),
    (dict(n_joins=0), 1), (dict(n_joins=5), 1), (dict(n_rows=-1), 2),
    (dict(bad_seed=True), 1), (dict(null_counters=True), 1),
])
def test_agms_build_validation(C, kw, status):
    L = C.lib()
    r, b = kw.get("r", 3), kw.get("b", 4)
    nj = kw.get("n_joins", 2)
    seeds = np.zeros((max(r * b, 1), 6), np.uint64)
    if kw.get("bad_seed"):
        seeds[-1, 1] = (1 << 61) - 1
    specs = (C.SketchSpec * max(nj, 1))()
    arr = np.ascontiguousarray(seeds.reshape(-1))
    for e in range(max(nj, 1)):
        specs[e].key_col = 16
        specs[e].key_dtype = C.I32
        specs[e].seeds = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    rc = L.compass_agms_build(kw.get("n_rows", 10), None, 0, None, 0, specs, nj, r, b, 0,
                              ctypes.c_void_p(0 if kw.get("null_counters") else 48),
                              ctypes.c_void_p(64), ctypes.c_void_p(0))
    assert rc == status
    assert L.compass_last_error().decode() != ""


@pytest.mark.parametrize("kw,status", [
    (dict(n_tables=0), 1), (dict(n_tables=17), 1), (dict(r=0), 1), (dict(b=2000), 1),
])
def test_agms_estimate_validation(C, kw, status):
    L = C.lib()
    nt = kw.get("n_tables", 2)
    sk = (ctypes.c_void_p * 17)(*([16] * 17))
    ns = (ctypes.c_void_p * 17)(*([32] * 17))
    rc = L.compass_agms_estimate(sk, ns, nt, kw.get("r", 3), kw.get("b", 4), None,
                                 ctypes.c_void_p(8), ctypes.c_void_p(8), ctypes.c_void_p(0))
    assert rc == status
    assert L.compass_last_error().decode() != ""


@pytest.mark.parametrize("kw,status", [
    (dict(cap=-1), 1), (dict(null_count=True), 1), (dict(null_out=True), 1),
    (dict(row_base=-5), 2), (dict(d=0), 1),
])
def test_build_select_validation(C, kw, status):
    L = C.lib()
    d = kw.get("d", 3)
    s, keep = _spec(C, d, np.zeros((max(d, 1), 6), np.uint64))
    rc = L.compass_sketch_build_select(
        10, None, 0, None, 0, s, 1, d, 64, 32, 0, ctypes.c_void_p(64),
        ctypes.c_void_p(0 if kw.get("null_out") else 128), kw.get("cap", 100),
        ctypes.c_void_p(0 if kw.get("null_count") else 256), kw.get("row_base", 0),
        ctypes.c_void_p(0))
    assert rc == status
    assert L.compass_last_error().decode() != ""


def test_mlp_entry_points_reject_bad_arguments(C):
    """Null handles and pointers, empty batches and a non-positive rate are
    rejected before any GPU work."""
    L = C.lib()
    C._bind_mlp(L)
    vp = ctypes.c_void_p
    one = vp(16)
    assert L.compass_mlp_train_step(None, one, one, one, 4, ctypes.c_float(1e-3),
                                    one, None) == 1
    assert L.compass_mlp_train_epoch(None, one, one, one, one, 1, 4,
                                     ctypes.c_float(1e-3), one, None) == 1
    assert L.compass_mlp_forward(None, one, one, 4, one, None) == 1
    h = vp(16)  # a non-null handle is still not dereferenced when an argument is bad
    assert L.compass_mlp_train_epoch(h, None, one, one, one, 1, 4,
                                     ctypes.c_float(1e-3), one, None) == 1
    assert L.compass_mlp_train_epoch(h, one, one, one, one, 1, 0,
                                     ctypes.c_float(1e-3), one, None) == 1
    assert L.compass_mlp_train_epoch(h, one, one, one, one, 1, 4,
                                     ctypes.c_float(0.0), one, None) == 1


@pytest.mark.parametrize("kw,status", [
    (dict(k=1), 1), (dict(k=5), 1), (dict(k=4, d=13), 1), (dict(k=3, d=17), 1),
    (dict(w=[64, 0, 8]), 1), (dict(w=[1 << 10, 1 << 10, 1 << 9]), 1),
    (dict(counter_bits=8), 1), (dict(n_rows=-1), 2), (dict(bad_seed=True), 1),
    (dict(null_counters=True), 1),
])
def test_build_kd_validation(C, kw, status):
    """Argument checks of compass_sketch_build_kd (no device work)."""
    L = C.lib()
    k = kw.get("k", 3)
    d = kw.get("d", 3)
    w = kw.get("w", [16, 8, 4, 2][:max(1, min(k, 4))] + [2] * max(0, k - 4))
    specs = (C.SketchSpec * max(1, k))()
    keep = []
    for m in range(max(1, k)):
        s = np.zeros((max(d, 1), 6), np.uint64)
        if kw.get("bad_seed") and m == 1:
            s[-1, 3] = (1 << 61) + 1
        keep.append(s)
        specs[m].key_col = 8
        specs[m].key_dtype = C.I32
        specs[m].seeds = s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))
    wa = (ctypes.c_int32 * max(1, len(w)))(*w)
    r = L.compass_sketch_build_kd(
        kw.get("n_rows", 10), None, 0, None, 0, specs, k, d, wa,
        kw.get("counter_bits", 32), 0,
        ctypes.c_void_p(0 if kw.get("null_counters") else 48), ctypes.c_void_p(64),
        ctypes.c_void_p(0))
    assert r == status
    assert L.compass_last_error().decode() != ""


@pytest.mark.parametrize("kw,status", [
    (dict(n_tables=1, eu=[], ev=[]), 2), (dict(eu=[0, 1, 0], ev=[1, 2, 2]), 3),
    (dict(eu=[0, 0], ev=[1, 1]), 3), (dict(eu=[0, 2], ev=[0, 1]), 3),
    (dict(d=0), 1), (dict(d=33), 1), (dict(counter_bits=16), 1),
    (dict(width=[0, 4]), 1), (dict(null_tensor=True), 1),
    (dict(n_tables=6, eu=[0, 0, 0, 0, 0], ev=[1, 2, 3, 4, 5]), 5),
])
def test_estimate_partitioned_validation(C, kw, status):
    """Argument checks of compass_estimate_partitioned (no device work):
    not a tree, disconnected, bad sizes, a table with five joins."""
    L = C.lib()
    nt = kw.get("n_tables", 3)
    eu, ev = kw.get("eu", [0, 1]), kw.get("ev", [1, 2])
    width = kw.get("width", [4] * len(eu))
    ne = len(eu)
    ea = (ctypes.c_int32 * max(1, ne))(*eu)
    eb = (ctypes.c_int32 * max(1, ne))(*ev)
    wa = (ctypes.c_int32 * max(1, ne))(*width)
    tp = (ctypes.c_void_p * max(1, nt))(*([0] if kw.get("null_tensor") else [64]) * max(1, nt))
    g = C.TensorGraph(nt, ne, kw.get("d", 3), kw.get("counter_bits", 32), ea, eb, wa,
                      tp, 8)
    r = L.compass_estimate_partitioned(ctypes.byref(g), None, ctypes.c_void_p(8),
                                       ctypes.c_void_p(8), ctypes.c_void_p(0))
    assert r == status, L.compass_last_error().decode()
    assert L.compass_last_error().decode() != ""
