"""compass_sketch_build_noalloc (fixed scratch region, no allocation)
against compass_sketch_build on the same inputs, bit for bit: two calls in
a row, the second with a smaller input, for the fused scan and for the
two-phase build (one batch, and many batches with flushes); and the
rejection of a build that cannot fit the region, before any GPU work."""
import os

import numpy as np
import pytest

from paper_2102_02440_amd import workloads as W

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(C, torch, n, pred_cols, preds, keys, seeds, d, w, bits):
    cdt = torch.int32 if bits == 32 else torch.int64
    ref = [torch.full((d, w), 5, dtype=cdt, device="cuda") for _ in keys]
    got = [torch.full((d, w), -9, dtype=cdt, device="cuda") for _ in keys]
    n_ref = torch.zeros(1, dtype=torch.int64, device="cuda")
    n_got = torch.full((1,), 77, dtype=torch.int64, device="cuda")
    C.sketch_build(n, pred_cols, preds, keys, seeds, ref, n_ref, d, w, bits)
    C.sketch_build(n, pred_cols, preds, keys, seeds, got, n_got, d, w, bits,
                   noalloc=True)
    torch.cuda.synchronize()
    assert n_got.item() == n_ref.item()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    return n_ref.item()


@gpu
def test_noalloc_fused_scan_two_calls():
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(71)
    print("[case] noalloc fused 3M rows, 2 sketches, d=7, w=8192", flush=True)
    n = 3_000_001
    keys = [torch.from_numpy(W.fk_column(rng, n, 100_000, 1.0,
                                         rng.permutation(100_000))).cuda()
            for _ in range(2)]
    seeds = [W.draw_seeds(rng, 1, 7)[0] for _ in keys]
    assert _both(C, torch, n, [], [], keys, seeds, 7, 8192, 32) == n
    print("[case] noalloc fused, smaller second call", flush=True)
    n2 = 200_003
    k2 = [keys[1][:n2]]
    s2 = [W.draw_seeds(rng, 1, 5)[0]]
    assert _both(C, torch, n2, [], [], k2, s2, 5, 1024, 32) == n2


@gpu
@pytest.mark.parametrize("cap", [None, 150_000])
def test_noalloc_two_phase_two_calls(cap):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(72)
    n = 4_000_037
    keys = [torch.from_numpy(W.fk_column(rng, n, 1_000_000, 1.1,
                                         rng.permutation(1_000_000)).astype(np.int64)).cuda(),
            torch.from_numpy(rng.integers(-2**40, 2**40, n).astype(np.int64)).cuda()]
    a = torch.from_numpy(rng.integers(0, 100, n).astype(np.int32)).cuda()
    f = torch.from_numpy(rng.random(n).astype(np.float32)).cuda()
    preds = [{"col": 0, "kind": "range", "lo": 10, "hi": 69},
             {"col": 1, "kind": "range", "lo": 0.0, "hi": 0.5}]
    seeds = [W.draw_seeds(rng, 1, 11)[0] for _ in keys]
    old = os.environ.get("COMPASS_SURVIVOR_CAP_ROWS")
    if cap:
        os.environ["COMPASS_SURVIVOR_CAP_ROWS"] = str(cap)
    try:
        print("[case] noalloc two-phase 4M rows, d=11, w=65536, cap", cap, flush=True)
        sel = _both(C, torch, n, [a, f], preds, keys, seeds, 11, 65536, 64)
        assert 0.25 * n < sel < 0.35 * n
        print("[case] noalloc two-phase, smaller second call", flush=True)
        n2 = 100_001
        sel2 = _both(C, torch, n2, [a[:n2]], preds[:1], [keys[0][:n2]], seeds[:1],
                     3, 40000, 32)
        assert 0.55 * n2 < sel2 < 0.65 * n2
    finally:
        if cap:
            if old is None:
                del os.environ["COMPASS_SURVIVOR_CAP_ROWS"]
            else:
                os.environ["COMPASS_SURVIVOR_CAP_ROWS"] = old


@gpu
def test_noalloc_rejects_builds_beyond_the_region():
    """Four sketches of d = 32 rows of 2^20 buckets: one chunk of partial
    counters is 512 MiB, above the 256 MiB region.  Refused with E_RANGE
    before any GPU work (the counters and the count are left as they were)."""
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    keys = [torch.zeros(16, dtype=torch.int32, device="cuda") for _ in range(4)]
    # full-size counters (512 MiB in all), so that even a build that went
    # ahead would stay inside its buffers
    cnt = [torch.full((32, 1 << 20), 3, dtype=torch.int32, device="cuda")
           for _ in range(4)]
    nsel = torch.full((1,), 11, dtype=torch.int64, device="cuda")
    seeds = [np.zeros((32, 6), np.uint64) for _ in range(4)]
    print("[case] noalloc rejection", flush=True)
    with pytest.raises(C.CompassError) as e:
        C.sketch_build(16, [], [], keys, seeds, cnt, nsel, 32, 1 << 20, 32,
                       noalloc=True)
    assert e.value.status == 2
    assert "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert nsel.item() == 11
    assert all(bool((c == 3).all()) for c in cnt)
