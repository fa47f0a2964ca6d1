"""Selection-output materialisation (Section 3, "Partitioned query
execution"): the qualifying row indices written next to the sketches,
compared as sets with the oracle's predicate evaluation (their order is
unspecified; each index is unique)."""
import numpy as np
import pytest

from paper_2102_02440_amd import workloads as W

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print("[case]", *a, flush=True)


def _dev_table(tb, dev):
    import torch
    cols = {c: torch.from_numpy(v).to(dev) for c, v in tb.cols.items()}
    names = list(cols)
    pr = []
    for p in tb.preds:
        e = {"col": names.index(p.col), "kind": p.kind, "lo": p.lo, "hi": p.hi}
        if p.kind == "subset":
            e["bitmap"] = torch.from_numpy(np.asarray(p.bitmap, np.uint64).view(np.int64)).to(dev)
            e["domain"] = p.domain
        pr.append(e)
    return cols, list(cols.values()), pr


def _select(tb, key, seeds, d, w, cap, bits=32, row_base=0, acc=False, rows=None,
            count=None, cnt=None, nsel=None, n_rows=None, cols_override=None):
    torch = _torch()
    from paper_2102_02440_amd import compass as C
    dev = "cuda"
    cols, cl, pr = cols_override or _dev_table(tb, dev)
    ct = torch.int32 if bits == 32 else torch.int64
    cnt = cnt if cnt is not None else torch.zeros((d, w), dtype=ct, device=dev)
    nsel = nsel if nsel is not None else torch.zeros(1, dtype=torch.int64, device=dev)
    rows = rows if rows is not None else torch.full((cap,), -1, dtype=torch.int64, device=dev)
    count = count if count is not None else torch.zeros(1, dtype=torch.int64, device=dev)
    C.sketch_build_select(tb.n_rows if n_rows is None else n_rows, cl, pr, [cols[key]],
                          [seeds], [cnt], nsel, d, w, rows, count, row_base=row_base,
                          counter_bits=bits, accumulate=acc)
    torch.cuda.synchronize()
    return cnt, nsel, rows, count


@gpu
@pytest.mark.parametrize("seed", range(4))
def test_select_rows_random(oracle, seed):
    rng = np.random.default_rng(800 + seed)
    q = W.small_random_query(rng, 2, int(rng.integers(1, 20000)), 1000, 3, 256,
                             pred_prob=1.0)
    tb = q.tables[0]
    _say("select random", seed, tb.n_rows, [p.kind for p in tb.preds])
    mask = oracle.eval_predicates(tb.cols, tb.preds)
    cnt, nsel, rows, count = _select(tb, "k0", q.seeds[0], q.d, q.w, tb.n_rows + 5)
    n = int(mask.sum())
    assert nsel.item() == n and count.item() == n
    got = np.sort(rows.cpu().numpy()[:n])
    assert np.array_equal(got, np.nonzero(mask)[0])
    assert (rows.cpu().numpy()[n:] == -1).all()
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64),
                          oracle.sketch(tb.cols["k0"][mask], q.seeds[0], q.d, q.w))


@gpu
def test_select_dense_wide_and_overflow(oracle):
    """No predicates (every row), the wide-sketch path (w = 65536), and a
    capacity below the count: then the output is a duplicate-free subset."""
    torch = _torch()
    rng = np.random.default_rng(9)
    n = 4096 * 5 + 311
    tb = W.Table("x", {"k": rng.integers(0, 10**6, n).astype(np.int32),
                       "a": rng.integers(0, 100, n).astype(np.int32)}, [])
    seeds = W.draw_seeds(rng, 1, 2)[0]
    _say("select dense", n)
    cnt, nsel, rows, count = _select(tb, "k", seeds, 2, 1024, n)
    assert count.item() == n
    assert np.array_equal(np.sort(rows.cpu().numpy()), np.arange(n))
    tb.preds = [W.Predicate("a", "range", 10, 29)]
    mask = oracle.eval_predicates(tb.cols, tb.preds)
    _say("select wide", n)
    cnt, nsel, rows, count = _select(tb, "k", seeds, 2, 65536, n, bits=64)
    m = int(mask.sum())
    assert count.item() == m
    assert np.array_equal(np.sort(rows.cpu().numpy()[:m]), np.nonzero(mask)[0])
    assert np.array_equal(cnt.cpu().numpy(), oracle.sketch(tb.cols["k"][mask], seeds, 2, 65536))
    _say("select overflow", n)
    cap = m // 3
    cnt, nsel, rows, count = _select(tb, "k", seeds, 2, 1024, cap)
    assert count.item() == m and nsel.item() == m
    got = rows.cpu().numpy()
    assert np.unique(got).size == cap
    assert mask[got].all()


@gpu
def test_select_two_partitions_accumulate(oracle):
    """Two calls over the two halves of a table, accumulating, with
    row_base = the second half's first row: the union is the whole
    selection with global row indices."""
    torch = _torch()
    rng = np.random.default_rng(10)
    n = 30000
    k = rng.integers(0, 5000, n).astype(np.int32)
    a = rng.integers(0, 1000, n).astype(np.int32)
    seeds = W.draw_seeds(rng, 1, 3)[0]
    pred = [W.Predicate("a", "range", 100, 399)]
    h = 12345
    t1 = W.Table("p1", {"k": k[:h], "a": a[:h]}, pred)
    t2 = W.Table("p2", {"k": k[h:], "a": a[h:]}, pred)
    _say("select partitions", n, h)
    cnt, nsel, rows, count = _select(t1, "k", seeds, 3, 512, n)
    cnt, nsel, rows, count = _select(t2, "k", seeds, 3, 512, n, row_base=h, acc=True,
                                     rows=rows, count=count, cnt=cnt, nsel=nsel)
    mask = (a >= 100) & (a <= 399)
    m = int(mask.sum())
    assert count.item() == m and nsel.item() == m
    assert np.array_equal(np.sort(rows.cpu().numpy()[:m]), np.nonzero(mask)[0])
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64),
                          oracle.sketch(k[mask], seeds, 3, 512))


@gpu
def test_select_6a_full_size(oracle):
    """The 6a-shaped tables at full size (t: range, n: subset, k: point,
    ci: no predicate, 36M rows), materialised with room for all rows."""
    q = W.job6a(seed=W.DEFAULT_SEED)
    for t in (0, 2, 4, 3):
        tb = q.tables[t]
        key = q.incident(t)[0][2]
        _say("select 6a", tb.name, tb.n_rows)
        mask = oracle.eval_predicates(tb.cols, tb.preds)
        m = int(mask.sum())
        cnt, nsel, rows, count = _select(tb, key, q.seeds[q.incident(t)[0][0]], q.d, q.w,
                                         m + 1)
        assert count.item() == m and nsel.item() == m
        r = rows.cpu().numpy()
        assert r[m] == -1
        assert np.array_equal(np.sort(r[:m]), np.nonzero(mask)[0])
