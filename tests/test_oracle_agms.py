"""Pins of the AGMS oracle (Section 4.1): the composed sketch of a table
(product over its joins' +-1 variables), the basic estimate as the
product of the tables' counters, row averages and their median."""
import numpy as np

from paper_2102_02440_amd import workloads as W


def _seeds(seed, K):
    return W.draw_seeds(np.random.default_rng(seed), 1, K)[0]


def test_single_key_is_exact(oracle):
    """One join key value on both sides: every counter is n * xi(a), so
    every basic estimate is n_A * n_B exactly."""
    s = _seeds(1, 6)
    A = oracle.agms_sketch([np.full(37, 12345)], [s], 2, 3)
    B = oracle.agms_sketch([np.full(11, 12345)], [s], 2, 3)
    rows, est, flag = oracle.agms_estimate([A, B], [37, 11])
    assert rows == [3 * 37 * 11, 3 * 37 * 11]
    assert est == 37.0 * 11
    assert flag == oracle.FLAG_EXACT


def test_three_table_basic_estimate_is_the_triple_sum(oracle):
    """Section 4.1.2: the basic estimate of k - mk - t is the sum over all
    tuple triples of xi1(x) xi1(y.k) xi2(y.m) xi2(z); the product of the
    composed sketches must equal that sum, counter by counter."""
    rng = np.random.default_rng(2)
    r, b = 2, 3
    K = r * b
    s1, s2 = _seeds(3, K), _seeds(4, K)
    kx = rng.integers(0, 7, 9)
    y1, y2 = rng.integers(0, 7, 12), rng.integers(0, 5, 12)
    kz = rng.integers(0, 5, 8)
    A = oracle.agms_sketch([kx], [s1], r, b)
    P = oracle.agms_sketch([y1, y2], [s1, s2], r, b)
    B = oracle.agms_sketch([kz], [s2], r, b)
    rows, _, _ = oracle.agms_estimate([A, P, B], [9, 12, 8])
    for i in range(r):
        total = 0
        for j in range(b):
            c = i * b + j
            x1 = [oracle.hash_key(s1[c], int(v), 1)[1] for v in kx]
            p1 = [oracle.hash_key(s1[c], int(v), 1)[1] for v in y1]
            p2 = [oracle.hash_key(s2[c], int(v), 1)[1] for v in y2]
            z2 = [oracle.hash_key(s2[c], int(v), 1)[1] for v in kz]
            brute = sum(a * py1 * py2 * zz for a in x1 for py1, py2 in zip(p1, p2)
                        for zz in z2)
            assert A[i, j] * P[i, j] * B[i, j] == brute
            total += brute
        assert rows[i] == total


def test_average_then_median(oracle):
    """r = 2 (even): the mean of the two row averages; each average is the
    row sum over b."""
    A = np.array([[1, 2, 3], [4, 5, -6]], dtype=np.int64)
    B = np.array([[1, 1, 1], [2, 2, 2]], dtype=np.int64)
    rows, est, _ = oracle.agms_estimate([A, B], [10, 10])
    assert rows == [6, 6]
    assert est == (6 / 3 + 6 / 3) / 2
    C = np.array([[1, 1, 1], [2, 2, 2], [9, 9, 9]], dtype=np.int64)
    rows, est, _ = oracle.agms_estimate([C, C], [10, 10])
    assert rows == [3, 12, 243] and est == 4.0


def test_unbiased_three_way(oracle):
    """Averaged over independent families the basic estimate of a chain is
    its join size."""
    rng = np.random.default_rng(5)
    kx = rng.integers(0, 6, 20)
    y1, y2 = rng.integers(0, 6, 30), rng.integers(0, 4, 30)
    kz = rng.integers(0, 4, 15)
    fa = np.bincount(kx, minlength=6)
    fb = np.bincount(kz, minlength=4)
    true = int(sum(fa[a] * fb[b] for a, b in zip(y1, y2)))
    r, b = 1, 400
    xs = []
    for t in range(6):
        s1, s2 = _seeds(100 + t, r * b), _seeds(200 + t, r * b)
        A = oracle.agms_sketch([kx], [s1], r, b)
        P = oracle.agms_sketch([y1, y2], [s1, s2], r, b)
        B = oracle.agms_sketch([kz], [s2], r, b)
        xs.append((A * P * B).reshape(-1))
    xs = np.concatenate(xs).astype(np.float64)
    se = xs.std(ddof=1) / np.sqrt(xs.size)
    assert abs(xs.mean() - true) < 4.5 * se, (xs.mean(), true, se)


def test_agms_sketch_is_linear(oracle):
    rng = np.random.default_rng(6)
    s1, s2 = _seeds(7, 8), _seeds(8, 8)
    k1, k2 = rng.integers(-50, 50, 100), rng.integers(0, 10**9, 100)
    whole = oracle.agms_sketch([k1, k2], [s1, s2], 2, 4)
    parts = (oracle.agms_sketch([k1[:40], k2[:40]], [s1, s2], 2, 4) +
             oracle.agms_sketch([k1[40:], k2[40:]], [s1, s2], 2, 4))
    assert np.array_equal(whole, parts)
