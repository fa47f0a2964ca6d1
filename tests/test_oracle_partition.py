"""Pins of the partitioned-sketch oracle (Section 5.1, sketch partitioning):
the two-dimensional sketch of a table with two joins and the three-table
chain estimate built from it."""
import numpy as np

from paper_2102_02440_amd import workloads as W


def _exact_chain(ka, kp1, kp2, kb):
    """|A join P join B| by counting (P joins A on its first key, B on its
    second)."""
    fa = {}
    for a in ka.tolist():
        fa[a] = fa.get(a, 0) + 1
    fb = {}
    for b in kb.tolist():
        fb[b] = fb.get(b, 0) + 1
    return sum(fa.get(a, 0) * fb.get(b, 0) for a, b in zip(kp1.tolist(), kp2.tolist()))


def _injective_seeds(rng, d):
    """Sign seeds drawn at random; bucket polynomial b0 = 0, b1 = 1, so
    h(x) = x mod w is one-to-one on keys below w."""
    s = W.draw_seeds(rng, 1, d)[0].copy()
    s[:, 4] = 0
    s[:, 5] = 1
    return s


def test_chain3_exact_without_collisions(oracle):
    """No bucket collisions: every sign appears squared, so each row's
    estimate is the exact join size (the unbiased estimator with zero
    variance)."""
    rng = np.random.default_rng(11)
    d, w1, w2 = 3, 16, 8
    s1, s2 = _injective_seeds(rng, d), _injective_seeds(rng, d)
    ka = rng.integers(0, w1, 40)
    kp1, kp2 = rng.integers(0, w1, 120), rng.integers(0, w2, 120)
    kb = rng.integers(0, w2, 30)
    A = oracle.sketch(ka, s1, d, w1)
    B = oracle.sketch(kb, s2, d, w2)
    P = oracle.sketch2d(kp1, kp2, s1, s2, d, w1, w2)
    vals, est, flag = oracle.chain3(A, P, B, [40, 120, 30])
    true = _exact_chain(ka, kp1, kp2, kb)
    assert vals == [true] * d
    assert est == float(true)
    assert flag == oracle.FLAG_EXACT


def test_sketch2d_constant_second_key_is_a_scaled_1d_sketch(oracle):
    """All second keys equal c: row i holds xi2_i(c) times the ordinary
    sketch of the first keys in column h2_i(c), zeros elsewhere."""
    rng = np.random.default_rng(12)
    d, w1, w2 = 4, 32, 16
    s1, s2 = W.draw_seeds(rng, 2, d)
    k1 = rng.integers(-1000, 1000, 500)
    c = 987654321
    P = oracle.sketch2d(k1, np.full(500, c), s1, s2, d, w1, w2)
    one = oracle.sketch(k1, s1, d, w1)
    for i in range(d):
        b, sg = oracle.hash_key(s2[i], c, w2)
        expect = np.zeros((w1, w2), dtype=np.int64)
        expect[:, b] = sg * one[i]
        assert np.array_equal(P[i], expect)


def test_sketch2d_is_linear(oracle):
    rng = np.random.default_rng(13)
    d, w1, w2 = 3, 8, 8
    s1, s2 = W.draw_seeds(rng, 2, d)
    k1, k2 = rng.integers(0, 10**6, 300), rng.integers(0, 10**6, 300)
    whole = oracle.sketch2d(k1, k2, s1, s2, d, w1, w2)
    parts = (oracle.sketch2d(k1[:111], k2[:111], s1, s2, d, w1, w2) +
             oracle.sketch2d(k1[111:], k2[111:], s1, s2, d, w1, w2))
    assert np.array_equal(whole, parts)
    assert np.abs(whole).sum(axis=(1, 2)).max() <= 300


def test_chain3_unbiased_over_seeds(oracle):
    """Averaged over independent hash functions the row estimate is the
    join size (4-wise independent signs, Section 5.1's unbiasedness)."""
    rng = np.random.default_rng(14)
    w1, w2 = 8, 8
    ka = rng.integers(0, 30, 60)
    kp1, kp2 = rng.integers(0, 30, 200), rng.integers(0, 30, 200)
    kb = rng.integers(0, 30, 50)
    true = _exact_chain(ka, kp1, kp2, kb)
    xs = []
    for t in range(600):
        s1, s2 = W.draw_seeds(np.random.default_rng(1000 + t), 2, 1)
        A = oracle.sketch(ka, s1, 1, w1)
        B = oracle.sketch(kb, s2, 1, w2)
        P = oracle.sketch2d(kp1, kp2, s1, s2, 1, w1, w2)
        xs.append(oracle.chain3(A, P, B, [60, 200, 50])[0][0])
    xs = np.asarray(xs, dtype=np.float64)
    se = xs.std(ddof=1) / np.sqrt(xs.size)
    assert abs(xs.mean() - true) < 4.5 * se, (xs.mean(), true, se)


def test_chain3_certificate(oracle):
    d, w1, w2 = 1, 2, 2
    A = np.zeros((d, w1), np.int64)
    P = np.zeros((d, w1, w2), np.int64)
    B = np.zeros((d, w2), np.int64)
    assert oracle.chain3(A, P, B, [10, 10, 10])[2] == oracle.FLAG_EXACT
    assert oracle.chain3(A, P, B, [2**43, 2**43, 2**42])[2] == 0
    assert oracle.chain3(A, P, B, [2**43, 2**42, 2**41])[2] == oracle.FLAG_EXACT
