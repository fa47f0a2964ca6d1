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


# ---------------------------------------------------------------------------
# partitioned sketches of tables with k joins, and the tree estimate
# ---------------------------------------------------------------------------
def test_sketch_kd_two_joins_is_the_2d_sketch(oracle):
    """k = 2 is the two-dimensional sketch (pinned above)."""
    rng = np.random.default_rng(21)
    d = 3
    s1, s2 = W.draw_seeds(rng, 2, d)
    k1, k2 = rng.integers(-500, 500, 300), rng.integers(0, 10**12, 300)
    T = oracle.sketch_kd([k1, k2], [s1, s2], d, [8, 32])
    assert np.array_equal(T, oracle.sketch2d(k1, k2, s1, s2, d, 8, 32))


def test_sketch_kd_single_row(oracle):
    """One row (a, b, c): each sketch row has the single entry
    xi1(a) xi2(b) xi3(c) at (h1(a), h2(b), h3(c)) and zeros elsewhere."""
    rng = np.random.default_rng(22)
    d, w = 4, [5, 7, 3]
    seeds = list(W.draw_seeds(rng, 3, d))
    key = [123456789, -42, 2**40 + 7]
    T = oracle.sketch_kd([[x] for x in key], seeds, d, w)
    for i in range(d):
        idx, sign = [], 1
        for m in range(3):
            b, g = oracle.hash_key(seeds[m][i], key[m], w[m])
            idx.append(b)
            sign *= g
        expect = np.zeros(w, dtype=np.int64)
        expect[tuple(idx)] = sign
        assert np.array_equal(T[i], expect)


def test_sketch_kd_constant_last_key_reduces_to_2d(oracle):
    """Every third key equal to c: row i is xi3_i(c) times the 2-D sketch of
    the first two keys, placed at third index h3_i(c); zeros elsewhere."""
    rng = np.random.default_rng(23)
    d, w = 3, [16, 8, 4]
    s1, s2, s3 = W.draw_seeds(rng, 3, d)
    k1, k2 = rng.integers(0, 1000, 400), rng.integers(0, 1000, 400)
    c = 31337
    T = oracle.sketch_kd([k1, k2, np.full(400, c)], [s1, s2, s3], d, w)
    P = oracle.sketch2d(k1, k2, s1, s2, d, w[0], w[1])
    for i in range(d):
        b, g = oracle.hash_key(s3[i], c, w[2])
        expect = np.zeros(w, dtype=np.int64)
        expect[:, :, b] = g * P[i]
        assert np.array_equal(T[i], expect)


def _edge_seeds(rng, n_edges, d, injective=False):
    return [(_injective_seeds(rng, d) if injective else W.draw_seeds(rng, 1, d)[0])
            for _ in range(n_edges)]


def test_tensor_join_chain_is_chain3(oracle):
    """The chain A - P - B (P a 2-D sketch) equals the chain estimate
    (pinned above), row by row."""
    rng = np.random.default_rng(24)
    d, w1, w2 = 3, 8, 16
    s1, s2 = _edge_seeds(rng, 2, d)
    ka, kb = rng.integers(0, 50, 70), rng.integers(0, 50, 60)
    kp1, kp2 = rng.integers(0, 50, 200), rng.integers(0, 50, 200)
    A = oracle.sketch(ka, s1, d, w1)
    B = oracle.sketch(kb, s2, d, w2)
    P = oracle.sketch2d(kp1, kp2, s1, s2, d, w1, w2)
    # tables A = 0, P = 1, B = 2; edges A-P (0) and P-B (1)
    vals, est, flag = oracle.tensor_join(3, [0, 1], [1, 2], d, [w1, w2], [A, P, B],
                                         [70, 200, 60])
    vc, ec, fc = oracle.chain3(A, P, B, [70, 200, 60])
    assert vals == [v % (1 << 128) for v in vc]
    assert est == ec and flag == fc


def _star(rng, n_center, n_leaf, dom):
    """A center table with three foreign keys and three leaf tables."""
    center = [rng.integers(0, dom, n_center) for _ in range(3)]
    leaves = [rng.integers(0, dom, n_leaf) for _ in range(3)]
    return center, leaves


def _star_size(center, leaves):
    cnt = []
    for lf in leaves:
        c = {}
        for x in lf.tolist():
            c[x] = c.get(x, 0) + 1
        cnt.append(c)
    return sum(cnt[0].get(a, 0) * cnt[1].get(b, 0) * cnt[2].get(e, 0)
               for a, b, e in zip(*(k.tolist() for k in center)))


def test_tensor_join_star_exact_without_collisions(oracle):
    """Star join (center with three joins, three leaves), keys below every
    width and one-to-one buckets: every product of signs squares to 1, so
    each row is the exact join size."""
    rng = np.random.default_rng(25)
    d, w = 2, [8, 8, 8]
    seeds = _edge_seeds(rng, 3, d, injective=True)
    center, leaves = _star(rng, 150, 40, 8)
    # tables: center 0, leaves 1..3; edge m joins center and leaf m + 1
    T0 = oracle.sketch_kd(center, seeds, d, w)
    Ls = [oracle.sketch(leaves[m], seeds[m], d, w[m]) for m in range(3)]
    vals, est, flag = oracle.tensor_join(4, [0, 0, 0], [1, 2, 3], d, w, [T0] + Ls,
                                         [150, 40, 40, 40])
    true = _star_size(center, leaves)
    assert vals == [true] * d
    assert est == float(true) and flag == oracle.FLAG_EXACT


def test_tensor_join_star_unbiased(oracle):
    """With bucket collisions, the estimate is unbiased over the hash
    functions (4-wise independent signs): the mean over 400 seed draws is
    within 5 standard errors of the exact star join size."""
    rng = np.random.default_rng(26)
    d, w = 1, [4, 4, 4]
    center, leaves = _star(rng, 60, 25, 12)
    true = _star_size(center, leaves)
    xs = []
    for _ in range(400):
        seeds = _edge_seeds(rng, 3, d)
        T0 = oracle.sketch_kd(center, seeds, d, w)
        Ls = [oracle.sketch(leaves[m], seeds[m], d, w[m]) for m in range(3)]
        vals, _, _ = oracle.tensor_join(4, [0, 0, 0], [1, 2, 3], d, w, [T0] + Ls,
                                        [60, 25, 25, 25])
        v = vals[0]
        xs.append(v - (1 << 128) if v >= 1 << 127 else v)
    xs = np.array(xs, dtype=np.float64)
    se = xs.std() / np.sqrt(len(xs))
    assert abs(xs.mean() - true) < 5 * se + 1e-9, (xs.mean(), true, se)


def test_tensor_join_certificate(oracle):
    """The flag certifies the rows only while the product of the selected
    rows stays below 2^127."""
    rng = np.random.default_rng(27)
    d, w = 1, [4]
    s = _edge_seeds(rng, 1, d)
    A = oracle.sketch(rng.integers(0, 9, 5), s[0], d, 4)
    B = oracle.sketch(rng.integers(0, 9, 5), s[0], d, 4)
    # two tables just below 2^63 each: below 2^126
    _, _, f1 = oracle.tensor_join(2, [0], [1], d, w, [A, B], [2**63 - 1, 2**63 - 1])
    assert f1 == oracle.FLAG_EXACT
    # three tables at 2^62 each: 2^186 > 2^127
    C = oracle.sketch2d(rng.integers(0, 9, 5), rng.integers(0, 9, 5), s[0], s[0], d, 4, 4)
    _, _, f3 = oracle.tensor_join(3, [0, 1], [1, 2], d, [4, 4], [A, C, B], [2**62] * 3)
    assert f3 == 0
