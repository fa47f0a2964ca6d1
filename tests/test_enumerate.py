"""Algorithm 1 (Section 6): the oracle's DFS is pinned by brute force over
all left-deep orders without cross products (exhaustive setting) and by a
hand-checked greedy case; the library's host implementation matches the
oracle on random graphs and estimates (no GPU needed)."""
import itertools

import numpy as np
import pytest

from paper_2102_02440_amd import workloads as W


def _graph(rng, n, extra):
    eu, ev = [], []
    for t in range(1, n):
        eu.append(int(rng.integers(0, t)))
        ev.append(t)
    for _ in range(extra):
        a, b = rng.choice(n, size=2, replace=False)
        if not any({a, b} == {u, v} for u, v in zip(eu, ev)):
            eu.append(int(a))
            ev.append(int(b))
    return eu, ev


def _brute(n, eu, ev, est):
    adj = [set() for _ in range(n)]
    for u, v in zip(eu, ev):
        adj[u].add(v)
        adj[v].add(u)
    best = float("inf")
    for perm in itertools.permutations(range(n)):
        ok = all(any(perm[k] in adj[perm[j]] for j in range(k)) for k in range(1, n))
        if not ok:
            continue
        m, c = 0, 0.0
        for v in perm:
            m |= 1 << v
            c += est[m]
        best = min(best, c)
    return best


def test_exhaustive_equals_brute_force(oracle):
    rng = np.random.default_rng(0)
    for rep in range(30):
        n = int(rng.integers(2, 7))
        eu, ev = _graph(rng, n, int(rng.integers(0, 3)))
        masks = W.connected_masks(n, eu, ev)
        est = {m: float(rng.integers(1, 10**6)) for m in masks}
        card = [est[1 << t] for t in range(n)]
        order, cost, _ = oracle.plan_enumeration(n, eu, ev, est, card, max_plans=0)
        assert cost == _brute(n, eu, ev, est)


def test_greedy_hand_example(oracle):
    # chain 0 - 1 - 2 with a pendant 3 on 1; estimates chosen by hand
    eu, ev = [0, 1, 1], [1, 2, 3]
    est = {1: 10.0, 2: 100.0, 4: 5.0, 8: 50.0, 3: 40.0, 6: 30.0, 10: 400.0,
           7: 60.0, 11: 500.0, 14: 90.0, 15: 70.0}
    card = [10, 100, 5, 50]
    # f: card/100 * .5 + deg/3 * .5 -> t2: .025+.167, t0: .05+.167, t3: .25+.167, t1: .5+.5
    order, cost, plans = oracle.plan_enumeration(4, eu, ev, est, card, max_plans=1)
    # from 2: {2} 5 -> +1 {1,2} 30 -> ext 0 (60) before 3 (90) -> {0,1,2} -> 3: 70
    assert order == [2, 1, 0, 3] and cost == 5 + 30 + 60 + 70


@pytest.mark.parametrize("max_plans", [1, 2, 10, 0])
def test_library_matches_oracle(oracle, max_plans):
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(max_plans + 5)
    for rep in range(40):
        n = int(rng.integers(2, 8))
        eu, ev = _graph(rng, n, int(rng.integers(0, 3)))
        masks = W.connected_masks(n, eu, ev)
        est = {m: float(rng.integers(-1000, 10**7)) for m in masks}
        card = [float(rng.integers(0, 10**6)) for _ in range(n)]
        o = oracle.plan_enumeration(n, eu, ev, est, card, max_plans=max_plans)
        g = C.enumerate_plan(n, eu, ev, list(est.keys()), list(est.values()), card,
                             max_plans=max_plans)
        assert (g[0], g[1], g[2]) == (o[0], o[1], o[2])


def test_greedy_hand_example_paper_variant(oracle):
    """Greedy of Section 7.2.8 by hand: chain 0 - 1 - 2 with a pendant 3 on
    1.  Two-way estimates {0,1} 40, {1,2} 30, {1,3} 400: the smallest is
    {1,2}; its smaller table by card is 2 (card 5 < 100).  From 2: only 1
    is adjacent -> {1,2} 30; then 0 ({0,1,2} 60) before 3 ({1,2,3} 90);
    then 3 -> 70.  Cost 5 + 30 + 60 + 70."""
    eu, ev = [0, 1, 1], [1, 2, 3]
    est = {1: 10.0, 2: 100.0, 4: 5.0, 8: 50.0, 3: 40.0, 6: 30.0, 10: 400.0,
           7: 60.0, 11: 500.0, 14: 90.0, 15: 70.0}
    card = [10, 100, 5, 50]
    order, cost = oracle.plan_greedy(4, eu, ev, est, card)
    assert order == [2, 1, 0, 3] and cost == 165.0
    # a source the f(v) order would not pick: {0,1} cheapest, card[1] < card[0]
    est2 = dict(est)
    est2[3] = 1.0
    order, cost = oracle.plan_greedy(4, eu, ev, est2, [10, 1, 5, 50])
    # from 1: {0,1} 1 < {1,2} 30 < {1,3} 400 -> 0; then {0,1,2} 60 < {0,1,3} 500
    assert order == [1, 0, 2, 3] and cost == 100.0 + 1.0 + 60.0 + 70.0


def test_plan_cost_is_sum_of_prefixes(oracle):
    vals = {1: 3, 3: 7, 7: 11, 4: 2, 6: 5}
    assert oracle.plan_cost([0, 1, 2], vals) == 3 + 7 + 11
    assert oracle.plan_cost([2, 1, 0], vals) == 2 + 5 + 11


def test_greedy_is_a_valid_plan_no_better_than_exhaustive(oracle):
    """Greedy returns a left-deep order without cross products whose cost is
    the sum of its prefixes' estimates, and never below the exhaustive
    optimum (brute force)."""
    rng = np.random.default_rng(11)
    for rep in range(40):
        n = int(rng.integers(2, 7))
        eu, ev = _graph(rng, n, int(rng.integers(0, 3)))
        masks = W.connected_masks(n, eu, ev)
        est = {m: float(rng.integers(1, 10**6)) for m in masks}
        card = [float(rng.integers(1, 10**6)) for _ in range(n)]
        order, cost = oracle.plan_greedy(n, eu, ev, est, card)
        assert sorted(order) == list(range(n))
        adj = [set() for _ in range(n)]
        for u, v in zip(eu, ev):
            adj[u].add(v)
            adj[v].add(u)
        assert all(any(order[k] in adj[order[j]] for j in range(k)) for k in range(1, n))
        assert cost == oracle.plan_cost(order, est)
        assert cost >= _brute(n, eu, ev, est)


def test_library_greedy_matches_oracle(oracle):
    from paper_2102_02440_amd import compass as C
    rng = np.random.default_rng(23)
    for rep in range(60):
        n = int(rng.integers(1, 9))
        eu, ev = _graph(rng, n, int(rng.integers(0, 3)) if n > 2 else 0)
        masks = W.connected_masks(n, eu, ev)
        est = {m: float(rng.integers(-100, 10**4)) for m in masks}   # ties happen
        card = [float(rng.integers(0, 50)) for _ in range(n)]
        o = oracle.plan_greedy(n, eu, ev, est, card)
        g = C.enumerate_greedy(n, eu, ev, list(est.keys()), list(est.values()), card)
        assert (g[0], g[1]) == (o[0], o[1]), (n, eu, ev)
