"""Which sub-plan shapes the library's estimate evaluates (test helper).

The documented rule: every connected sub-plan whose generic contraction
fits its bounds (at most 6 independent cycles, 2^36 element steps of
w^cycles x list length x d); a table with more than 8 join edges may or may
not fit (it depends on the spanning tree).  Returns True (must be
evaluated), False (must be flagged unsupported) or None (either is allowed).
"""


def supported_shape(edge_u, edge_v, mask, w=None, d=1):
    tabs = [t for t in range(64) if mask >> t & 1]
    es = [(u, v) for u, v in zip(edge_u, edge_v) if mask >> u & 1 and mask >> v & 1]
    if len(tabs) == 1:
        return True
    deg = {t: 0 for t in tabs}
    for u, v in es:
        deg[u] += 1
        deg[v] += 1
    cycles = len(es) - len(tabs) + 1
    if cycles == 0:
        # the specialised path; beyond 6 children the generic one (up to 8)
        return True if max(deg.values()) <= 8 else None
    if cycles == 1 and _is_triangle(tabs, es, deg):
        return True if max(deg.values()) <= 6 else None
    if cycles > 6:
        return False
    if max(deg.values()) > 8:
        return None
    if w is not None:
        work = float(w) ** cycles * 2 * (len(tabs) - 1) * w * d
        if work > 2.0 ** 36 * 0.9:
            return None if work < 2.0 ** 36 * 1.1 else False
    return True


def _is_triangle(tabs, es, deg):
    """One cycle of three tables, no repeated pair: peeling tables of degree
    one leaves exactly three."""
    if len({tuple(sorted(e)) for e in es}) != len(es):
        return False
    d = dict(deg)
    alive = set(tabs)
    changed = True
    while changed:
        changed = False
        for t in list(alive):
            if d[t] == 1:
                alive.discard(t)
                for u, v in es:
                    if (u == t and v in alive) or (v == t and u in alive):
                        d[u if v == t else v] -= 1
                d[t] = 0
                changed = True
    return len(alive) == 3


def expected_flag_est(oracle, n_tables, edge_u, edge_v, d, w, sketches, n_sel,
                      mask, vals_o, flag_o, est_o):
    """(flag, est, tolerance) the library must report for one sub-plan,
    given the oracle's exact rows (vals_o, modulo 2^128), flag and median.
    Certified (oracle flag EXACT): the oracle's flag and median, exactly.
    Not certified: APPROX and the median of an fp64 evaluation, so within
    1e-12 of the contraction over absolute values of the exact median; the
    tests that use this keep |X_i| below 2^127 (no wrap), so vals_o are the
    exact rows."""
    if flag_o & 1 or bin(mask).count("1") == 1:
        return flag_o, est_o, 0.0
    import numpy as np
    ab = [np.abs(np.asarray(s, dtype=np.int64)) for s in sketches]
    babs, _, _ = oracle.estimate(n_tables, edge_u, edge_v, d, w, ab, n_sel, [mask])
    v = sorted(vals_o)
    med = v[d // 2] if d & 1 else (v[d // 2 - 1] + v[d // 2]) / 2
    return 4, float(med), 1e-12 * float(max(babs[0]))
