"""Which sub-plan shapes the library's estimate evaluates (test helper).

The documented rule: trees, and trees plus one edge that closes a triangle
(no two edges between the same pair of tables), as long as some rooting
leaves every table at most 6 child edges.  Returns True (must be
evaluated), False (must be flagged unsupported) or None (a table of
degree 7 or more: the outcome depends on the rooting, either is allowed).
"""


def supported_shape(edge_u, edge_v, mask):
    tabs = [t for t in range(64) if mask >> t & 1]
    es = [(u, v) for u, v in zip(edge_u, edge_v) if mask >> u & 1 and mask >> v & 1]
    if len(tabs) == 1:
        return True
    deg = {t: 0 for t in tabs}
    for u, v in es:
        deg[u] += 1
        deg[v] += 1
    pairs = {tuple(sorted(e)) for e in es}
    cycles = len(es) - len(tabs) + 1
    if cycles == 0:
        ok = True
    elif cycles == 1 and len(pairs) == len(es):
        # the single cycle is a triangle iff peeling leaves of degree one
        # leaves exactly three tables
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
        ok = len(alive) == 3
    else:
        ok = False
    if ok and max(deg.values()) > 6:
        return None
    return ok
