"""The two packings of edge-disjoint spanning forests that certify lambda >= t in the item
kernel, modelled in plain Python on the CPU (no GPU, no oracle arithmetic beyond building
the inputs).

t edge-disjoint spanning forests of a connected set prove that every cut crosses t edges.
The first packing is a sampled greedy: every vertex links two entries of its row per
forest (entries 2f and 2f + 1, modulo the row length, toward larger ids), then every
unused edge joins the first forest in which it connects two trees.  On the 5-cores of
power-law clusters (minimum degree 5, lambda = 5) it misses a few links in the last
forests for t = 4: low-degree vertices, which need one edge in every forest, lose edges to
forests that did not need them.  The second packing places every edge from its endpoint
with the shorter row (ties: the smaller id), rows of at most 2t entries first, and spreads
each row's edges over the forests in turn; it spans all four forests on the same sets, in
any order of the vertices (the kernel's threads run in no fixed order).  Both must give
edge-disjoint forests whatever the order."""
import numpy as np
import pytest

import gen
import oracle


def _find(p, x):
    while p[x] != x:
        p[x] = p[p[x]]
        x = p[x]
    return x


def _sampled_greedy(off, adj, t):
    n = len(off) - 1
    par = [list(range(n)) for _ in range(t)]
    used = {}
    for x in range(n):
        r0, dg = int(off[x]), int(off[x + 1] - off[x])
        for f in range(t):
            for e in (r0 + (2 * f) % dg, r0 + (2 * f + 1) % dg):
                y = int(adj[e])
                key = (x, y)
                if y > x and key not in used:
                    a, b = _find(par[f], x), _find(par[f], y)
                    if a != b:
                        par[f][a] = b
                        used[key] = f
    for x in range(n):
        for e in range(off[x], off[x + 1]):
            y = int(adj[e])
            if y <= x or (x, y) in used:
                continue
            for f in range(t):
                a, b = _find(par[f], x), _find(par[f], y)
                if a != b:
                    par[f][a] = b
                    used[(x, y)] = f
                    break
    return used


def _by_shorter_row(off, adj, t, order):
    n = len(off) - 1
    ln = np.diff(off)
    par = [list(range(n)) for _ in range(t)]
    used = {}
    for phase in (0, 1):
        for x in order:
            x = int(x)
            if (ln[x] <= 2 * t) != (phase == 0):
                continue
            f0 = 0
            for e in range(off[x], off[x + 1]):
                y = int(adj[e])
                if ln[y] < ln[x] or (ln[y] == ln[x] and y < x):
                    continue  # y places this edge
                for j in range(t):
                    f = (f0 + j) % t
                    a, b = _find(par[f], x), _find(par[f], y)
                    if a != b:
                        par[f][a] = b
                        assert (min(x, y), max(x, y)) not in used
                        used[(min(x, y), max(x, y))] = f
                        f0 = (f + 1) % t
                        break
    return used


def _forest_sizes(n, used, t):
    """Edges per forest, after checking that each forest is acyclic (every edge joins two
    trees when the forest is rebuilt from scratch)."""
    sizes = [0] * t
    par = [list(range(n)) for _ in range(t)]
    for (x, y), f in used.items():
        a, b = _find(par[f], x), _find(par[f], y)
        assert a != b, "forest %d has a cycle" % f
        par[f][a] = b
        sizes[f] += 1
    return sizes


def _five_core_of_largest_cluster(seed):
    g = gen.chung_lu(20000, 30.0, 2.3, 2000, 6000, 1.5, 0.2, 0.0, 0.0, seed=seed, intra_mult=1.4)
    memb = g.membership
    c = int(np.bincount(memb[memb >= 0]).argmax())
    vs = np.nonzero(memb == c)[0]
    loc = -np.ones(g.n, np.int64)
    loc[vs] = np.arange(len(vs))
    rows = []
    for v in vs:
        nb = loc[g.indices[g.offsets[v]:g.offsets[v + 1]]]
        rows.append(np.sort(nb[nb >= 0]))
    off = np.zeros(len(vs) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    adj = np.concatenate(rows).astype(np.int32)
    keep = np.nonzero(oracle.kcore(off, adj, 5))[0]
    loc2 = -np.ones(len(vs), np.int64)
    loc2[keep] = np.arange(len(keep))
    rows = [loc2[rows[i]][loc2[rows[i]] >= 0] for i in keep]
    off = np.zeros(len(keep) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rows])
    return off, np.concatenate(rows).astype(np.int32)


@pytest.mark.parametrize("seed", [103, 104])
def test_second_packing_spans_where_the_greedy_does_not(seed):
    off, adj = _five_core_of_largest_cluster(seed)
    n, t = len(off) - 1, 4
    assert n > 2000 and int(np.diff(off).min()) == 5
    assert oracle.mincut(off, adj, 5)[0] == 5          # four spanning trees are possible
    greedy = _forest_sizes(n, _sampled_greedy(off, adj, t), t)
    assert min(greedy) < n - 1, greedy                  # the first packing falls short
    for s in range(3):
        order = np.random.default_rng(s).permutation(n)
        sizes = _forest_sizes(n, _by_shorter_row(off, adj, t, order), t)
        assert sizes == [n - 1] * t, (s, sizes)
