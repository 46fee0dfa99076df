"""Small-graph helpers for the tests: CSR construction, families with known cuts,
brute-force cut enumeration and an independent Stoer-Wagner.  Nothing here calls the
oracle or the GPU library."""
from __future__ import annotations

import itertools

import numpy as np


def csr_from_edges(n, edges):
    """Symmetric CSR (int64 offsets, int32 indices) of an undirected simple edge list."""
    rows = [set() for _ in range(n)]
    for a, b in edges:
        a, b = int(a), int(b)
        if a == b:
            continue
        rows[a].add(b)
        rows[b].add(a)
    off = np.zeros(n + 1, np.int64)
    for i in range(n):
        off[i + 1] = off[i] + len(rows[i])
    adj = np.array([x for r in rows for x in sorted(r)], np.int32)
    return off, adj


def edges_of(off, adj):
    n = len(off) - 1
    return [(u, int(adj[e])) for u in range(n) for e in range(off[u], off[u + 1]) if u < adj[e]]


def degrees(off):
    return np.diff(np.asarray(off))


def is_connected(n, edges, subset=None):
    verts = set(range(n)) if subset is None else set(subset)
    if not verts:
        return True
    adj = {v: [] for v in verts}
    for a, b in edges:
        if a in verts and b in verts:
            adj[a].append(b)
            adj[b].append(a)
    start = next(iter(verts))
    seen = {start}
    stack = [start]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == len(verts)


def random_connected(rng, n, p):
    """A random spanning tree plus G(n, p) edges: always connected."""
    edges = set()
    perm = rng.permutation(n)
    for i in range(1, n):
        j = int(rng.integers(0, i))
        a, b = int(perm[i]), int(perm[j])
        edges.add((min(a, b), max(a, b)))
    for a in range(n):
        for b in range(a + 1, n):
            if rng.random() < p:
                edges.add((a, b))
    return sorted(edges)


def brute_force_cuts(n, edges):
    """Every bipartition (S, V-S) with vertex n-1 outside S.  Returns (masks, values)."""
    e = np.array(edges, np.int64).reshape(-1, 2)
    masks = np.arange(1, 1 << (n - 1), dtype=np.int64)
    bu = (masks[:, None] >> e[None, :, 0]) & 1
    bv = (masks[:, None] >> e[None, :, 1]) & 1
    vals = (bu ^ bv).sum(axis=1)
    return masks, vals


def cut_value(edges, side):
    side = np.asarray(side, bool)
    return sum(1 for a, b in edges if side[a] != side[b])


def stoer_wagner(n, edges):
    """Textbook Stoer-Wagner (one merge per phase, weighted adjacency matrix)."""
    if n < 2:
        return 0
    W = np.zeros((n, n), np.int64)
    for a, b in edges:
        W[a, b] += 1
        W[b, a] += 1
    active = list(range(n))
    best = None
    while len(active) > 1:
        used = [active[0]]
        w = W[active[0], :].copy()
        rest = set(active[1:])
        prev = active[0]
        last = active[0]
        while rest:
            nxt = max(rest, key=lambda v: w[v])
            rest.remove(nxt)
            prev, last = last, nxt
            used.append(nxt)
            w += W[nxt, :]
        cut = int(W[last, :].sum() - W[last, last])
        best = cut if best is None else min(best, cut)
        # merge last into prev
        W[prev, :] += W[last, :]
        W[:, prev] += W[:, last]
        W[prev, prev] = 0
        W[last, :] = 0
        W[:, last] = 0
        active.remove(last)
    return best


# ---------------------------------------------------------------- families
def complete(n, base=0):
    return [(base + a, base + b) for a in range(n) for b in range(a + 1, n)]


def cycle(n):
    return [(i, (i + 1) % n) for i in range(n)]


def path(n):
    return [(i, i + 1) for i in range(n - 1)]


def hypercube(d):
    n = 1 << d
    return n, [(v, v ^ (1 << i)) for v in range(n) for i in range(d) if v < v ^ (1 << i)]


def complete_bipartite(a, b):
    return [(i, a + j) for i in range(a) for j in range(b)]


def two_cliques(a, b):
    """Two K_a on 0..a-1 and a..2a-1 joined by b vertex-disjoint edges."""
    e = complete(a) + complete(a, a)
    e += [(i, a + i) for i in range(b)]
    return 2 * a, e


def random_tree(rng, n):
    return [(i, int(rng.integers(0, i))) for i in range(1, n)]


def all_subsets(n):
    return itertools.chain.from_iterable(itertools.combinations(range(n), r) for r in range(n + 1))
