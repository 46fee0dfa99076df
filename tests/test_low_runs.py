"""The fact behind the GPU's PAPER-mode runs at the minimum degree, checked on the CPU
against the oracle's one-cut-at-a-time replay (no GPU).

In PAPER mode (Alg. 1-3 as printed) a connected set H whose edge connectivity equals its
minimum degree delta has the canonical cut (delta, {smallest vertex of degree delta}):
Phase 0 of the cut rule sets it and the rounds replace it only by a strictly smaller cut.
When delta < k(|H|), that vertex is split off, its part is dropped, and the rest is
checked again.  The GPU proposes a whole run of such removals at once:

  v_1, v_2, ...: v_t the smallest vertex of minimum degree d_t of H_{t-1} = H - {v_1..v_{t-1}},
  taken while |H_{t-1}| > s_post, d_t < k(|H_{t-1}|) and d_1 <= d_2 <= ... (a removal that
  would leave a degree below d_t ends the run before it);

and accepts it when lambda(H_P) >= d_P for the set left after P steps.  Then every step
is the canonical cut: adding back a vertex of degree d to a graph of connectivity c gives
connectivity >= min(c, d), so lambda(H_{t-1}) >= min(lambda(H_P), d_t, ..., d_P) = d_t, and
lambda <= minimum degree gives equality.

Ears: at degree 2 a removal may leave neighbours of degree 1 when they start paths of
degree-2 vertices.  The one-at-a-time process peels those paths right after v (cuts of 1,
smallest leaf first) and stops at their ends z, which must keep degree >= 2.  The set
before v is the set after the paths plus an ear, whose connectivity is at least
min(that set's connectivity, 2); so v's cut is 2 when the rest of the run ends in a set
certified at its largest class degree.  A path back to v (the set is a cycle), an end
falling below degree 2 (a bridge hangs there), or a path leaving s_post or fewer vertices
ends the run before v.

This test replays WCC with these shortcuts in plain Python (the accepted run's records
written at once, the rest through the oracle's cut) and compares every split record and
saved set with the oracle's PAPER-mode WCC."""
import numpy as np
import pytest

import oracle
from graphs import csr_from_edges


def _induced(off, adj, verts):
    loc = {v: i for i, v in enumerate(verts)}
    rows = [sorted(loc[u] for u in adj[off[v]:off[v + 1]] if u in loc) for v in verts]
    o = np.zeros(len(verts) + 1, np.int64)
    for i, r in enumerate(rows):
        o[i + 1] = o[i] + len(r)
    a = np.array([x for r in rows for x in r], np.int32)
    return o, a, rows


def _propose_run(rows, k_of, s_post, ears=True, counts=None):
    """The run of minimum-degree removals (local ids) and their degrees (1 for the path
    vertices peeled after an ear's vertex)."""
    n = len(rows)
    deg = np.array([len(r) for r in rows])
    alive = np.ones(n, bool)
    order, ds = [], []
    size, dc = n, int(deg.min())
    ears = ears and k_of(s_post + 1) >= 2       # the peeled path vertices fail their cut

    def remove(u, d):
        nonlocal size
        for x in rows[u]:
            if alive[x]:
                deg[x] -= 1
        alive[u] = False
        order.append(u)
        ds.append(d)
        size -= 1

    while size > s_post and dc < k_of(size):
        cands = [v for v in range(n) if alive[v] and deg[v] == dc]
        if not cands:
            dc += 1
            continue
        v = min(cands)
        if any(alive[w] and deg[w] - 1 < dc for w in rows[v]):
            if not ears or dc != 2:
                break
            paths, loss = [], {}
            for w in rows[v]:
                if not alive[w]:
                    continue
                path, prev, x = [], v, w
                while x != v and deg[x] == 2:
                    path.append(x)
                    prev, x = x, next(y for y in rows[x] if alive[y] and y != prev)
                if x == v:
                    break
                loss[x] = loss.get(x, 0) + 1
                paths.append(path)
            if (len(paths) < 2 or any(deg[z] - l < 2 for z, l in loss.items())
                    or size - 1 - sum(len(p) for p in paths) <= s_post):
                break
            remove(v, 2)
            while any(paths):
                p = min((p for p in paths if p), key=lambda p: p[0])
                remove(p.pop(0), 1)
            if counts is not None:
                counts["ears"] += 1
            continue
        remove(v, dc)
    return order, ds, alive


def _wcc_with_runs(off, adj, crit, s_post, counts, ears=True):
    k_of = lambda n: oracle.threshold(n, crit)
    recs, saved = [], []
    comp = oracle.components(off, adj)
    queue = [sorted(np.nonzero(comp == c)[0].tolist()) for c in np.unique(comp)]
    queue = [q for q in queue if len(q) > s_post]
    while queue:
        X = queue.pop()
        n = len(X)
        o, a, rows = _induced(off, adj, X)
        if len(a) == 0:
            continue
        k = k_of(n)
        if int(np.diff(o).min()) < k:
            order, ds, alive = _propose_run(rows, k_of, s_post, ears, counts)
            if order:
                rest = [v for v in range(n) if alive[v]]
                oo, aa, _ = _induced(o, a, rest)
                # (certified at the largest class degree: the last step may be a path vertex)
                if len(rest) <= 1 or oracle.mincut(oo, aa, max(ds))[0] >= max(ds):
                    counts["runs"] += 1
                    counts["steps"] += len(order)
                    for t in range(len(order)):
                        members = [X[v] for v in rest] + [X[u] for u in order[t:]]
                        recs.append((min(members), n - t, k_of(n - t), ds[t], 1, oracle.set_hash([X[order[t]]])))
                    if len(rest) > s_post:
                        queue.append([X[v] for v in rest])
                    continue
                counts["refuted"] += 1
        lam, side = oracle.mincut(o, a, k)
        S = [X[i] for i in range(n) if side[i]]
        recs.append((X[0], n, k, int(lam), len(S), oracle.set_hash(S)))
        if lam >= k:
            saved.append(tuple(X))
            continue
        T = [X[i] for i in range(n) if not side[i]]
        queue += [sorted(p) for p in (S, T) if len(p) > s_post]
    return sorted(recs), sorted(saved)


def _random_graph(rng):
    """A random core, periphery vertices of degree 2-6 attached to earlier vertices, short
    paths between vertices, and sometimes a second half joined by one bridge (a proposed
    run is then refuted: the set's cut is 1)."""
    n_core = int(rng.integers(15, 90))
    p = float(rng.uniform(0.1, 0.4))
    e = [(i, j) for i in range(n_core) for j in range(i + 1, n_core) if rng.random() < p]
    nxt = n_core
    for _ in range(int(rng.integers(0, 50))):
        d = int(rng.choice([2, 3, 4, 5, 6]))
        e += [(int(u), nxt) for u in rng.choice(nxt, size=min(d, nxt), replace=False)]
        nxt += 1
    for _ in range(int(rng.integers(0, 5))):
        prev = int(rng.integers(0, nxt))
        for _ in range(int(rng.integers(1, 4))):
            e.append((prev, nxt))
            prev, nxt = nxt, nxt + 1
        e.append((prev, int(rng.integers(0, n_core))))
    if rng.random() < 0.3:
        h = n_core // 2
        e += [(nxt + i, nxt + j) for i in range(h) for j in range(i + 1, h) if rng.random() < p]
        e.append((0, nxt))
        nxt += h
    perm = rng.permutation(nxt)
    return csr_from_edges(nxt, [(int(perm[a]), int(perm[b])) for a, b in e])


def _ear_graph(rng):
    """A random core with paths of 1-5 degree-2 vertices between core vertices, cycles
    hanging at one core vertex (whose degree decides whether the ear may be taken), a
    triangle hanging by a bridge, and periphery vertices of degree 2-3."""
    n_core = int(rng.integers(40, 120))
    p = float(rng.uniform(0.1, 0.3))
    e = [(i, j) for i in range(n_core) for j in range(i + 1, n_core) if rng.random() < p]
    nxt = n_core
    for _ in range(int(rng.integers(5, 30))):
        a, b = (int(x) for x in rng.choice(n_core, 2, replace=False))
        prev = a
        for _ in range(int(rng.integers(1, 6))):
            e.append((prev, nxt))
            prev, nxt = nxt, nxt + 1
        e.append((prev, b))
    for _ in range(int(rng.integers(0, 3))):
        a = int(rng.integers(0, n_core))
        ring = list(range(nxt, nxt + int(rng.integers(3, 7))))
        e += [(a, ring[0]), (a, ring[-1])] + list(zip(ring[:-1], ring[1:]))
        nxt += len(ring)
    if rng.random() < 0.4:
        a = int(rng.integers(0, n_core))
        e += [(a, nxt), (nxt, nxt + 1), (nxt + 1, nxt + 2), (nxt + 2, nxt)]
        nxt += 3
    for _ in range(int(rng.integers(0, 20))):
        d = int(rng.choice([2, 3]))
        e += [(int(u), nxt) for u in rng.choice(nxt, size=min(d, nxt), replace=False)]
        nxt += 1
    perm = rng.permutation(nxt)
    return csr_from_edges(nxt, [(int(perm[a]), int(perm[b])) for a, b in e])


@pytest.mark.parametrize("crit", ["log10", "log2", "sqrt"])
def test_certified_runs_equal_one_cut_at_a_time(crit):
    rng = np.random.default_rng({"log10": 21, "log2": 22, "sqrt": 23}[crit])
    counts = {"runs": 0, "steps": 0, "refuted": 0, "ears": 0}
    for _ in range(40):
        off, adj = _random_graph(rng)
        memb = np.zeros(len(off) - 1, np.int32)
        want, wrec = oracle.wcc(off, adj, memb, mode="paper", criterion=crit, s_pre=10, s_post=10, nthreads=1)
        wkey = sorted(tuple(int(q[f]) for f in ("minv", "n", "k", "lam", "ssize", "shash")) for q in wrec)
        got, saved = _wcc_with_runs(off, adj, crit, 10, counts)
        assert got == wkey
        sets = {}
        for v in np.nonzero(want >= 0)[0]:
            sets.setdefault(int(want[v]), []).append(int(v))
        assert sorted(tuple(s) for s in sets.values()) == saved
    # the shortcut was taken, with runs of several steps, and refuted at least once
    assert counts["runs"] > 10 and counts["steps"] > 2 * counts["runs"], counts
    if crit == "log10":
        assert counts["refuted"] > 0, counts


@pytest.mark.parametrize("crit", ["log10", "log2"])
def test_certified_ears_equal_one_cut_at_a_time(crit):
    rng = np.random.default_rng({"log10": 31, "log2": 32}[crit])
    counts = {"runs": 0, "steps": 0, "refuted": 0, "ears": 0}
    for _ in range(40):
        off, adj = _ear_graph(rng)
        memb = np.zeros(len(off) - 1, np.int32)
        want, wrec = oracle.wcc(off, adj, memb, mode="paper", criterion=crit, s_pre=10, s_post=10, nthreads=1)
        wkey = sorted(tuple(int(q[f]) for f in ("minv", "n", "k", "lam", "ssize", "shash")) for q in wrec)
        got, saved = _wcc_with_runs(off, adj, crit, 10, counts)
        assert got == wkey
        sets = {}
        for v in np.nonzero(want >= 0)[0]:
            sets.setdefault(int(want[v]), []).append(int(v))
        assert sorted(tuple(s) for s in sets.values()) == saved
    assert counts["ears"] > 100 and counts["refuted"] > 0, counts
