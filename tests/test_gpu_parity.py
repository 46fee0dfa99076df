"""Parity of the HIP path (through the C ABI) with the CPU oracle: bit-exact compacted
subgraphs, cut values and sides, split records and final membership."""
import numpy as np
import pytest

import gen
import oracle
from graphs import complete, csr_from_edges, cycle, random_connected, random_tree

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _w():
    import paper_2509_02590_amd as w
    return w


def _t(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else a.astype(dtype))
    return torch.from_numpy(a).to(_dev())


def _run(off, adj, memb, offsets32=True, **kw):
    w = _w()
    o = _t(off, np.int32 if offsets32 else np.int64)
    out, st, rec = w.wcc_run(o, _t(adj, np.int32), _t(memb, np.int32), records_cap=2 * len(memb) + 16, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), st, rec


def _rec_key(r):
    return sorted(tuple(int(x) for x in (q["minv"], q["n"], q["k"], q["lam"], q["ssize"], q["shash"])) for q in r)


def _compare(off, adj, memb, s_pre=10, s_post=10, mode="kcore", offsets32=True, criterion="log10"):
    want, wrec = oracle.wcc(off, adj, memb, s_pre=s_pre, s_post=s_post, mode=mode, criterion=criterion)
    got, st, grec = _run(off, adj, memb, offsets32=offsets32, s_pre=s_pre, s_post=s_post, mode=mode,
                         criterion=criterion)
    assert np.array_equal(got, want), "membership differs (%d of %d)" % ((got != want).sum(), len(want))
    assert _rec_key(grec) == _rec_key(wrec)
    return st


# ------------------------------------------------------------------ compaction
@pytest.mark.parametrize("which", ["tiny", "chunglu_small"])
def test_cluster_csr_matches_oracle(which):
    g = gen.c0() if which == "tiny" else gen.chung_lu(30000, 30.0, 2.5, 11, 800, 2.0, 0.2, 0.15, 0.05, seed=9)
    memb = g.membership.copy()
    memb[::17] = -1                                  # some unassigned vertices
    memb = np.where(memb >= 0, memb * 7 + 3, memb)   # non-dense cluster ids
    want = oracle.cluster_csr(g.offsets, g.indices, memb)
    w = _w()
    got = w.cluster_csr(_t(g.offsets), _t(g.indices), _t(memb, np.int32))
    got = {k: v.cpu().numpy() for k, v in got.items()}
    for k in ("cl_ids", "cl_start", "vert", "row_off"):
        assert np.array_equal(got[k], want[k]), k
    ro = want["row_off"]
    ga = got["adj"].copy()
    for i in range(len(ro) - 1):
        ga[ro[i]:ro[i + 1]].sort()                   # row order is unspecified
    assert np.array_equal(ga, want["adj"])


# ------------------------------------------------------------------ min cut
def _pack(graphs):
    """Disjoint union of (n, edges) graphs -> CSR, verts, set offsets."""
    edges, base, so = [], 0, [0]
    for n, e in graphs:
        edges += [(a + base, b + base) for a, b in e]
        base += n
        so.append(base)
    off, adj = csr_from_edges(base, edges)
    return off, adj, np.arange(base, dtype=np.int32), np.array(so, np.int64)


def test_mincut_split_batch_random_small():
    rng = np.random.default_rng(4242)
    graphs = []
    for i in range(600):
        n = int(rng.integers(2, 40))
        p = float(rng.choice([0.08, 0.2, 0.5, 0.9]))
        graphs.append((n, random_connected(rng, n, p)))
    graphs += [(12, complete(12)), (30, cycle(30)), (25, random_tree(rng, 25)), (1, []), (2, [])]
    off, adj, verts, so = _pack(graphs)
    caps = rng.integers(1, 8, len(graphs)).astype(np.int32)
    caps[::5] = 2**31 - 1
    caps[-6:] = [3, 2**31 - 1, 2, 2, 2, 2]
    w = _w()
    lam, side = w.mincut_split_batch(_t(off, np.int32), _t(adj), _t(verts), _t(so), _t(caps))
    lam, side = lam.cpu().numpy(), side.cpu().numpy().astype(bool)
    for i, (n, e) in enumerate(graphs):
        wl, ws = oracle.mincut_split(off, adj, verts[so[i]:so[i + 1]], int(caps[i]))
        assert lam[i] == wl, (i, n)
        assert np.array_equal(side[so[i]:so[i + 1]], ws), (i, n)


def test_mincut_split_single_and_disconnected():
    w = _w()
    e = complete(6) + [(a + 6, b + 6) for a, b in complete(5)]
    off, adj = csr_from_edges(11, e)
    lam, side = w.mincut_split(_t(off), _t(adj), _t(np.arange(11), np.int32), 3)
    assert lam == 0 and side.cpu().numpy().astype(bool).tolist() == [True] * 6 + [False] * 5
    lam, side = w.mincut_split(_t(off), _t(adj), _t(np.arange(6, 11), np.int32), 2**31 - 1)
    assert lam == 4 and side.cpu().numpy().tolist() == [1, 0, 0, 0, 0]


def _cert_graph(rng):
    """Clusters that reach the spanning-forest certificate in every way: dense ones it
    certifies, sparse ones with fewer edges than the certificate needs, two dense halves
    joined by fewer bridges than k (the certificate must fail and the scan split them),
    and complete bipartite ones whose cut equals their minimum degree."""
    parts, base = [], 0
    def add(n, edges):
        nonlocal base
        parts.append((base, n, [(a + base, b + base) for a, b in edges]))
        base += n
    for n in (12, 20, 33, 60):
        add(n, complete(n))
    for n in (40, 120):
        ring = cycle(n) + [(i, (i + n // 2) % n) for i in range(0, n, 7)]
        add(n, sorted({(min(a, b), max(a, b)) for a, b in ring if a != b}))
    for h, b in ((15, 1), (30, 2), (60, 2)):
        e = complete(h) + [(a + h, c + h) for a, c in complete(h)]
        e += [(int(rng.integers(0, h)), int(rng.integers(h, 2 * h))) for _ in range(b)]
        add(2 * h, sorted(set(e)))
    for a, b in ((6, 9), (12, 14)):
        add(a + b, [(i, a + j) for i in range(a) for j in range(b)])
    memb = np.concatenate([np.full(n, i, np.int32) for i, (_, n, _) in enumerate(parts)])
    edges = [e for _, _, es in parts for e in es]
    # a few edges between clusters
    for _ in range(40):
        u, v = rng.integers(0, base, 2)
        if memb[u] != memb[v]:
            edges.append((int(min(u, v)), int(max(u, v))))
    off, adj = csr_from_edges(base, sorted(set(edges)))
    return off, adj, memb


@pytest.mark.parametrize("mode", ["kcore", "paper"])
def test_certificate_and_scan_paths(mode):
    """Items ended by the certificate, items too sparse for it, and items it cannot
    certify (lambda below the bound) all give the oracle's membership and records."""
    rng = np.random.default_rng(303 if mode == "kcore" else 304)
    off, adj, memb = _cert_graph(rng)
    for crit in ("log10", "log2"):
        st = _compare(off, adj, memb, mode=mode, criterion=crit)
        assert st.mincuts > 0


# ------------------------------------------------------------------ whole WCC
@pytest.mark.parametrize("mode", ["kcore", "paper"])
def test_wcc_tiny_workload(mode):
    g = gen.c0()
    st = _compare(g.offsets, g.indices, g.membership, mode=mode)
    assert st.accepted > 0


@pytest.mark.parametrize("mode", ["kcore", "paper"])
def test_wcc_random_clustered(mode):
    rng = np.random.default_rng(55 if mode == "kcore" else 56)
    for trial in range(12):
        n = int(rng.integers(50, 400))
        nclust = int(rng.integers(1, 8))
        memb = rng.integers(-1, nclust, n).astype(np.int32)
        edges = set()
        for a in range(n):
            for b in range(a + 1, n):
                same = memb[a] == memb[b] and memb[a] >= 0
                if rng.random() < (float(rng.choice([0.1, 0.3])) if same else 0.01):
                    edges.add((a, b))
        off, adj = csr_from_edges(n, sorted(edges))
        for s in (1, 5, 10):
            _compare(off, adj, memb, s_pre=s, s_post=s, mode=mode)


def test_wcc_special_cases():
    # two K11 joined by a bridge; K_n; tree; disjoint union; cycle with a pendant
    e = complete(11) + complete(11, 11) + [(10, 11)]
    off, adj = csr_from_edges(22, e)
    for s in (10, 11):
        for mode in ("kcore", "paper"):
            _compare(off, adj, np.zeros(22, np.int32), s_pre=s, s_post=s, mode=mode)
    e = cycle(99) + [(98, 99)]
    off, adj = csr_from_edges(100, e)
    for mode in ("kcore", "paper"):
        _compare(off, adj, np.zeros(100, np.int32), mode=mode)
    rng = np.random.default_rng(2)
    off, adj = csr_from_edges(60, random_tree(rng, 60))
    _compare(off, adj, np.zeros(60, np.int32), mode="paper")


def test_wcc_edge_cases():
    w = _w()
    # empty graph
    out, st, _ = _run(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert out.shape == (0,)
    # no edges at all
    memb = np.zeros(50, np.int32)
    got, _, _ = _run(np.zeros(51, np.int64), np.zeros(0, np.int32), memb)
    assert np.all(got == -1)
    # everything unassigned
    off, adj = csr_from_edges(30, complete(30))
    got, _, _ = _run(off, adj, np.full(30, -1, np.int32))
    assert np.all(got == -1)
    # large cluster ids and 64-bit offsets
    memb = np.full(30, 2**31 - 2, np.int32)
    _compare(off, adj, memb, offsets32=False)
    # invalid parameters are rejected
    with pytest.raises(w.WccError):
        _run(off, adj, memb, s_post=-1)


def test_wcc_validate_flag():
    w = _w()
    off, adj = csr_from_edges(20, complete(20))
    memb = np.zeros(20, np.int32)
    _run(off, adj, memb, validate=True)
    bad = adj.copy()
    bad[0] = 0  # self-loop on vertex 0
    with pytest.raises(w.WccError) as ei:
        _run(off, bad, memb, validate=True)
    assert ei.value.code == -2
    bad = adj.copy()
    bad[5] = (bad[5] + 1) % 20 if bad[5] != 19 else 18   # asymmetric entry
    with pytest.raises(w.WccError):
        _run(off, bad, memb, validate=True)


@pytest.mark.parametrize("mode", ["kcore", "paper"])
def test_wcc_chunglu_medium(mode):
    g = gen.chung_lu(60000, 30.0, 2.5, 11, 2000, 2.0, 0.2, 0.15, 0.05, seed=77, intra_mult=1.8)
    _compare(g.offsets, g.indices, g.membership, mode=mode)


def test_wcc_c1_full_kcore():
    """The 1M-vertex / 20M-edge workload in the benchmark's launch configuration."""
    g = gen.c1()
    st = _compare(g.offsets, g.indices, g.membership, mode="kcore")
    assert st.mincuts > 1000


def _multi_component_clusters(rng, specs, n_free=50):
    """Clusters made of several disjoint components (a ring plus random chords each), the
    vertices of all clusters spread over the id range by a random permutation, so that the
    components of a cluster interleave in its local ids.  specs: (components, size, extra
    chords per vertex) per cluster."""
    n = sum(c * sz for c, sz, _ in specs) + n_free
    perm = rng.permutation(n)
    memb = np.full(n, -1, np.int32)
    edges = []
    pos = 0
    for cl, (c, sz, extra) in enumerate(specs):
        for _ in range(c):
            ids = perm[pos:pos + sz]
            pos += sz
            memb[ids] = cl
            for i in range(sz):
                edges.append((ids[i], ids[(i + 1) % sz]))
            for _ in range(int(extra * sz)):
                a, b = rng.integers(0, sz, 2)
                edges.append((ids[a], ids[b]))
    # a few inter-cluster edges (never inside one cluster: the components stay apart) and
    # unassigned vertices
    for _ in range(n // 20):
        a, b = rng.integers(0, n, 2)
        if memb[a] != memb[b] or memb[a] < 0:
            edges.append((a, b))
    off, adj = csr_from_edges(n, edges)
    return off, adj, memb


@pytest.mark.parametrize("exec_mode", ["plain", "batched"])
def test_rebuild_child_placement(exec_mode):
    """Children placed by the packed block scan (up to four per split) and by the
    single-wavefront walk (more), with state in LDS and, for clusters above the LDS
    budget, in global memory; the components interleave in each cluster's local ids, so
    the stable new positions are exercised; against the oracle."""
    # (PAPER mode on denser components: sparse ones lose their degree-2 vertices one cut
    # at a time, which the oracle replays slowly)
    cases = (("kcore", 404, [(4, 30, 1.5), (7, 25, 1.5), (1, 40, 1.5), (3, 4000, 3.0), (6, 2500, 3.0),
                             (9, 1800, 3.0)]),
             ("paper", 405, [(4, 30, 3.0), (7, 25, 3.0), (3, 3000, 6.0), (6, 1600, 6.0)]))
    for mode, seed, specs in cases:
        off, adj, memb = _multi_component_clusters(np.random.default_rng(seed), specs)
        want, wrec = oracle.wcc(off, adj, memb, mode=mode)
        got, st, grec = _run(off, adj, memb, mode=mode, exec_mode=exec_mode)
        assert np.array_equal(got, want), mode
        assert _rec_key(grec) == _rec_key(wrec), mode
        assert len(np.unique(want[want >= 0])) > 10


@pytest.mark.parametrize("exec_mode", ["plain", "batched"])
def test_wcc_global_state_items(exec_mode):
    """Items whose scan state does not fit the large bin's LDS run from global memory:
    forced here by tiny LDS budgets, checked against the oracle."""
    w = _w()
    g = gen.chung_lu(60000, 30.0, 2.5, 11, 2000, 2.0, 0.2, 0.15, 0.05, seed=77, intra_mult=1.8)
    try:
        w.set_exec_config(small_lds_kb=4, big_lds_kb=4, big_max_pct=50)
        # (log2 gives bounds of 5-11: the one-pass certificate takes bounds up to 4, the
        # forest-per-pass certificate the larger ones)
        for mode, crit in (("kcore", "log10"), ("paper", "log10"), ("kcore", "log2")):
            want, wrec = oracle.wcc(g.offsets, g.indices, g.membership, mode=mode, criterion=crit)
            got, st, grec = _run(g.offsets, g.indices, g.membership, mode=mode, criterion=crit,
                                 exec_mode=exec_mode, graph=False)
            assert np.array_equal(got, want), (mode, crit)
            assert _rec_key(grec) == _rec_key(wrec)
    finally:
        w.set_exec_config()


def _ccr_expected(off, adj, memb):
    """Components of the intra-cluster graph by the oracle (smallest vertex; -1 unassigned)."""
    n = len(memb)
    off = np.asarray(off, np.int64)
    src = np.repeat(np.arange(n), np.diff(off))
    keep = (memb[src] >= 0) & (memb[src] == memb[adj])
    off2 = np.concatenate([[0], np.cumsum(np.bincount(src[keep], minlength=n))]).astype(np.int64)
    return oracle.components(off2, np.asarray(adj)[keep].astype(np.int32), alive=(memb >= 0))


def test_ccr_components_match_oracle():
    w = _w()
    rng = np.random.default_rng(31)
    cases = []
    for trial in range(6):
        n = int(rng.integers(50, 500))
        memb = rng.integers(-1, 6, n).astype(np.int32) * 5 + 2
        memb[memb < 0] = -1
        edges = {(a, b) for a in range(n) for b in range(a + 1, n) if rng.random() < 0.02}
        off, adj = csr_from_edges(n, sorted(edges))
        cases.append((off, adj, memb))
    g = gen.chung_lu(60000, 30.0, 2.5, 11, 2000, 2.0, 0.2, 0.15, 0.05, seed=78, intra_mult=1.8)
    memb = g.membership.copy()
    memb[::23] = -1
    cases.append((g.offsets, g.indices, memb))
    c0 = gen.c0()
    cases.append((c0.offsets, c0.indices, c0.membership))
    for off, adj, memb in cases:
        got = w.ccr_components(_t(off, np.int32), _t(adj, np.int32), _t(memb, np.int32)).cpu().numpy()
        assert np.array_equal(got, _ccr_expected(off, adj, memb))


def _hanging_trees_graph(rng, n_core, n_tree_vertices, clusters=3):
    """Clusters made of a dense-enough core (a cycle with chords) plus hanging trees of
    every shape (paths, stars, random trees) attached to core vertices, a few pure trees
    and a long pendant path: every PAPER-mode item starts with vertices of degree 1."""
    edges, memb, base = [], [], 0
    for c in range(clusters):
        core = list(range(base, base + n_core))
        edges += [(core[i], core[(i + 1) % n_core]) for i in range(n_core)]
        edges += [(core[i], core[(i + 7) % n_core]) for i in range(0, n_core, 3)]
        nxt = base + n_core
        verts = list(core)
        while nxt < base + n_core + n_tree_vertices:
            kind = int(rng.integers(0, 3))
            size = int(rng.integers(1, 12))
            root = int(rng.choice(verts))
            new = list(range(nxt, nxt + size))
            if kind == 0:    # a path
                chain = [root] + new
                edges += list(zip(chain[:-1], chain[1:]))
            elif kind == 1:  # a star
                edges += [(root, new[0])] + [(new[0], x) for x in new[1:]]
            else:            # a random tree
                pool = [root]
                for x in new:
                    edges.append((int(rng.choice(pool)), x))
                    pool.append(x)
            verts += new
            nxt += size
        memb += [c] * (nxt - base)
        base = nxt
    # a pure tree cluster and a core with one long pendant path
    tree = [(base + i, base + int(rng.integers(0, i))) for i in range(1, 40)]
    edges += tree
    memb += [clusters] * 40
    base += 40
    edges += [(base + i, base + (i + 1) % 12) for i in range(12)] + [(base + 11 + i, base + 12 + i) for i in range(300)]
    memb += [clusters + 1] * 312
    base += 312
    # a shuffled labelling so that ids do not follow the tree structure
    perm = rng.permutation(base)
    edges = [(int(perm[a]), int(perm[b])) for a, b in edges]
    memb_p = np.empty(base, np.int32)
    memb_p[perm] = np.array(memb, np.int32)
    off, adj = csr_from_edges(base, edges)
    return off, adj, memb_p


@pytest.mark.parametrize("crit", ["log10", "log2"])
def test_paper_leaf_runs(crit):
    """PAPER mode on items with hanging trees: the removal of vertices of degree 1 one at a
    time (each a split record) is computed by the GPU in one batch whenever every step
    fails its cut, and by single steps otherwise; both against the oracle."""
    rng = np.random.default_rng(808 if crit == "log10" else 809)
    for trial in range(3):
        off, adj, memb = _hanging_trees_graph(rng, int(rng.integers(15, 60)), int(rng.integers(50, 400)))
        for s in (1, 3, 9, 10, 25):
            st = _compare(off, adj, memb, s_pre=s, s_post=s, mode="paper", criterion=crit)
            assert st.mincuts > 0


def test_wcc_c1_full_paper():
    """The 1M-vertex / 20M-edge workload in PAPER mode (runs of single-vertex splits)."""
    g = gen.c1()
    st = _compare(g.offsets, g.indices, g.membership, mode="paper")
    assert st.mincuts > 1000


def _low_degree_clusters(rng, n_clusters):
    """Clusters on which PAPER mode removes vertices of the minimum degree (>= 2) one split
    at a time: a random core with periphery vertices of degree 2-6 attached to earlier
    vertices and short paths between vertices (their inner vertices end runs early); some
    carry a second half joined by one bridge, so that a proposed run is refuted by its
    certificate (the item's cut is 1, below its minimum degree)."""
    edges, memb, base = [], [], 0
    for c in range(n_clusters):
        n_core = int(rng.integers(20, 160))
        p = float(rng.uniform(0.08, 0.4))
        e = [(i, j) for i in range(n_core) for j in range(i + 1, n_core) if rng.random() < p]
        nxt = n_core
        for _ in range(int(rng.integers(0, 80))):
            d = int(rng.choice([2, 3, 4, 5, 6]))
            e += [(int(u), nxt) for u in rng.choice(nxt, size=min(d, nxt), replace=False)]
            nxt += 1
        for _ in range(int(rng.integers(0, 6))):
            prev = int(rng.integers(0, nxt))
            for _ in range(int(rng.integers(1, 5))):
                e.append((prev, nxt))
                prev, nxt = nxt, nxt + 1
            e.append((prev, int(rng.integers(0, n_core))))
        if rng.random() < 0.3:
            h = n_core // 2
            e += [(nxt + i, nxt + j) for i in range(h) for j in range(i + 1, h) if rng.random() < p]
            e.append((0, nxt))
            nxt += h
        perm = rng.permutation(nxt)
        edges += [(base + int(perm[a]), base + int(perm[b])) for a, b in e if a != b]
        memb += [c] * nxt
        base += nxt
    for _ in range(base // 20):   # edges between clusters (dropped by the compaction)
        u, v = rng.integers(0, base, 2)
        if memb[u] != memb[v]:
            edges.append((int(u), int(v)))
    off, adj = csr_from_edges(base, edges)
    return off, adj, np.array(memb, np.int32)


def _waiting_overflow_cluster(n_pairs=100, n_core=200, p=0.3, seed=5):
    """One cluster whose run at degree 2 makes more than 64 vertices wait to enter the
    degree class: vertices 0..n_pairs-1 (degree 2) each join a vertex of degree 3 with a
    larger id and a core vertex; removing them lowers those to degree 2 while the class
    list still holds smaller ids.  PAPER mode removes all 2 * n_pairs one at a time."""
    rng = np.random.default_rng(seed)
    lo, hi, core = 0, n_pairs, 2 * n_pairs
    e = [(core + i, core + j) for i in range(n_core) for j in range(i + 1, n_core) if rng.random() < p]
    for i in range(n_pairs):
        c1, c2, c3 = (core + int(x) for x in rng.choice(n_core, 3, replace=False))
        e += [(lo + i, hi + i), (lo + i, c1), (hi + i, c2), (hi + i, c3)]
    off, adj = csr_from_edges(core + n_core, e)
    return off, adj, np.zeros(core + n_core, np.int32)


def _ear_clusters(rng, n_clusters):
    """Clusters from the CPU run test's ear graphs (paths of degree-2 vertices between core
    vertices, cycles hanging at one vertex, a triangle hanging by a bridge), joined into
    one graph with a few edges between clusters."""
    from test_low_runs import _ear_graph
    edges, memb, base = [], [], 0
    for c in range(n_clusters):
        off, adj = _ear_graph(rng)
        n = len(off) - 1
        edges += [(base + u, base + int(adj[e])) for u in range(n) for e in range(off[u], off[u + 1])
                  if u < adj[e]]
        memb += [c] * n
        base += n
    for _ in range(base // 30):
        u, v = rng.integers(0, base, 2)
        if memb[u] != memb[v]:
            edges.append((int(u), int(v)))
    off, adj = csr_from_edges(base, edges)
    return off, adj, np.array(memb, np.int32)


@pytest.mark.parametrize("crit", ["log10", "log2", "sqrt"])
def test_paper_low_runs(crit):
    """PAPER mode: runs of single-vertex splits at the minimum degree (>= 2), computed in
    one batch and certified by spanning forests of the rest, against the oracle's one cut
    at a time; with item state in LDS and in global memory, in both execution forms."""
    w = _w()
    rng = np.random.default_rng({"log10": 910, "log2": 911, "sqrt": 912}[crit])
    cases = [_low_degree_clusters(rng, 40) for _ in range(2)]
    if crit != "sqrt":
        cases.append(_ear_clusters(rng, 40))
    overflow = -1
    if crit == "log10":
        overflow = len(cases)
        cases.append(_waiting_overflow_cluster())
    for i, (off, adj, memb) in enumerate(cases):
        want, wrec = oracle.wcc(off, adj, memb, mode="paper", criterion=crit)
        for exec_mode, tiny_lds in (("plain", False), ("batched", False), ("plain", True)):
            try:
                if tiny_lds:
                    w.set_exec_config(small_lds_kb=4, big_lds_kb=4, big_max_pct=50)
                got, st, grec = _run(off, adj, memb, mode="paper", criterion=crit, exec_mode=exec_mode,
                                     graph=False)
            finally:
                w.set_exec_config()
            assert np.array_equal(got, want), (i, exec_mode, tiny_lds)
            assert _rec_key(grec) == _rec_key(wrec), (i, exec_mode, tiny_lds)
            if i == overflow:
                # 200 single-vertex splits in a handful of levels: the run was taken
                assert len(wrec) > 200 and st.levels < 10, (len(wrec), st.levels)
