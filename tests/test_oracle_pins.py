"""Pins of the CPU oracle against facts that do not come from the oracle itself:
exact definitions, brute-force enumeration, closed forms, library routines, an
independent Stoer-Wagner, hand traces and independent drivers of Alg. 1-3."""
import json
import math
import os
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import gen
import oracle
from graphs import (all_subsets, brute_force_cuts, complete, complete_bipartite, csr_from_edges,
                    cut_value, cycle, edges_of, hypercube, is_connected, path, random_connected,
                    random_tree, stoer_wagner, two_cliques)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
INF = 2**31 - 1


# ------------------------------------------------------------------ criterion k(n)
def _k_by_definition(n, crit, num=1, den=1):
    """Least integer c with c > f(n), found by counting up and testing c > f(n) exactly."""
    c = 0
    while True:
        if crit == "log10" and 10 ** c > n:        # c > log10 n  <=>  10^c > n
            return c
        if crit == "log2" and 2 ** c > n:          # c > log2 n   <=>  2^c > n
            return c
        if crit == "sqrt" and c * c > n:           # c > sqrt n   <=>  c^2 > n (c >= 0)
            return c
        if crit == "linear" and Fraction(c) > Fraction(num * n, den):
            return c
        c += 1


@pytest.mark.parametrize("crit", ["log10", "log2", "sqrt"])
def test_threshold_matches_definition(crit):
    ns = list(range(1, 2000)) + [9, 10, 11, 99, 100, 101, 999, 1000, 1001, 10**6 - 1, 10**6,
                                  10**6 + 1, 2**20 - 1, 2**20, 2**20 + 1, 65535, 65536, 65537]
    for n in ns:
        assert oracle.threshold(n, crit) == _k_by_definition(n, crit), (crit, n)


def test_threshold_linear():
    for num, den in [(1, 1), (1, 2), (3, 10), (0, 1), (7, 3)]:
        for n in range(1, 300):
            assert oracle.threshold(n, "linear", num, den) == _k_by_definition(n, "linear", num, den)


def test_threshold_log10_agrees_with_libm_below_1e15():
    # the float rule "cut > log10(n)" of Alg. 3 and the integer rule agree wherever
    # double precision resolves log10 (checked on boundaries and random n)
    rng = np.random.default_rng(7)
    ns = [10**j + d for j in range(15) for d in (-1, 0, 1) if 10**j + d >= 1]
    ns += [int(x) for x in rng.integers(1, 10**15, 2000)]
    for n in ns:
        k = oracle.threshold(n, "log10")
        assert k > math.log10(n) and k - 1 <= math.log10(n), n


# ------------------------------------------------------------------ min cut: brute force
def _check_cut_against_bruteforce(n, edges, cap):
    off, adj = csr_from_edges(n, edges)
    masks, vals = brute_force_cuts(n, edges)
    lam = int(vals.min())
    got, side = oracle.mincut(off, adj, cap)
    assert got == min(lam, cap), (n, edges, cap)
    deg = np.diff(off)
    if lam < cap:
        # S must be a minimum cut, both sides non-empty and connected (a min cut of a
        # connected graph has connected sides)
        assert 0 < side.sum() < n
        assert cut_value(edges, side) == lam
        assert is_connected(n, edges, np.flatnonzero(side))
        assert is_connected(n, edges, np.flatnonzero(~side))
    if deg.min() <= cap and lam == deg.min():
        # nothing beats the degree pre-pass: S is the smallest vertex of minimum degree
        assert np.flatnonzero(side).tolist() == [int(np.argmin(deg))]
    if deg.min() > cap:
        assert got == cap


def test_mincut_bruteforce_random():
    rng = np.random.default_rng(12345)
    for trial in range(400):
        n = int(rng.integers(2, 15))
        p = float(rng.choice([0.1, 0.25, 0.5, 0.8]))
        edges = random_connected(rng, n, p)
        for cap in (INF, int(rng.integers(1, 6))):
            _check_cut_against_bruteforce(n, edges, cap)


def test_mincut_bruteforce_bridged_blocks():
    rng = np.random.default_rng(99)
    for trial in range(150):
        a = int(rng.integers(3, 8))
        b = int(rng.integers(3, 8))
        e1 = random_connected(rng, a, 0.7)
        e2 = [(x + a, y + a) for x, y in random_connected(rng, b, 0.7)]
        nb = int(rng.integers(1, 4))
        br = {(int(rng.integers(0, a)), a + int(rng.integers(0, b))) for _ in range(nb)}
        edges = sorted(set(e1 + e2 + list(br)))
        _check_cut_against_bruteforce(a + b, edges, INF)


def test_mincut_all_small_graphs_exhaustive():
    # every connected graph on 5 labelled vertices
    n = 5
    pairs = [(a, b) for a in range(n) for b in range(a + 1, n)]
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        if not is_connected(n, edges):
            continue
        _check_cut_against_bruteforce(n, edges, INF)
        _check_cut_against_bruteforce(n, edges, 2)


# ------------------------------------------------------------------ min cut: closed forms
def _lam(n, edges, cap=INF):
    off, adj = csr_from_edges(n, edges)
    return oracle.mincut(off, adj, cap)


def test_closed_forms():
    rng = np.random.default_rng(3)
    for n in range(2, 40):
        assert _lam(n, complete(n))[0] == n - 1
        assert _lam(n, path(n))[0] == 1
        assert _lam(n, random_tree(rng, n))[0] == 1
    for n in range(3, 60):
        assert _lam(n, cycle(n))[0] == 2
    for d in range(1, 8):
        n, e = hypercube(d)
        assert _lam(n, e)[0] == d
    for a in range(1, 9):
        for b in range(1, 9):
            assert _lam(a + b, complete_bipartite(a, b))[0] == min(a, b)
    for a in range(3, 12):
        for b in range(1, a - 1):
            n, e = two_cliques(a, b)
            lam, side = _lam(n, e)
            assert lam == b
            got = sorted(np.flatnonzero(side).tolist())
            assert got in (list(range(a)), list(range(a, 2 * a)))  # one of the two cliques


def test_cap_semantics():
    # K_12 has lambda 11; capped at 4 the answer is 4 with an empty side (min degree > cap)
    lam, side = _lam(12, complete(12), 4)
    assert lam == 4 and side.sum() == 0
    # capped exactly at the min degree: the smallest min-degree vertex is recorded
    lam, side = _lam(12, complete(12), 11)
    assert lam == 11 and np.flatnonzero(side).tolist() == [0]


# ------------------------------------------------------------------ min cut: SW, networkx
def test_lambda_matches_stoer_wagner_and_networkx():
    rng = np.random.default_rng(2024)
    for trial in range(60):
        n = int(rng.integers(15, 120))
        p = float(rng.choice([0.03, 0.08, 0.2]))
        edges = random_connected(rng, n, p)
        lam = _lam(n, edges)[0]
        assert lam == stoer_wagner(n, edges)
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from(edges)
        cv, _ = nx.stoer_wagner(G)
        assert lam == cv


def test_lambda_on_bridged_power_law_blocks():
    # dense blocks with a planted sparse seam: the seam is a minimum cut
    rng = np.random.default_rng(5)
    for trial in range(20):
        a, b = int(rng.integers(20, 60)), int(rng.integers(20, 60))
        e1 = random_connected(rng, a, 0.4)
        e2 = [(x + a, y + a) for x, y in random_connected(rng, b, 0.4)]
        nb = int(rng.integers(1, 4))
        br = set()
        while len(br) < nb:
            br.add((int(rng.integers(0, a)), a + int(rng.integers(0, b))))
        edges = sorted(set(e1 + e2) | br)
        deg = np.diff(csr_from_edges(a + b, edges)[0])
        if deg.min() <= nb:
            continue
        lam, side = _lam(a + b, edges)
        assert lam == nb
        s = set(np.flatnonzero(side).tolist())
        assert s == set(range(a)) or s == set(range(a, a + b))


# ------------------------------------------------------------------ hand traces
def test_hand_traces():
    with open(os.path.join(GOLDEN, "mincut_traces.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        cap = INF if c["cap"] is None else c["cap"]
        lam, side = _lam(c["n"], [tuple(e) for e in c["edges"]], cap)
        assert lam == c["lambda"], c["name"]
        assert np.flatnonzero(side).tolist() == c["S"], c["name"]


# ------------------------------------------------------------------ k-core, components
def test_kcore_matches_networkx():
    rng = np.random.default_rng(11)
    for trial in range(60):
        n = int(rng.integers(1, 200))
        edges = [(a, b) for a, b in random_connected(rng, n, float(rng.choice([0.01, 0.05, 0.1])))] if n > 1 else []
        off, adj = csr_from_edges(n, edges)
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from(edges)
        for k in range(0, 7):
            want = set(nx.k_core(G, k).nodes()) if k > 0 else set(range(n))
            got = set(np.flatnonzero(oracle.kcore(off, adj, k)).tolist())
            assert got == want, (n, k)


def test_components_match_scipy():
    rng = np.random.default_rng(13)
    for trial in range(60):
        n = int(rng.integers(1, 300))
        m = int(rng.integers(0, 2 * n))
        edges = [(int(rng.integers(0, n)), int(rng.integers(0, n))) for _ in range(m)]
        off, adj = csr_from_edges(n, edges)
        comp = oracle.components(off, adj)
        A = sp.csr_matrix((np.ones(len(adj)), adj, off), shape=(n, n))
        nc, lab = connected_components(A, directed=False)
        # same partition, labelled by the smallest member
        for c in range(nc):
            members = np.flatnonzero(lab == c)
            assert np.all(comp[members] == members.min())


# ------------------------------------------------------------------ independent drivers
def _induced(G, U):
    return G.subgraph(U)


def _k(n):
    return oracle.threshold(n, "log10")


def _ref_wcc(n, edges, membership, s_pre, s_post, mode):
    """Alg. 1-3 written out with networkx for the set logic; the canonical cut side comes
    from the (separately pinned) oracle.mincut, its value is re-checked by Stoer-Wagner."""
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from(edges)
    clusters = {}
    for v in range(n):
        if membership[v] >= 0:
            clusters.setdefault(int(membership[v]), []).append(v)
    queue = []
    for cid, V in clusters.items():          # CCR (Alg. 1)
        H = _induced(G, V)
        if H.number_of_edges() == 0:
            continue
        for cc in nx.connected_components(H):
            if len(cc) > s_pre:
                queue.append(sorted(cc))
    saved = []
    while queue:                              # isWCC (Alg. 3), any order
        U = queue.pop()
        H = _induced(G, U)
        k = _k(len(U))
        if mode == "kcore":
            core = set(nx.k_core(H, k).nodes()) if k > 0 else set(U)
            if len(core) < len(U):
                for cc in nx.connected_components(H.subgraph(core)):
                    if len(cc) > s_post:
                        queue.append(sorted(cc))
                continue
        if H.number_of_edges() == 0:
            continue
        loc = {v: i for i, v in enumerate(U)}
        off, adj = csr_from_edges(len(U), [(loc[a], loc[b]) for a, b in H.edges()])
        lam, side = oracle.mincut(off, adj, k)
        true_lam = stoer_wagner(len(U), [(loc[a], loc[b]) for a, b in H.edges()])
        assert lam == min(true_lam, k)
        if lam >= k:
            saved.append(U)
            continue
        S = [U[i] for i in range(len(U)) if side[i]]
        T = [U[i] for i in range(len(U)) if not side[i]]
        for P in (S, T):
            if len(P) > s_post:
                queue.append(P)
    out = np.full(n, -1, np.int32)
    for lab, U in enumerate(sorted(saved, key=lambda u: u[0])):
        out[U] = lab
    return out


def _random_clustered(rng, n, nclust, p_in, p_out):
    memb = rng.integers(-1, nclust, n).astype(np.int32)
    edges = set()
    for a in range(n):
        for b in range(a + 1, n):
            p = p_in if memb[a] == memb[b] and memb[a] >= 0 else p_out
            if rng.random() < p:
                edges.add((a, b))
    return sorted(edges), memb


@pytest.mark.parametrize("mode", ["paper", "kcore"])
def test_wcc_matches_independent_driver(mode):
    rng = np.random.default_rng(77 if mode == "paper" else 78)
    for trial in range(25):
        n = int(rng.integers(20, 120))
        edges, memb = _random_clustered(rng, n, int(rng.integers(1, 5)),
                                        float(rng.choice([0.15, 0.3, 0.6])), 0.02)
        off, adj = csr_from_edges(n, edges)
        for s in (1, 3, 10):
            want = _ref_wcc(n, edges, memb, s, s, mode)
            got, _ = oracle.wcc(off, adj, memb, s_pre=s, s_post=s, mode=mode, nthreads=3)
            assert np.array_equal(got, want), (trial, s, mode)


# ------------------------------------------------------------------ special cases
def _wcc_edges(n, edges, memb, **kw):
    off, adj = csr_from_edges(n, edges)
    return oracle.wcc(off, adj, np.asarray(memb, np.int32), **kw)


@pytest.mark.parametrize("mode", ["paper", "kcore"])
def test_special_cases(mode):
    kw = dict(s_pre=10, s_post=10, mode=mode, nthreads=2)
    # K_n with n > s_post is accepted whole
    out, _ = _wcc_edges(15, complete(15), [0] * 15, **kw)
    assert np.all(out == 0)
    # a tree is dropped
    rng = np.random.default_rng(1)
    out, _ = _wcc_edges(40, random_tree(rng, 40), [0] * 40, **kw)
    assert np.all(out == -1)
    # a disjoint union is split by CCR into its parts
    e = complete(12) + complete(13, 12)
    out, _ = _wcc_edges(25, e, [0] * 25, **kw)
    assert np.all(out[:12] == 0) and np.all(out[12:] == 1)
    # unassigned vertices stay -1 and never join a set
    out, _ = _wcc_edges(25, e, [0] * 12 + [-1] * 13, **kw)
    assert np.all(out[:12] == 0) and np.all(out[12:] == -1)


@pytest.mark.parametrize("mode", ["paper", "kcore"])
def test_two_k11_golden(mode):
    with open(os.path.join(GOLDEN, "wcc_two_k11.json")) as f:
        json.load(f)
    e = complete(11) + complete(11, 11) + [(10, 11)]
    out, recs = _wcc_edges(22, e, [0] * 22, s_pre=10, s_post=10, mode=mode)
    assert out.tolist() == [0] * 11 + [1] * 11
    r = sorted(tuple(x) for x in recs.tolist())
    # the 22-set fails with cut 1 and side {0..10}; both halves pass with the cap k(11)=2
    assert [x[:5] for x in r] == [(0, 11, 2, 2, 0), (0, 22, 2, 1, 11), (11, 11, 2, 2, 0)]
    assert oracle.set_hash(np.arange(11)) == r[1][6]
    out, _ = _wcc_edges(22, e, [0] * 22, s_pre=10, s_post=11, mode=mode)
    assert np.all(out == -1)


def test_modes_differ_on_pendant_cycle():
    # a 99-cycle plus one pendant vertex, log10, s_post = 10.  PAPER peels the pendant
    # (cut 1) and accepts the 99-cycle (k(99) = 2, cut 2).  KCORE takes the 3-core of the
    # 100-set (k(100) = 3), which is empty, so nothing is saved.
    e = cycle(99) + [(98, 99)]
    out, _ = _wcc_edges(100, e, [0] * 100, s_pre=10, s_post=10, mode="paper")
    assert np.all(out[:99] == 0) and out[99] == -1
    out, _ = _wcc_edges(100, e, [0] * 100, s_pre=10, s_post=10, mode="kcore")
    assert np.all(out == -1)


# ------------------------------------------------------------------ planted bridges
def test_planted_bridges_are_cut():
    rng = np.random.default_rng(21)
    for trial in range(10):
        blocks, edges, base = [], [], 0
        for j in range(int(rng.integers(2, 5))):
            a = int(rng.integers(15, 40))
            edges += [(x + base, y + base) for x, y in random_connected(rng, a, 0.5)]
            blocks.append(list(range(base, base + a)))
            base += a
        bridges = []
        for j in range(len(blocks) - 1):   # one bridge between consecutive blocks
            u = int(rng.choice(blocks[j]))
            v = int(rng.choice(blocks[j + 1]))
            bridges.append((u, v))
        n = base
        for mode in ("paper", "kcore"):
            out, _ = _wcc_edges(n, edges + bridges, [0] * n, s_pre=10, s_post=10, mode=mode)
            for u, v in bridges:
                assert out[u] < 0 or out[u] != out[v]
            # every block is dense (min degree >= k), so each is saved whole
            for B in blocks:
                assert len(set(out[B].tolist())) == 1 and out[B[0]] >= 0


# ------------------------------------------------------------------ invariants
@pytest.mark.parametrize("mode", ["paper", "kcore"])
def test_invariants_tiny_workload(mode):
    g = gen.c0()
    out, recs = oracle.wcc(g, s_pre=10, s_post=10, mode=mode)
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    G.add_edges_from(edges_of(g.offsets, g.indices))
    labels = sorted(set(out.tolist()) - {-1})
    assert labels == list(range(len(labels)))
    mins = []
    for lab in labels:
        U = np.flatnonzero(out == lab)
        assert len(set(g.membership[U].tolist())) == 1      # subset of one input cluster
        assert len(U) > 10
        H = G.subgraph(U.tolist())
        assert nx.is_connected(H)
        cv, _ = nx.stoer_wagner(H)
        assert cv >= oracle.threshold(len(U))                # cut > log10 n
        mins.append(U.min())
    assert mins == sorted(mins)                              # canonical numbering


def test_mincut_split_semantics():
    e = complete(6) + complete(5, 6)                     # disconnected: K6 + K5
    off, adj = csr_from_edges(11, e)
    lam, side = oracle.mincut_split(off, adj, np.arange(11), 3)
    assert lam == 0 and np.flatnonzero(side).tolist() == list(range(6))
    lam, side = oracle.mincut_split(off, adj, np.arange(6, 11), 100)
    assert lam == 4 and np.flatnonzero(side).tolist() == [0]
    lam, side = oracle.mincut_split(off, adj, np.array([3]), 2)
    assert lam == 0 and side.sum() == 0


def test_cluster_csr_matches_scipy():
    rng = np.random.default_rng(31)
    n = 300
    edges, memb = _random_clustered(rng, n, 7, 0.2, 0.05)
    memb = np.where(memb >= 0, memb * 1000 + 17, memb).astype(np.int32)  # non-dense ids
    off, adj = csr_from_edges(n, edges)
    cc = oracle.cluster_csr(off, adj, memb)
    A = sp.csr_matrix((np.ones(len(adj)), adj, off), shape=(n, n))
    ids = sorted(set(memb.tolist()) - {-1})
    assert cc["cl_ids"].tolist() == ids
    for j, cid in enumerate(ids):
        V = np.flatnonzero(memb == cid)
        s, e = cc["cl_start"][j], cc["cl_start"][j + 1]
        assert cc["vert"][s:e].tolist() == V.tolist()
        sub = A[V][:, V].tocsr()
        for i in range(len(V)):
            row = cc["adj"][cc["row_off"][s + i]:cc["row_off"][s + i + 1]]
            assert row.tolist() == sorted(sub.indices[sub.indptr[i]:sub.indptr[i + 1]].tolist())
