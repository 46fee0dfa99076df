"""Pins of the oracle's Connectivity Modifier (CM, Alg. 4, and its check CMC, Alg. 5) and of
its community detection step, against facts that do not come from the oracle itself:

* with connected components as the CDA, CM equals WCC without pruning (Alg. 1-3): both
  sides of a minimum cut of a connected graph are connected (each side of a minimum cut
  is connected, else moving a detached piece back would cut fewer edges), so every part
  is one community and is "processed as a single unit", exactly as isWCC recurses;
* hand-traced label propagation (synchronous rounds, ties to the smallest label) on a
  path, on cliques, and on the worked example below;
* a hand-worked CM case where the CDA splits a part that WCC keeps whole;
* invariants of every CM output set: inside one input cluster, pairwise disjoint, larger
  than s_post, and a minimum cut of at least k(n), checked with networkx's Stoer-Wagner.
"""
import json
import os

import networkx as nx
import numpy as np
import pytest

import gen
import oracle
from graphs import complete, csr_from_edges, cycle, path

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rec_key(r):
    return sorted(tuple(int(x) for x in (q["minv"], q["n"], q["k"], q["lam"], q["ssize"], q["shash"])) for q in r)


# ------------------------------------------------------------------ label propagation
def test_labelprop_path_oscillates():
    # P3 = 0-1-2.  Round 1: 0 sees {1} -> 1, 1 sees {0, 2} (tie) -> 0, 2 sees {1} -> 1.
    # Round 2 swaps again (0 sees {0}, 1 sees {1, 1}, 2 sees {0}): the bipartite flip.
    off, adj = csr_from_edges(3, path(3))
    assert oracle.cda(off, adj, "labelprop", 0)[0].tolist() == [0, 1, 2]
    assert oracle.cda(off, adj, "labelprop", 1)[0].tolist() == [1, 0, 1]
    assert oracle.cda(off, adj, "labelprop", 2)[0].tolist() == [0, 1, 0]
    assert oracle.cda(off, adj, "labelprop", 3)[0].tolist() == [1, 0, 1]


def test_labelprop_cliques_and_isolated():
    # K_a, a >= 3: round 1 gives the smallest vertex the second-smallest label and every
    # other vertex the smallest; round 2 gives everyone the smallest label.
    # An isolated vertex keeps its own label.
    e = complete(4) + complete(3, 4) + complete(6, 7)
    off, adj = csr_from_edges(14, e)
    lab1, _ = oracle.cda(off, adj, "labelprop", 1)
    assert lab1.tolist() == [1, 0, 0, 0, 5, 4, 4, 8, 7, 7, 7, 7, 7, 13]
    for t in (2, 3, 7):
        lab, nc = oracle.cda(off, adj, "labelprop", t)
        assert lab.tolist() == [0] * 4 + [4] * 3 + [7] * 6 + [13]
        assert nc == 4
    lab, nc = oracle.cda(off, adj, "components", 0)
    assert lab.tolist() == [0] * 4 + [4] * 3 + [7] * 6 + [13] and nc == 4


def _worked_example():
    """Three K12 (A = 0..11, B = 12..23, C = 24..35): A and B joined by three disjoint
    edges 9-21, 10-22, 11-23, and a bridge 23-24 from B to C."""
    e = complete(12) + complete(12, 12) + complete(12, 24) + [(9, 21), (10, 22), (11, 23), (23, 24)]
    return csr_from_edges(36, e)


def test_labelprop_worked_example():
    # Round 1 (labels are still the ids): 0 -> 1 and the rest of A -> 0; 12 -> 13, the
    # rest of B -> 12 except 21, 22, 23, whose smallest neighbour is 9, 10, 11 in A; 24
    # -> 23 (its neighbour in B) and the rest of C -> 24.  Round 2: every vertex sees its
    # own clique's label most often.
    off, adj = _worked_example()
    lab1, nc1 = oracle.cda(off, adj, "labelprop", 1)
    want1 = [1] + [0] * 11 + [13] + [12] * 8 + [9, 10, 11] + [23] + [24] * 11
    assert lab1.tolist() == want1 and nc1 == 9
    lab2, nc2 = oracle.cda(off, adj, "labelprop", 2)
    assert lab2.tolist() == [0] * 12 + [12] * 12 + [24] * 12 and nc2 == 3


def test_cm_worked_example():
    # The cluster (n = 36, k = 2) has minimum cut 1 (the bridge): S = A + B (the side of
    # vertex 0), the rest C.  WCC checks A + B as one set (n = 24, k = 2, cut 3) and saves
    # it; CM first runs the CDA on it: components give one community (saved whole, as
    # WCC), label propagation gives A and B, each saved (n = 12, k = 2, cut 11).
    off, adj = _worked_example()
    memb = np.zeros(36, np.int32)
    wcc, _ = oracle.wcc(off, adj, memb, mode="paper")
    comp, _ = oracle.cm(off, adj, memb, cda="components")
    lpa, rec = oracle.cm(off, adj, memb, cda="labelprop", cda_iters=3)
    assert wcc.tolist() == [0] * 24 + [1] * 12
    assert comp.tolist() == wcc.tolist()
    assert lpa.tolist() == [0] * 12 + [1] * 12 + [2] * 12
    assert sorted((int(r["n"]), int(r["lam"])) for r in rec) == [(12, 2), (12, 2), (12, 2), (36, 1)]
    golden = json.load(open(os.path.join(GOLDEN, "cm_worked_example.json")))
    assert lpa.tolist() == golden["membership_labelprop"]


# ------------------------------------------------------------------ CM = WCC with components
def _random_clustered(rng, n, nclust, p_in, p_out):
    memb = rng.integers(-1, nclust, n).astype(np.int32)
    edges = set()
    for a in range(n):
        for b in range(a + 1, n):
            same = memb[a] == memb[b] and memb[a] >= 0
            if rng.random() < (p_in if same else p_out):
                edges.add((a, b))
    off, adj = csr_from_edges(n, sorted(edges))
    return off, adj, memb


@pytest.mark.parametrize("s", [1, 5, 10])
def test_cm_components_equals_wcc_paper(s):
    rng = np.random.default_rng(100 + s)
    for trial in range(10):
        off, adj, memb = _random_clustered(rng, int(rng.integers(40, 300)), int(rng.integers(1, 6)),
                                           float(rng.choice([0.08, 0.2, 0.4])), 0.01)
        for crit in ("log10", "log2"):
            w, wr = oracle.wcc(off, adj, memb, s_pre=s, s_post=s, mode="paper", criterion=crit)
            c, cr = oracle.cm(off, adj, memb, s_pre=s, s_post=s, cda="components", criterion=crit)
            assert np.array_equal(w, c)
            assert _rec_key(wr) == _rec_key(cr)


def test_cm_components_equals_wcc_paper_chunglu():
    g = gen.chung_lu(20000, 24.0, 2.5, 11, 600, 2.0, 0.2, 0.15, 0.05, seed=91, intra_mult=1.8)
    w, wr = oracle.wcc(g, mode="paper")
    c, cr = oracle.cm(g, cda="components")
    assert np.array_equal(w, c)
    assert _rec_key(wr) == _rec_key(cr)


# ------------------------------------------------------------------ invariants with label propagation
def _check_invariants(off, adj, memb, out, s_post, crit="log10"):
    G = nx.Graph()
    n = len(memb)
    G.add_nodes_from(range(n))
    for u in range(n):
        for e in range(off[u], off[u + 1]):
            if u < adj[e]:
                G.add_edge(u, int(adj[e]))
    labels = np.unique(out[out >= 0])
    assert labels.tolist() == list(range(len(labels)))
    mins = []
    for L in labels:
        vs = np.nonzero(out == L)[0]
        mins.append(int(vs[0]))
        assert len(vs) > s_post
        assert len(np.unique(memb[vs])) == 1 and memb[vs[0]] >= 0   # one input cluster
        H = G.subgraph(vs.tolist())
        assert nx.is_connected(H)
        lam, _ = nx.stoer_wagner(H)
        assert lam >= oracle.threshold(len(vs), crit)                # well connected
    assert mins == sorted(mins)                                      # canonical labels


def test_cm_labelprop_invariants():
    rng = np.random.default_rng(7)
    for trial in range(6):
        off, adj, memb = _random_clustered(rng, int(rng.integers(80, 240)), int(rng.integers(1, 4)),
                                           float(rng.choice([0.15, 0.3])), 0.02)
        for it in (1, 3, 5):
            out, rec = oracle.cm(off, adj, memb, cda="labelprop", cda_iters=it, s_pre=5, s_post=5)
            _check_invariants(off, adj, memb, out, 5)
            assert np.all(rec["lam"][rec["lam"] >= rec["k"]] >= 1)
    g = gen.c0()
    out, rec = oracle.cm(g, cda="labelprop", cda_iters=5)
    _check_invariants(g.offsets, g.indices, g.membership, out, 10)
    assert out.max() >= 0
