"""The order fact behind the GPU's batched PAPER-mode peel, checked by brute force (no
oracle, no GPU).

In PAPER mode (Alg. 1-3 as printed) a connected set with a vertex of degree 1 has cut 1
with S = {its smallest vertex of degree 1}; when the criterion rejects it, that vertex is
split off and the rest is checked again.  The sequence of removed vertices is the greedy
"remove the smallest leaf" order.  The GPU computes it without replaying it: a synchronous
peel of the vertices of degree <= 1 gives every removed vertex u its round r(u) and M(u),
the largest id in u's hanging subtree (u and what hangs below it); a tree is rooted at its
largest id, which stays.  The greedy order is the sort by (M(u), r(u)).

Why: a vertex becomes a leaf once its subtree is gone; two subtrees that do not contain
each other are consumed independently, and the greedy merge of two such sequences takes,
between their heads, the smaller -- which orders every element by the largest id that
precedes it in its own sequence (for u: M(u)); equal M only happens along one root path,
where a descendant (smaller round) goes first."""
import heapq
import random


def greedy(n, adj, stop_at):
    deg = [len(adj[v]) for v in range(n)]
    alive = [True] * n
    size = n
    h = [v for v in range(n) if deg[v] == 1]
    heapq.heapify(h)
    seq = []
    while h and size > stop_at:
        v = heapq.heappop(h)
        if not alive[v] or deg[v] != 1:
            continue
        alive[v] = False
        size -= 1
        seq.append(v)
        for u in adj[v]:
            if alive[u]:
                deg[u] -= 1
                if deg[u] == 1:
                    heapq.heappush(h, u)
    return seq


def by_subtree_max(n, adj, stop_at):
    edges = sum(len(a) for a in adj) // 2
    pin = n - 1 if edges == n - 1 else -1          # a tree keeps its largest vertex
    deg = [len(adj[v]) for v in range(n)]
    rnd = [-1] * n
    front = [v for v in range(n) if deg[v] <= 1 and v != pin]
    for v in front:
        rnd[v] = 0
    r = 0
    while front:
        nxt = []
        for v in front:
            for u in adj[v]:
                if rnd[u] < 0 or rnd[u] > r:
                    deg[u] -= 1
                    if deg[u] == 1 and u != pin and rnd[u] < 0:
                        rnd[u] = r + 1
                        nxt.append(u)
        front = nxt
        r += 1
    removed = sorted((v for v in range(n) if rnd[v] >= 0), key=lambda v: rnd[v])
    M = {}
    for v in removed:
        M[v] = max([v] + [M[u] for u in adj[v] if 0 <= rnd[u] < rnd[v]])
    seq = sorted(removed, key=lambda v: (M[v], rnd[v]))
    return seq[:max(0, n - stop_at)]


def _random_connected(rng, n, extra):
    perm = list(range(n))
    rng.shuffle(perm)
    edges = set()
    for i in range(1, n):
        a, b = perm[i], perm[rng.randrange(i)]
        edges.add((min(a, b), max(a, b)))
    for _ in range(extra):
        a, b = rng.sample(range(n), 2)
        edges.add((min(a, b), max(a, b)))
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    return adj


def test_greedy_leaf_order_is_sort_by_subtree_max():
    rng = random.Random(11)
    for _ in range(6000):
        n = rng.randint(2, 16)
        adj = _random_connected(rng, n, rng.choice([0, 0, 1, 2, 4]))
        stop = rng.choice([0, 1, 2, n // 2])
        assert greedy(n, adj, stop) == by_subtree_max(n, adj, stop), (n, adj, stop)


def test_long_paths_and_stars():
    # a cycle with a long pendant path and a star hanging from it
    n = 40
    adj = [[] for _ in range(n)]
    def e(a, b):
        adj[a].append(b)
        adj[b].append(a)
    for i in range(5):
        e(i, (i + 1) % 5)
    for i in range(5, 25):
        e(i - 1 if i > 5 else 2, i)
    for i in range(25, 40):
        e(30 if i != 30 else 0, i)
    assert greedy(n, adj, 0) == by_subtree_max(n, adj, 0)
