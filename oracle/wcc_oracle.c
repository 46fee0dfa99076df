/*
 * wcc_oracle.c -- CPU ORACLE of the Well-Connected Clusters (WCC) hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg call it.  The GPU library never links, loads or calls it, and the two
 * share no code.
 *
 * It is a plain, slow, direct transcription of what the method computes, written from
 * the paper (Dindoost et al., "On the Optimization of Methods for Establishing
 * Well-Connected Communities", arXiv 2509.02590):
 *
 *   - CCR (Alg. 1): for every input cluster, its induced subgraph; if that has at least
 *     one edge, its connected components; components larger than s_pre are queued.
 *   - WCC (Alg. 2) / isWCC (Alg. 3): for each queued vertex set, the global minimum edge
 *     cut of its induced subgraph is compared with the criterion f(n) of its size n
 *     (Sec. 2: log10 n, log2 n, sqrt n or a linear k*n); "cut > f(n)" accepts the set,
 *     otherwise it is split along the cut and every part larger than s_post recurses.
 *   - CM (Alg. 4) / CMC (Alg. 5): the same check, but each side of a failing cut is first
 *     split into communities by a community detection algorithm (CDA); see orc_cm.
 *   - GetMinCut / MinCutPartition (Alg. 3, Sec. 2.1): an exact global minimum cut.  The
 *     paper runs a sequential VieCut variant and does not say which of several equal
 *     cuts it returns; the oracle fixes one canonical cut (see orc_mincut below).
 *
 * Readings taken where the paper is silent (each is also listed in the design notes):
 *   - the threshold "cut > f(n)" is evaluated in exact integers as cut >= k(n) with
 *     k(n) the least integer above f(n) (orc_threshold);
 *   - a saved set is every set accepted at any depth of the recursion (Alg. 3 saves
 *     inside the recursion);
 *   - output labels are canonical: accepted sets numbered by ascending smallest vertex
 *     id, every other vertex -1;
 *   - an optional pruning mode (KCORE) that the paper does not have: at entry a set of
 *     size n is replaced by the connected components of its k(n)-core whenever that
 *     core is not the whole set.  PAPER mode is Alg. 1-3 as printed.
 *
 * Everything is integer; there is no floating point anywhere in this file.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -3
#define ORC_ENOTCONN -5

enum { CRIT_LOG10 = 0, CRIT_LOG2 = 1, CRIT_SQRT = 2, CRIT_LINEAR = 3 };
enum { MODE_PAPER = 0, MODE_KCORE = 1 };

typedef struct {
  int32_t criterion; /* CRIT_* */
  int32_t lin_num;   /* LINEAR: f(n) = lin_num * n / lin_den */
  int32_t lin_den;
  int32_t s_pre;     /* CCR keeps components with size > s_pre */
  int32_t s_post;    /* recursion keeps parts with size > s_post */
  int32_t prune_mode;/* MODE_* */
} orc_params;

/* One record per minimum-cut evaluation. */
typedef struct {
  int32_t minv;   /* smallest global vertex id of the set */
  int32_t n;      /* set size */
  int32_t k;      /* threshold k(n) used as the cut cap */
  int32_t lambda; /* returned cut value (capped at k) */
  int32_t ssize;  /* |S| of the recorded side */
  int32_t pad;
  uint64_t shash; /* order-free hash of S's global ids */
} orc_record;

/* ------------------------------------------------------------------ criterion */
/* Least integer strictly greater than f(n), for n >= 1 (Sec. 2 names the criteria;
 * Alg. 3 accepts when the cut exceeds the criterion). */
int64_t orc_threshold(int32_t crit, int64_t n, int64_t num, int64_t den) {
  if (n < 1) return 0;
  switch (crit) {
    case CRIT_LOG10: { /* floor(log10 n) + 1 = number of decimal digits */
      int64_t d = 0;
      for (int64_t x = n; x > 0; x /= 10) d++;
      return d;
    }
    case CRIT_LOG2: { /* floor(log2 n) + 1 = bit length */
      int64_t b = 0;
      for (int64_t x = n; x > 0; x >>= 1) b++;
      return b;
    }
    case CRIT_SQRT: { /* floor(sqrt n) + 1 */
      int64_t r = 0;
      while ((r + 1) * (r + 1) <= n) r++;
      return r + 1;
    }
    case CRIT_LINEAR:
      if (den <= 0 || num < 0) return -1;
      return (num * n) / den + 1;
  }
  return -1;
}

/* ------------------------------------------------------------------ small helpers */
static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t vhash(int32_t v) { return mix64((uint64_t)(uint32_t)v + 0x9E3779B97F4A7C15ULL); }

typedef struct {
  int32_t *a;
  int64_t n, cap;
} ivec;
static int iv_push(ivec *v, int32_t x) {
  if (v->n == v->cap) {
    int64_t nc = v->cap ? 2 * v->cap : 16;
    int32_t *na = (int32_t *)realloc(v->a, (size_t)nc * sizeof(int32_t));
    if (!na) return -1;
    v->a = na;
    v->cap = nc;
  }
  v->a[v->n++] = x;
  return 0;
}
static void iv_free(ivec *v) {
  free(v->a);
  v->a = NULL;
  v->n = v->cap = 0;
}

/* ------------------------------------------------------------------ components */
/* Connected components of a CSR graph on 0..n-1 restricted to vertices with alive[v]
 * (alive may be NULL = all).  comp[v] = smallest vertex of v's component, -1 if dead.
 * Breadth-first search.  Returns the number of components or a negative error. */
int32_t orc_components(int32_t n, const int64_t *off, const int32_t *adj, const uint8_t *alive,
                       int32_t *comp) {
  int32_t *queue = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  if (!queue) return ORC_ENOMEM;
  for (int32_t v = 0; v < n; v++) comp[v] = -1;
  int32_t nc = 0;
  for (int32_t s = 0; s < n; s++) {
    if (comp[s] >= 0 || (alive && !alive[s])) continue;
    /* s is the smallest unvisited vertex, hence the smallest of its component */
    int32_t head = 0, tail = 0;
    queue[tail++] = s;
    comp[s] = s;
    while (head < tail) {
      int32_t x = queue[head++];
      for (int64_t e = off[x]; e < off[x + 1]; e++) {
        int32_t y = adj[e];
        if (comp[y] >= 0 || (alive && !alive[y])) continue;
        comp[y] = s;
        queue[tail++] = y;
      }
    }
    nc++;
  }
  free(queue);
  return nc;
}

/* ------------------------------------------------------------------ k-core */
/* alive[v] = 1 iff v is in the k-core (the maximal subgraph of minimum degree >= k),
 * found by repeatedly deleting vertices of degree < k.  Returns the core size. */
int32_t orc_kcore(int32_t n, const int64_t *off, const int32_t *adj, int32_t k, uint8_t *alive) {
  int32_t *deg = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  int32_t *stack = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  if (!deg || !stack) {
    free(deg);
    free(stack);
    return ORC_ENOMEM;
  }
  int32_t top = 0, left = n;
  for (int32_t v = 0; v < n; v++) {
    deg[v] = (int32_t)(off[v + 1] - off[v]);
    alive[v] = 1;
  }
  for (int32_t v = 0; v < n; v++)
    if (deg[v] < k) {
      alive[v] = 0;
      stack[top++] = v;
    }
  while (top > 0) {
    int32_t x = stack[--top];
    left--;
    for (int64_t e = off[x]; e < off[x + 1]; e++) {
      int32_t y = adj[e];
      if (!alive[y]) continue;
      if (--deg[y] < k) {
        alive[y] = 0;
        stack[top++] = y;
      }
    }
  }
  free(deg);
  free(stack);
  return left;
}

/* ------------------------------------------------------------------ minimum cut */
/*
 * Canonical exact global minimum cut of a connected simple graph H on 0..n-1 (n >= 2),
 * capped at cap >= 1.  This is one fully specified choice among the equal cuts the
 * paper's GetMinCut may return.  Algorithm: maximum-adjacency scans with contraction in
 * the style of Nagamochi, Ono and Ibaraki, with scan keys capped at the current bound
 * as in the CAPFOREST routine of VieCut (Henzinger, Noe, Schulz), the paper's min-cut
 * code (Sec. 2.1).
 *
 *   Super-vertices are sets of vertices; a super-vertex's id is its smallest member.
 *   Phase 0:  delta = minimum degree; bound = min(delta, cap); if delta <= cap then
 *             S = {smallest vertex of degree delta}.  Stop if bound <= 1.
 *   Round:    maximum-adjacency scan of the super-vertex graph starting at id 0; the
 *             next scanned super-vertex is the unscanned one with the largest key
 *             (keys capped at the bound), ties to the smallest id.  Scanning x adds
 *             w(x,y) to the key of every unscanned neighbour y; the edge (x,y) is
 *             contractible when key(y) + w(x,y) >= bound (key(y) before the update,
 *             itself capped).  All contractible edges are then contracted at once
 *             (new ids = smallest members), parallel edges summed, self-loops dropped.
 *             Degree check: in ascending id order, a super-vertex whose weighted degree
 *             is strictly below the bound becomes S and its degree the new bound; stop
 *             at bound 1.
 *   End:      when one super-vertex remains.
 *
 * If the true minimum cut lambda < cap, returns lambda and S is a minimum cut side;
 * otherwise returns cap (then S may be empty).  side[v] = 1 for v in S.
 */
typedef struct {
  int32_t y, w;
} wedge;
typedef struct {
  int32_t key, id;
} hnode;

/* max-heap on (key desc, id asc) */
static int hless(hnode a, hnode b) { return a.key < b.key || (a.key == b.key && a.id > b.id); }
static void hpush(hnode *h, int64_t *hn, hnode x) {
  int64_t i = (*hn)++;
  h[i] = x;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (!hless(h[p], h[i])) break;
    hnode t = h[p];
    h[p] = h[i];
    h[i] = t;
    i = p;
  }
}
static hnode hpop(hnode *h, int64_t *hn) {
  hnode top = h[0];
  h[0] = h[--(*hn)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, b = i;
    if (l < *hn && hless(h[b], h[l])) b = l;
    if (r < *hn && hless(h[b], h[r])) b = r;
    if (b == i) break;
    hnode t = h[b];
    h[b] = h[i];
    h[i] = t;
    i = b;
  }
  return top;
}

typedef struct {
  int32_t a, b, w;
} triple;
static int cmp_triple(const void *p, const void *q) {
  const triple *x = (const triple *)p, *y = (const triple *)q;
  if (x->a != y->a) return x->a < y->a ? -1 : 1;
  if (x->b != y->b) return x->b < y->b ? -1 : 1;
  return 0;
}
static int32_t uf_find(int32_t *par, int32_t x) {
  while (par[x] != x) {
    par[x] = par[par[x]]; /* path halving */
    x = par[x];
  }
  return x;
}

int32_t orc_mincut(int32_t n, const int64_t *off, const int32_t *adj, int32_t cap,
                   uint8_t *side) {
  if (n < 2 || cap < 1) return ORC_EINVAL;
  int32_t rc = ORC_ENOMEM;
  int64_t m2 = off[n];
  /* super-vertex graph: per id, a contiguous weighted adjacency list */
  int64_t *sofs = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
  wedge *sadj = (wedge *)malloc((size_t)(m2 ? m2 : 1) * sizeof(wedge));
  int32_t *svof = (int32_t *)malloc((size_t)n * sizeof(int32_t));  /* vertex -> super id */
  uint8_t *alive = (uint8_t *)malloc((size_t)n);                  /* id is a super-vertex */
  int32_t *key = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  uint8_t *scanned = (uint8_t *)malloc((size_t)n);
  int32_t *par = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  hnode *heap = (hnode *)malloc((size_t)(m2 + n + 1) * sizeof(hnode));
  triple *tr = (triple *)malloc((size_t)(m2 ? m2 : 1) * sizeof(triple));
  int32_t *pa = (int32_t *)malloc((size_t)(m2 ? m2 : 1) * sizeof(int32_t));
  int32_t *pb = (int32_t *)malloc((size_t)(m2 ? m2 : 1) * sizeof(int32_t));
  if (!sofs || !sadj || !svof || !alive || !key || !scanned || !par || !heap || !tr || !pa || !pb)
    goto done;

  /* Phase 0 */
  int32_t delta = INT32_MAX, dv = -1;
  for (int32_t v = 0; v < n; v++) {
    int32_t d = (int32_t)(off[v + 1] - off[v]);
    if (d < delta) {
      delta = d;
      dv = v;
    }
  }
  int32_t bound = delta < cap ? delta : cap;
  memset(side, 0, (size_t)n);
  if (delta <= cap) side[dv] = 1;
  if (bound <= 1) {
    rc = bound;
    goto done;
  }

  for (int32_t v = 0; v < n; v++) {
    svof[v] = v;
    alive[v] = 1;
    sofs[v] = off[v];
  }
  sofs[n] = m2;
  for (int64_t e = 0; e < m2; e++) {
    sadj[e].y = adj[e];
    sadj[e].w = 1;
  }
  int32_t nalive = n;

  while (nalive > 1) {
    /* maximum-adjacency scan with capped keys */
    int64_t hn = 0, np = 0;
    for (int32_t x = 0; x < n; x++) {
      key[x] = 0;
      scanned[x] = 0;
      if (alive[x]) hpush(heap, &hn, (hnode){0, x});
    }
    while (hn > 0) {
      hnode t = hpop(heap, &hn);
      int32_t x = t.id;
      if (scanned[x] || t.key != key[x]) continue;
      scanned[x] = 1;
      for (int64_t e = sofs[x]; e < sofs[x + 1]; e++) {
        int32_t y = sadj[e].y;
        if (scanned[y]) continue;
        int32_t r = key[y] + sadj[e].w;
        if (r >= bound) {
          pa[np] = x;
          pb[np] = y;
          np++;
        }
        key[y] = r < bound ? r : bound;
        hpush(heap, &hn, (hnode){key[y], y});
      }
    }
    /* contract all contractible edges; the root of each merged group is its min id */
    for (int32_t x = 0; x < n; x++) par[x] = x;
    for (int64_t i = 0; i < np; i++) {
      int32_t a = uf_find(par, pa[i]), b = uf_find(par, pb[i]);
      if (a == b) continue;
      if (a < b) par[b] = a;
      else par[a] = b;
    }
    int64_t nt = 0;
    for (int32_t x = 0; x < n; x++) {
      if (!alive[x]) continue;
      int32_t a = uf_find(par, x);
      for (int64_t e = sofs[x]; e < sofs[x + 1]; e++) {
        int32_t b = uf_find(par, sadj[e].y);
        if (a != b) tr[nt++] = (triple){a, b, sadj[e].w};
      }
    }
    qsort(tr, (size_t)nt, sizeof(triple), cmp_triple);
    /* rebuild the super-vertex graph, summing parallel edges */
    for (int32_t x = 0; x < n; x++) alive[x] = 0;
    for (int32_t v = 0; v < n; v++) {
      svof[v] = uf_find(par, svof[v]);
      alive[svof[v]] = 1;
    }
    nalive = 0;
    for (int32_t x = 0; x < n; x++) nalive += alive[x];
    int64_t w = 0, i = 0;
    for (int32_t x = 0; x < n; x++) {
      sofs[x] = w;
      while (i < nt && tr[i].a == x) {
        int32_t b = tr[i].b, s = 0;
        while (i < nt && tr[i].a == x && tr[i].b == b) s += tr[i++].w;
        sadj[w].y = b;
        sadj[w].w = s;
        w++;
      }
    }
    sofs[n] = w;
    /* degree check in ascending id */
    if (nalive > 1) {
      for (int32_t x = 0; x < n; x++) {
        if (!alive[x]) continue;
        int32_t d = 0;
        for (int64_t e = sofs[x]; e < sofs[x + 1]; e++) d += sadj[e].w;
        if (d < bound) {
          bound = d;
          for (int32_t v = 0; v < n; v++) side[v] = (uint8_t)(svof[v] == x);
          if (bound <= 1) break;
        }
      }
      if (bound <= 1) break;
    }
  }
  rc = bound;
done:
  free(sofs);
  free(sadj);
  free(svof);
  free(alive);
  free(key);
  free(scanned);
  free(par);
  free(heap);
  free(tr);
  free(pa);
  free(pb);
  return rc;
}

/* ------------------------------------------------------------------ induced subgraph */
/* Induced subgraph of the sorted vertex set U (global ids) in G, with local id = rank
 * in U (Alg. 1: E_c = edges with both endpoints in V_c).  lmap is a shared N-array of
 * hints: a hint is trusted only after checking U[hint] == w, so concurrent calls on
 * disjoint sets may share it.  Rows keep the order of G's rows. */
typedef struct {
  int64_t *off;
  int32_t *adj;
  int64_t cap_n, cap_e;
} lgraph;

static int induced(const int64_t *goff, const int32_t *gidx, int32_t *lmap, const int32_t *U,
                   int32_t n, lgraph *H) {
  if (H->cap_n < (int64_t)n + 1) {
    int64_t *no = (int64_t *)realloc(H->off, (size_t)(n + 1) * sizeof(int64_t));
    if (!no) return -1;
    H->off = no;
    H->cap_n = n + 1;
  }
  for (int32_t i = 0; i < n; i++) __atomic_store_n(&lmap[U[i]], i, __ATOMIC_RELAXED);
  int64_t cnt = 0;
  for (int32_t i = 0; i < n; i++) {
    int32_t u = U[i];
    for (int64_t e = goff[u]; e < goff[u + 1]; e++) {
      int32_t w = gidx[e];
      int32_t j = __atomic_load_n(&lmap[w], __ATOMIC_RELAXED);
      if (j >= 0 && j < n && U[j] == w) cnt++;
    }
  }
  if (H->cap_e < cnt + 1) {
    int32_t *na = (int32_t *)realloc(H->adj, (size_t)(cnt + 1) * sizeof(int32_t));
    if (!na) return -1;
    H->adj = na;
    H->cap_e = cnt + 1;
  }
  int64_t p = 0;
  for (int32_t i = 0; i < n; i++) {
    H->off[i] = p;
    int32_t u = U[i];
    for (int64_t e = goff[u]; e < goff[u + 1]; e++) {
      int32_t w = gidx[e];
      int32_t j = __atomic_load_n(&lmap[w], __ATOMIC_RELAXED);
      if (j >= 0 && j < n && U[j] == w) H->adj[p++] = j;
    }
  }
  H->off[n] = p;
  return 0;
}

/* ------------------------------------------------------------------ WCC driver */
typedef struct {
  int32_t *v; /* sorted global ids */
  int32_t n;
} item;

typedef struct {
  item *a;
  int64_t n, cap;
} ilist;
static int il_push(ilist *l, item it) {
  if (l->n == l->cap) {
    int64_t nc = l->cap ? 2 * l->cap : 64;
    item *na = (item *)realloc(l->a, (size_t)nc * sizeof(item));
    if (!na) return -1;
    l->a = na;
    l->cap = nc;
  }
  l->a[l->n++] = it;
  return 0;
}

typedef struct {
  /* input */
  int64_t N;
  const int64_t *off;
  const int32_t *idx;
  orc_params P;
  int32_t *lmap;
  /* current level */
  ilist *cur;
  int64_t next_item;
  /* outputs, under the lock */
  pthread_mutex_t lock;
  ilist next;
  ilist accepted;
  orc_record *log;
  int64_t log_cap, log_n;
  int32_t err;
  /* Connectivity Modifier (Alg. 4-5) instead of WCC: community detection after splits */
  int32_t cm, cda, cda_iters;
} wcc_ctx;

static int push_child(wcc_ctx *c, const int32_t *src, int32_t n) {
  int32_t *v = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  if (!v) return -1;
  memcpy(v, src, (size_t)n * sizeof(int32_t));
  pthread_mutex_lock(&c->lock);
  int r = il_push(&c->next, (item){v, n});
  pthread_mutex_unlock(&c->lock);
  if (r) free(v);
  return r;
}

/* Process one queued set (Alg. 3 step, with optional KCORE pruning at entry). */
static int process_item(wcc_ctx *c, item it, lgraph *H, ivec *tmp) {
  const orc_params *P = &c->P;
  int32_t n = it.n;
  if (induced(c->off, c->idx, c->lmap, it.v, n, H)) return ORC_ENOMEM;
  int64_t m2 = H->off[n];
  int32_t k = (int32_t)orc_threshold(P->criterion, n, P->lin_num, P->lin_den);
  int rc = ORC_OK;
  uint8_t *mark = (uint8_t *)malloc((size_t)(n ? n : 1));
  int32_t *comp = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  if (!mark || !comp) {
    rc = ORC_ENOMEM;
    goto out;
  }
  if (P->prune_mode == MODE_KCORE) {
    int32_t ksz = orc_kcore(n, H->off, H->adj, k, mark);
    if (ksz < 0) {
      rc = ksz;
      goto out;
    }
    if (ksz < n) {
      /* children: components of the core larger than s_post */
      orc_components(n, H->off, H->adj, mark, comp);
      for (int32_t r = 0; r < n; r++) {
        if (comp[r] != r) continue;
        tmp->n = 0;
        for (int32_t i = r; i < n; i++)
          if (comp[i] == r && iv_push(tmp, it.v[i])) {
            rc = ORC_ENOMEM;
            goto out;
          }
        if (tmp->n > P->s_post && push_child(c, tmp->a, (int32_t)tmp->n)) {
          rc = ORC_ENOMEM;
          goto out;
        }
      }
      goto out;
    }
  }
  /* Alg. 3: only sets with at least one edge are tested */
  if (m2 == 0) goto out;
  if (orc_components(n, H->off, H->adj, NULL, comp) != 1) {
    rc = ORC_ENOTCONN; /* cannot happen: every queued set is connected */
    goto out;
  }
  int32_t lam = orc_mincut(n, H->off, H->adj, k, mark);
  if (lam < 0) {
    rc = lam;
    goto out;
  }
  {
    orc_record rec = {it.v[0], n, k, lam, 0, 0, 0};
    for (int32_t i = 0; i < n; i++)
      if (mark[i]) {
        rec.ssize++;
        rec.shash += vhash(it.v[i]);
      }
    pthread_mutex_lock(&c->lock);
    if (c->log && c->log_n < c->log_cap) c->log[c->log_n] = rec;
    c->log_n++;
    pthread_mutex_unlock(&c->lock);
  }
  if (lam >= k) { /* cut > f(n): save the set */
    int32_t *v = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!v) {
      rc = ORC_ENOMEM;
      goto out;
    }
    memcpy(v, it.v, (size_t)n * sizeof(int32_t));
    pthread_mutex_lock(&c->lock);
    int r = il_push(&c->accepted, (item){v, n});
    pthread_mutex_unlock(&c->lock);
    if (r) {
      free(v);
      rc = ORC_ENOMEM;
    }
    goto out;
  }
  /* split along the cut; recurse on parts larger than s_post */
  for (int side = 1; side >= 0; side--) {
    tmp->n = 0;
    for (int32_t i = 0; i < n; i++)
      if (mark[i] == side && iv_push(tmp, it.v[i])) {
        rc = ORC_ENOMEM;
        goto out;
      }
    if (tmp->n > P->s_post && push_child(c, tmp->a, (int32_t)tmp->n)) {
      rc = ORC_ENOMEM;
      goto out;
    }
  }
out:
  free(mark);
  free(comp);
  return rc;
}

/* ------------------------------------------------------------------ Connectivity Modifier */
/* The community detection step of Alg. 5 (GetCommunities with a chosen CDA) on the
 * induced subgraph of one part, local ids 0..n-1.  comm[i] receives the community of i as
 * a local id; returns the number of communities.
 *   CDA_COMPONENTS: the connected components (labelled by their smallest vertex).
 *   CDA_LABELPROP: label propagation (Raghavan, Albert and Kumara 2007) made
 *     deterministic: every vertex starts with its own id; in each of `iters` synchronous
 *     rounds every vertex with a neighbour takes the label that occurs most often among
 *     its neighbours' labels of the previous round, the smallest such label on ties; the
 *     communities are the classes of equal final labels. */
enum { CDA_COMPONENTS = 0, CDA_LABELPROP = 1 };

static int cmp_i32(const void *p, const void *q) {
  int32_t a = *(const int32_t *)p, b = *(const int32_t *)q;
  return (a > b) - (a < b);
}

static int32_t cda_communities(int32_t cda, int32_t iters, int32_t n, const int64_t *off,
                               const int32_t *adj, int32_t *comm) {
  if (cda == CDA_COMPONENTS) return orc_components(n, off, adj, NULL, comm);
  int32_t *prev = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  int64_t maxdeg = 0;
  for (int32_t i = 0; i < n; i++)
    if (off[i + 1] - off[i] > maxdeg) maxdeg = off[i + 1] - off[i];
  int32_t *nb = (int32_t *)malloc((size_t)(maxdeg ? maxdeg : 1) * sizeof(int32_t));
  if (!prev || !nb) {
    free(prev);
    free(nb);
    return ORC_ENOMEM;
  }
  for (int32_t i = 0; i < n; i++) comm[i] = i;
  for (int32_t t = 0; t < iters; t++) {
    memcpy(prev, comm, (size_t)n * sizeof(int32_t));
    for (int32_t i = 0; i < n; i++) {
      int64_t d = off[i + 1] - off[i];
      if (d == 0) continue;
      for (int64_t e = 0; e < d; e++) nb[e] = prev[adj[off[i] + e]];
      qsort(nb, (size_t)d, sizeof(int32_t), cmp_i32);
      /* longest run of equal labels; the first (smallest) label wins a tie */
      int32_t best = nb[0];
      int64_t best_len = 0;
      for (int64_t a = 0; a < d;) {
        int64_t b = a;
        while (b < d && nb[b] == nb[a]) b++;
        if (b - a > best_len) {
          best_len = b - a;
          best = nb[a];
        }
        a = b;
      }
      comm[i] = best;
    }
  }
  /* number of distinct labels */
  memcpy(prev, comm, (size_t)n * sizeof(int32_t));
  qsort(prev, (size_t)n, sizeof(int32_t), cmp_i32);
  int32_t nc = 0;
  for (int32_t i = 0; i < n; i++) nc += (i == 0 || prev[i] != prev[i - 1]);
  free(prev);
  free(nb);
  return nc;
}

/* One queued set of CM (the CMC check of Alg. 5): a set with at least one edge is
 * saved when its canonical cut reaches k(n); otherwise each side of the cut larger than
 * s_post is handed to the CDA, and either each of its communities larger than s_post
 * (when there are several) or the whole part (when there is one, "processed as a single
 * unit") is checked again.  A disconnected set (only a CDA community can be one) has
 * cut 0 with S = the component of its smallest vertex.  No pruning: CM as printed. */
static int cm_item(wcc_ctx *c, item it, lgraph *H, ivec *tmp) {
  const orc_params *P = &c->P;
  int32_t n = it.n;
  if (induced(c->off, c->idx, c->lmap, it.v, n, H)) return ORC_ENOMEM;
  if (H->off[n] == 0) return ORC_OK; /* |E_c| = 0: nothing to test */
  int32_t k = (int32_t)orc_threshold(P->criterion, n, P->lin_num, P->lin_den);
  int rc = ORC_OK;
  uint8_t *side = (uint8_t *)malloc((size_t)n);
  int32_t *comp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  int32_t *part = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  lgraph Hp = {0};
  if (!side || !comp || !part) {
    rc = ORC_ENOMEM;
    goto out;
  }
  int32_t lam;
  if (orc_components(n, H->off, H->adj, NULL, comp) > 1) {
    lam = 0;
    for (int32_t i = 0; i < n; i++) side[i] = comp[i] == 0;
  } else {
    lam = orc_mincut(n, H->off, H->adj, k, side);
    if (lam < 0) {
      rc = lam;
      goto out;
    }
  }
  {
    orc_record rec = {it.v[0], n, k, lam, 0, 0, 0};
    for (int32_t i = 0; i < n; i++)
      if (side[i]) {
        rec.ssize++;
        rec.shash += vhash(it.v[i]);
      }
    pthread_mutex_lock(&c->lock);
    if (c->log && c->log_n < c->log_cap) c->log[c->log_n] = rec;
    c->log_n++;
    pthread_mutex_unlock(&c->lock);
  }
  if (lam >= k) { /* cut > criterion: save the set */
    int32_t *v = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    if (!v) {
      rc = ORC_ENOMEM;
      goto out;
    }
    memcpy(v, it.v, (size_t)n * sizeof(int32_t));
    pthread_mutex_lock(&c->lock);
    int r = il_push(&c->accepted, (item){v, n});
    pthread_mutex_unlock(&c->lock);
    if (r) {
      free(v);
      rc = ORC_ENOMEM;
    }
    goto out;
  }
  for (int sd = 1; sd >= 0; sd--) {
    int32_t np = 0;
    for (int32_t i = 0; i < n; i++)
      if (side[i] == sd) part[np++] = it.v[i];
    if (np <= P->s_post) continue;
    if (induced(c->off, c->idx, c->lmap, part, np, &Hp)) {
      rc = ORC_ENOMEM;
      goto out;
    }
    int32_t nc = cda_communities(c->cda, c->cda_iters, np, Hp.off, Hp.adj, comp);
    if (nc < 0) {
      rc = nc;
      goto out;
    }
    if (nc <= 1) {
      if (push_child(c, part, np)) {
        rc = ORC_ENOMEM;
        goto out;
      }
      continue;
    }
    /* each community V_i (ascending ids) larger than s_post */
    for (int32_t r = 0; r < np; r++) {
      int32_t lab = comp[r];
      int first = 1;
      for (int32_t i = 0; i < r; i++)
        if (comp[i] == lab) {
          first = 0;
          break;
        }
      if (!first) continue;
      tmp->n = 0;
      for (int32_t i = r; i < np; i++)
        if (comp[i] == lab && iv_push(tmp, part[i])) {
          rc = ORC_ENOMEM;
          goto out;
        }
      if (tmp->n > P->s_post && push_child(c, tmp->a, (int32_t)tmp->n)) {
        rc = ORC_ENOMEM;
        goto out;
      }
    }
  }
out:
  free(side);
  free(comp);
  free(part);
  free(Hp.off);
  free(Hp.adj);
  return rc;
}

static void *worker(void *arg) {
  wcc_ctx *c = (wcc_ctx *)arg;
  lgraph H = {0};
  ivec tmp = {0};
  for (;;) {
    int64_t i = __atomic_fetch_add(&c->next_item, 1, __ATOMIC_RELAXED);
    if (i >= c->cur->n) break;
    int rc = c->cm ? cm_item(c, c->cur->a[i], &H, &tmp) : process_item(c, c->cur->a[i], &H, &tmp);
    if (rc) {
      pthread_mutex_lock(&c->lock);
      if (!c->err) c->err = rc;
      pthread_mutex_unlock(&c->lock);
    }
  }
  free(H.off);
  free(H.adj);
  iv_free(&tmp);
  return NULL;
}

static void run_level(wcc_ctx *c, int nthreads) {
  c->next_item = 0;
  if (nthreads <= 1) {
    worker(c);
    return;
  }
  if (nthreads > 512) nthreads = 512;
  pthread_t th[512];
  int started = 0;
  for (int t = 0; t < nthreads - 1; t++)
    if (pthread_create(&th[started], NULL, worker, c) == 0) started++;
  worker(c);
  for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
}

typedef struct {
  int32_t key, v;
} kv;
static int cmp_kv(const void *p, const void *q) {
  const kv *a = (const kv *)p, *b = (const kv *)q;
  if (a->key != b->key) return a->key < b->key ? -1 : 1;
  return (a->v > b->v) - (a->v < b->v);
}
static int cmp_item_min(const void *p, const void *q) {
  const item *a = (const item *)p, *b = (const item *)q;
  return (a->v[0] > b->v[0]) - (a->v[0] < b->v[0]);
}

static void free_list(ilist *l) {
  for (int64_t i = 0; i < l->n; i++) free(l->a[i].v);
  free(l->a);
  l->a = NULL;
  l->n = l->cap = 0;
}

static int check_params(const orc_params *P) {
  if (P->s_pre < 0 || P->s_post < 0) return ORC_EINVAL;
  if (P->criterion < CRIT_LOG10 || P->criterion > CRIT_LINEAR) return ORC_EINVAL;
  if (P->criterion == CRIT_LINEAR && (P->lin_den <= 0 || P->lin_num < 0)) return ORC_EINVAL;
  if (P->prune_mode != MODE_PAPER && P->prune_mode != MODE_KCORE) return ORC_EINVAL;
  return ORC_OK;
}

/*
 * Full WCC (Alg. 2 with CCR, Alg. 1, and isWCC, Alg. 3).
 *   off/idx: symmetric simple CSR of G (N vertices); membership[v] >= 0 is v's input
 *   cluster, < 0 unassigned.  out[v] = canonical label of v's accepted set or -1.
 *   log (nullable): one record per minimum-cut evaluation, up to log_cap of them;
 *   *log_n receives the total count.  Items are processed level by level with
 *   nthreads threads; the result does not depend on the order.
 */
static int32_t orc_drive(int64_t N, const int64_t *off, const int32_t *idx, const int32_t *membership,
                         const orc_params *P, int32_t *out, orc_record *log, int64_t log_cap,
                         int64_t *log_n, int32_t nthreads, int32_t cm, int32_t cda, int32_t cda_iters) {
  int32_t rc = check_params(P);
  if (rc) return rc;
  wcc_ctx c;
  memset(&c, 0, sizeof(c));
  c.cm = cm;
  c.cda = cda;
  c.cda_iters = cda_iters;
  c.N = N;
  c.off = off;
  c.idx = idx;
  c.P = *P;
  c.log = log;
  c.log_cap = log_cap;
  pthread_mutex_init(&c.lock, NULL);
  ilist level = {0};
  lgraph H = {0};
  int32_t *comp = NULL;
  kv *pairs = NULL;
  c.lmap = (int32_t *)malloc((size_t)(N ? N : 1) * sizeof(int32_t));
  if (!c.lmap) {
    rc = ORC_ENOMEM;
    goto done;
  }
  for (int64_t v = 0; v < N; v++) c.lmap[v] = -1;

  /* CCR (Alg. 1): group vertices by cluster id, ascending ids inside each cluster */
  int64_t na = 0;
  for (int64_t v = 0; v < N; v++) na += membership[v] >= 0;
  pairs = (kv *)malloc((size_t)(na ? na : 1) * sizeof(kv));
  if (!pairs) {
    rc = ORC_ENOMEM;
    goto done;
  }
  na = 0;
  for (int64_t v = 0; v < N; v++)
    if (membership[v] >= 0) pairs[na++] = (kv){membership[v], (int32_t)v};
  qsort(pairs, (size_t)na, sizeof(kv), cmp_kv);
  int32_t *U = (int32_t *)malloc((size_t)(na ? na : 1) * sizeof(int32_t));
  if (!U) {
    rc = ORC_ENOMEM;
    goto done;
  }
  for (int64_t i = 0; i < na; i++) U[i] = pairs[i].v;
  comp = (int32_t *)malloc((size_t)(na ? na : 1) * sizeof(int32_t));
  if (!comp) {
    free(U);
    rc = ORC_ENOMEM;
    goto done;
  }
  for (int64_t s = 0; s < na;) {
    int64_t e = s;
    while (e < na && pairs[e].key == pairs[s].key) e++;
    int32_t n = (int32_t)(e - s);
    if (induced(off, idx, c.lmap, U + s, n, &H)) {
      rc = ORC_ENOMEM;
      break;
    }
    if (H.off[n] > 0) { /* |E_c| > 0 */
      orc_components(n, H.off, H.adj, NULL, comp);
      for (int32_t r = 0; r < n; r++) {
        if (comp[r] != r) continue;
        int32_t sz = 0;
        for (int32_t i = r; i < n; i++) sz += comp[i] == r;
        if (sz <= P->s_pre) continue;
        int32_t *v = (int32_t *)malloc((size_t)sz * sizeof(int32_t));
        if (!v) {
          rc = ORC_ENOMEM;
          break;
        }
        int32_t q = 0;
        for (int32_t i = r; i < n; i++)
          if (comp[i] == r) v[q++] = U[s + i];
        if (il_push(&level, (item){v, sz})) {
          free(v);
          rc = ORC_ENOMEM;
          break;
        }
      }
    }
    s = e;
  }
  free(U);
  if (rc) goto done;

  /* recursion, processed one level at a time */
  while (level.n > 0) {
    c.cur = &level;
    c.next.n = 0;
    run_level(&c, nthreads);
    free_list(&level);
    level = c.next;
    memset(&c.next, 0, sizeof(c.next));
    if (c.err) {
      rc = c.err;
      goto done;
    }
  }

  /* canonical labels: accepted sets by ascending smallest vertex */
  for (int64_t v = 0; v < N; v++) out[v] = -1;
  qsort(c.accepted.a, (size_t)c.accepted.n, sizeof(item), cmp_item_min);
  for (int64_t i = 0; i < c.accepted.n; i++)
    for (int32_t j = 0; j < c.accepted.a[i].n; j++) out[c.accepted.a[i].v[j]] = (int32_t)i;
  if (log_n) *log_n = c.log_n;
done:
  free_list(&level);
  free_list(&c.next);
  free_list(&c.accepted);
  free(c.lmap);
  free(H.off);
  free(H.adj);
  free(comp);
  free(pairs);
  pthread_mutex_destroy(&c.lock);
  return rc;
}

int32_t orc_wcc(int64_t N, const int64_t *off, const int32_t *idx, const int32_t *membership,
                const orc_params *P, int32_t *out, orc_record *log, int64_t log_cap,
                int64_t *log_n, int32_t nthreads) {
  return orc_drive(N, off, idx, membership, P, out, log, log_cap, log_n, nthreads, 0, 0, 0);
}

/*
 * Full CM (Alg. 4 with CCR, Alg. 1, and the check CMC, Alg. 5) with a built-in CDA
 * (CDA_COMPONENTS, or CDA_LABELPROP with cda_iters rounds).  P->prune_mode is ignored
 * (CM as printed prunes nothing).  Outputs as orc_wcc: canonical labels of the saved
 * sets and one record per minimum-cut evaluation.
 */
int32_t orc_cm(int64_t N, const int64_t *off, const int32_t *idx, const int32_t *membership,
               const orc_params *P, int32_t cda, int32_t cda_iters, int32_t *out, orc_record *log,
               int64_t log_cap, int64_t *log_n, int32_t nthreads) {
  if ((cda != CDA_COMPONENTS && cda != CDA_LABELPROP) || cda_iters < 0) return ORC_EINVAL;
  return orc_drive(N, off, idx, membership, P, out, log, log_cap, log_n, nthreads, 1, cda, cda_iters);
}

/* The CDA alone on a graph (local ids): comm[i] = community label; returns their count. */
int32_t orc_cda(int32_t cda, int32_t iters, int32_t n, const int64_t *off, const int32_t *adj, int32_t *comm) {
  if ((cda != CDA_COMPONENTS && cda != CDA_LABELPROP) || iters < 0) return ORC_EINVAL;
  return cda_communities(cda, iters, n, off, adj, comm);
}

/*
 * mincut_split: the minimum-cut-and-split step of Alg. 3 / Alg. 5 on one vertex set.
 * verts: sorted, unique global ids (nv of them).  If the induced subgraph is
 * disconnected, returns 0 with S = the component of verts[0]; otherwise the canonical
 * cut with the given cap (cap >= 1).  side[i] = 1 iff verts[i] is in S.  nv < 2 returns
 * 0 with an empty S.
 */
int32_t orc_mincut_split(int64_t N, const int64_t *off, const int32_t *idx, const int32_t *verts,
                         int32_t nv, int32_t cap, uint8_t *side) {
  if (nv < 0 || cap < 1) return ORC_EINVAL;
  memset(side, 0, (size_t)(nv ? nv : 1));
  if (nv < 2) return 0;
  for (int32_t i = 0; i < nv; i++)
    if (verts[i] < 0 || verts[i] >= N || (i && verts[i] <= verts[i - 1])) return ORC_EINVAL;
  int32_t *lmap = (int32_t *)malloc((size_t)N * sizeof(int32_t));
  int32_t *comp = (int32_t *)malloc((size_t)nv * sizeof(int32_t));
  lgraph H = {0};
  int32_t rc = ORC_ENOMEM;
  if (!lmap || !comp) goto out;
  for (int64_t v = 0; v < N; v++) lmap[v] = -1;
  if (induced(off, idx, lmap, verts, nv, &H)) goto out;
  if (orc_components(nv, H.off, H.adj, NULL, comp) > 1) {
    for (int32_t i = 0; i < nv; i++) side[i] = comp[i] == 0;
    rc = 0;
    goto out;
  }
  rc = orc_mincut(nv, H.off, H.adj, cap, side);
out:
  free(lmap);
  free(comp);
  free(H.off);
  free(H.adj);
  return rc;
}

/*
 * Cluster-major induced subgraphs (the compaction the GPU path performs first):
 * clusters in ascending cluster id, vertices ascending inside each, rows holding local
 * ids (rank inside the cluster) in ascending order.  With NULL outputs only the sizes
 * are returned (*nclusters, *nassigned, *nentries).
 */
int32_t orc_cluster_csr(int64_t N, const int64_t *off, const int32_t *idx, const int32_t *membership,
                        int64_t *nclusters, int64_t *nassigned, int64_t *nentries,
                        int32_t *cl_ids, int64_t *cl_start, int32_t *vert, int64_t *row_off,
                        int32_t *adj) {
  int64_t na = 0;
  for (int64_t v = 0; v < N; v++) na += membership[v] >= 0;
  kv *pairs = (kv *)malloc((size_t)(na ? na : 1) * sizeof(kv));
  int32_t *lmap = (int32_t *)malloc((size_t)(N ? N : 1) * sizeof(int32_t));
  int32_t *U = (int32_t *)malloc((size_t)(na ? na : 1) * sizeof(int32_t));
  lgraph H = {0};
  int32_t rc = ORC_ENOMEM;
  if (!pairs || !lmap || !U) goto out;
  for (int64_t v = 0; v < N; v++) lmap[v] = -1;
  na = 0;
  for (int64_t v = 0; v < N; v++)
    if (membership[v] >= 0) pairs[na++] = (kv){membership[v], (int32_t)v};
  qsort(pairs, (size_t)na, sizeof(kv), cmp_kv);
  for (int64_t i = 0; i < na; i++) U[i] = pairs[i].v;
  int64_t K = 0, E = 0;
  for (int64_t s = 0; s < na;) {
    int64_t e = s;
    while (e < na && pairs[e].key == pairs[s].key) e++;
    int32_t n = (int32_t)(e - s);
    if (induced(off, idx, lmap, U + s, n, &H)) goto out;
    if (vert) {
      cl_ids[K] = pairs[s].key;
      cl_start[K] = s;
      for (int32_t i = 0; i < n; i++) {
        vert[s + i] = U[s + i];
        row_off[s + i] = E + H.off[i];
        int64_t a = H.off[i], b = H.off[i + 1];
        for (int64_t q = a; q < b; q++) adj[E + q] = H.adj[q];
        /* ascending row order */
        for (int64_t q = a + 1; q < b; q++) {
          int32_t x = adj[E + q];
          int64_t r = q - 1;
          while (r >= a && adj[E + r] > x) {
            adj[E + r + 1] = adj[E + r];
            r--;
          }
          adj[E + r + 1] = x;
        }
      }
    }
    E += H.off[n];
    K++;
    s = e;
  }
  if (vert) {
    cl_start[K] = na;
    row_off[na] = E;
  }
  *nclusters = K;
  *nassigned = na;
  *nentries = E;
  rc = 0;
out:
  free(pairs);
  free(lmap);
  free(U);
  free(H.off);
  free(H.adj);
  return rc;
}

/* order-free hash of a vertex set, as recorded in orc_record.shash */
uint64_t orc_set_hash(const int32_t *v, int64_t n) {
  uint64_t h = 0;
  for (int64_t i = 0; i < n; i++) h += vhash(v[i]);
  return h;
}
