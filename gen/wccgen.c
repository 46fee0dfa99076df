/*
 * wccgen.c -- seeded synthetic inputs for WCC workloads: an undirected simple graph in
 * CSR form plus a planted (disjoint) clustering.
 *
 * This module only manufactures inputs.  It contains none of the WCC method's
 * arithmetic (no induced subgraphs, components, pruning, cuts or thresholds); both the
 * CPU oracle and the GPU path consume what it writes.
 *
 * Randomness is counter based: every draw is SplitMix64's output function applied to a
 * (seed, stream, index) triple, so the result does not depend on thread count or
 * scheduling.  SplitMix64: Steele, Lea & Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014.
 *
 * Workload shapes (they stand in for the paper's real networks, Table 1, and its
 * Leiden-CPM input clusterings, which are not available):
 *   - tiny planted graph: equal clusters of Erdos-Renyi blocks, some built from two
 *     halves joined by one bridge, some with a pendant path, plus uniform noise edges;
 *   - Chung-Lu graph with Pareto (power-law) expected degrees and a planted clustering
 *     with power-law cluster sizes, a mixing fraction of inter-cluster edges, clusters
 *     built as halves joined by 1..3 bridges (optionally nested), and clusters built as
 *     disconnected unions of two blocks.
 */
#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* One 64-bit draw keyed by (seed, stream, index). */
static inline uint64_t rng64(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t k = mix64(seed + GOLDEN * (stream + 1));
  return mix64(k + GOLDEN * (idx + 1));
}
static inline double rngu(uint64_t seed, uint64_t stream, uint64_t idx) {
  return (double)(rng64(seed, stream, idx) >> 11) * 0x1.0p-53;
}
/* uniform integer in [0, n) */
static inline int64_t rngi(uint64_t seed, uint64_t stream, uint64_t idx, int64_t n) {
  return (int64_t)(rngu(seed, stream, idx) * (double)n);
}

/* stream tags */
enum {
  ST_PERM = 1, ST_WEIGHT = 2, ST_SIZE = 3, ST_KIND = 4, ST_INTRA = 5, ST_BRIDGE = 6,
  ST_INTER = 7, ST_DEPTH = 8, ST_TINY_ER = 9, ST_TINY_NOISE = 10
};
static inline uint64_t stream_of(uint64_t tag, uint64_t sub) { return (tag << 48) ^ sub; }

/* ------------------------------------------------------------------ edge buffers */
typedef struct {
  int32_t *u, *v;
  int64_t n, cap;
} ebuf;

static int eb_push(ebuf *b, int32_t u, int32_t v) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? b->cap * 2 : 1024;
    int32_t *nu = (int32_t *)realloc(b->u, (size_t)nc * sizeof(int32_t));
    if (!nu) return -1;
    b->u = nu;
    int32_t *nv = (int32_t *)realloc(b->v, (size_t)nc * sizeof(int32_t));
    if (!nv) return -1;
    b->v = nv;
    b->cap = nc;
  }
  b->u[b->n] = u;
  b->v[b->n] = v;
  b->n++;
  return 0;
}
static void eb_free(ebuf *b) {
  free(b->u);
  free(b->v);
  memset(b, 0, sizeof(*b));
}

/* ------------------------------------------------------------------ output graph */
typedef struct {
  int64_t n;          /* vertices */
  int64_t nnz;        /* directed CSR entries (2m) */
  int64_t *offsets;   /* n+1 */
  int32_t *indices;   /* nnz */
  int32_t *membership;/* n, -1 = unassigned */
  int64_t nclusters;
  int64_t inter_edges;/* undirected edges whose endpoints lie in different clusters */
} gen_graph;

void gen_free(gen_graph *g) {
  if (!g) return;
  free(g->offsets);
  free(g->indices);
  free(g->membership);
  free(g);
}
int64_t gen_n(const gen_graph *g) { return g->n; }
int64_t gen_nnz(const gen_graph *g) { return g->nnz; }
int64_t gen_nclusters(const gen_graph *g) { return g->nclusters; }
int64_t gen_inter_edges(const gen_graph *g) { return g->inter_edges; }
void gen_export(const gen_graph *g, int64_t *offsets, int32_t *indices, int32_t *membership) {
  memcpy(offsets, g->offsets, (size_t)(g->n + 1) * sizeof(int64_t));
  memcpy(indices, g->indices, (size_t)g->nnz * sizeof(int32_t));
  memcpy(membership, g->membership, (size_t)g->n * sizeof(int32_t));
}

/* ------------------------------------------------------------------ threading */
typedef void (*task_fn)(void *ctx, int64_t task);
typedef struct {
  task_fn fn;
  void *ctx;
  int64_t ntasks;
  int64_t next;
  int64_t done;
  const char *name;
} pool_job;

/* With WCCGEN_VERBOSE set (or gen_set_verbose(1)), every phase reports each eighth of its
 * tasks on stderr (long generations otherwise print nothing for minutes). */
static int g_verbose = -1;
static int gen_verbose(void) {
  if (g_verbose < 0) {
    const char *e = getenv("WCCGEN_VERBOSE");
    g_verbose = e && *e && *e != '0';
  }
  return g_verbose;
}
void gen_set_verbose(int v) { g_verbose = v ? 1 : 0; }

static void *pool_worker(void *arg) {
  pool_job *j = (pool_job *)arg;
  int64_t step = (j->ntasks + 7) / 8;
  for (;;) {
    int64_t t = __atomic_fetch_add(&j->next, 1, __ATOMIC_RELAXED);
    if (t >= j->ntasks) break;
    j->fn(j->ctx, t);
    int64_t d = __atomic_add_fetch(&j->done, 1, __ATOMIC_RELAXED);
    if (gen_verbose() && step > 0 && (d % step == 0 || d == j->ntasks)) {
      fprintf(stderr, "[gen] %s %lld/%lld tasks\n", j->name, (long long)d, (long long)j->ntasks);
      fflush(stderr);
    }
  }
  return NULL;
}
static void parallel_for_named(const char *name, int nthreads, int64_t ntasks, task_fn fn, void *ctx) {
  pool_job j = {fn, ctx, ntasks, 0, 0, name};
  if (nthreads <= 1 || ntasks <= 1) {
    pool_worker(&j);
    return;
  }
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  int started = 0;
  for (int i = 0; i < nthreads - 1; i++)
    if (pthread_create(&th[started], NULL, pool_worker, &j) == 0) started++;
  pool_worker(&j);
  for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
}

#define parallel_for(nt, n, fn, ctx) parallel_for_named(#fn, nt, n, fn, ctx)

/* ------------------------------------------------------------------ CSR builder */
static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}
static void sort_row(int32_t *r, int64_t len) {
  if (len <= 24) {
    for (int64_t i = 1; i < len; i++) {
      int32_t x = r[i];
      int64_t j = i - 1;
      while (j >= 0 && r[j] > x) {
        r[j + 1] = r[j];
        j--;
      }
      r[j + 1] = x;
    }
  } else {
    qsort(r, (size_t)len, sizeof(int32_t), cmp_i32);
  }
}

typedef struct {
  const int32_t *u, *v;
  int64_t m, chunk;
  int64_t n;
  int32_t *deg;     /* n */
  int64_t *off;     /* n+1 */
  int64_t *cur;     /* n */
  int32_t *tmp;     /* 2m */
  int32_t *ndeg;    /* n */
  int64_t *noff;
  int32_t *out;
} csr_ctx;

static void t_count(void *c_, int64_t t) {
  csr_ctx *c = (csr_ctx *)c_;
  int64_t a = t * c->chunk, b = a + c->chunk < c->m ? a + c->chunk : c->m;
  for (int64_t i = a; i < b; i++) {
    if (c->u[i] == c->v[i]) continue;
    __atomic_fetch_add(&c->deg[c->u[i]], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&c->deg[c->v[i]], 1, __ATOMIC_RELAXED);
  }
}
static void t_fill(void *c_, int64_t t) {
  csr_ctx *c = (csr_ctx *)c_;
  int64_t a = t * c->chunk, b = a + c->chunk < c->m ? a + c->chunk : c->m;
  for (int64_t i = a; i < b; i++) {
    int32_t x = c->u[i], y = c->v[i];
    if (x == y) continue;
    int64_t p = __atomic_fetch_add(&c->cur[x], 1, __ATOMIC_RELAXED);
    c->tmp[p] = y;
    p = __atomic_fetch_add(&c->cur[y], 1, __ATOMIC_RELAXED);
    c->tmp[p] = x;
  }
}
#define ROWCHUNK 4096
static void t_sortdedup(void *c_, int64_t t) {
  csr_ctx *c = (csr_ctx *)c_;
  int64_t a = t * ROWCHUNK, b = a + ROWCHUNK < c->n ? a + ROWCHUNK : c->n;
  for (int64_t r = a; r < b; r++) {
    int32_t *row = c->tmp + c->off[r];
    int64_t len = c->off[r + 1] - c->off[r];
    sort_row(row, len);
    int64_t k = 0;
    for (int64_t i = 0; i < len; i++)
      if (k == 0 || row[i] != row[k - 1]) row[k++] = row[i];
    c->ndeg[r] = (int32_t)k;
  }
}
static void t_copy(void *c_, int64_t t) {
  csr_ctx *c = (csr_ctx *)c_;
  int64_t a = t * ROWCHUNK, b = a + ROWCHUNK < c->n ? a + ROWCHUNK : c->n;
  for (int64_t r = a; r < b; r++)
    memcpy(c->out + c->noff[r], c->tmp + c->off[r], (size_t)c->ndeg[r] * sizeof(int32_t));
}

/* Symmetric simple CSR from an undirected pair list: both directions, self-loops and
 * duplicates removed, rows sorted ascending. */
static int build_csr(int64_t n, const ebuf *e, int nthreads, gen_graph *g) {
  csr_ctx c;
  memset(&c, 0, sizeof(c));
  c.u = e->u;
  c.v = e->v;
  c.m = e->n;
  c.n = n;
  c.chunk = 1 << 20;
  c.deg = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  c.off = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  c.cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  c.ndeg = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  c.noff = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  if (!c.deg || !c.off || !c.cur || !c.ndeg || !c.noff) goto fail;
  int64_t nch = (c.m + c.chunk - 1) / c.chunk;
  parallel_for(nthreads, nch, t_count, &c);
  c.off[0] = 0;
  for (int64_t i = 0; i < n; i++) c.off[i + 1] = c.off[i] + c.deg[i];
  memcpy(c.cur, c.off, (size_t)n * sizeof(int64_t));
  c.tmp = (int32_t *)malloc((size_t)(c.off[n] ? c.off[n] : 1) * sizeof(int32_t));
  if (!c.tmp) goto fail;
  parallel_for(nthreads, nch, t_fill, &c);
  int64_t nrch = (n + ROWCHUNK - 1) / ROWCHUNK;
  parallel_for(nthreads, nrch, t_sortdedup, &c);
  c.noff[0] = 0;
  for (int64_t i = 0; i < n; i++) c.noff[i + 1] = c.noff[i] + c.ndeg[i];
  c.out = (int32_t *)malloc((size_t)(c.noff[n] ? c.noff[n] : 1) * sizeof(int32_t));
  if (!c.out) goto fail;
  parallel_for(nthreads, nrch, t_copy, &c);
  free(c.deg);
  free(c.off);
  free(c.cur);
  free(c.tmp);
  free(c.ndeg);
  g->offsets = c.noff;
  g->indices = c.out;
  g->nnz = c.noff[n];
  return 0;
fail:
  free(c.deg);
  free(c.off);
  free(c.cur);
  free(c.tmp);
  free(c.ndeg);
  free(c.noff);
  free(c.out);
  return -1;
}

static void count_inter(gen_graph *g) {
  int64_t x = 0;
  for (int64_t v = 0; v < g->n; v++)
    for (int64_t e = g->offsets[v]; e < g->offsets[v + 1]; e++) {
      int32_t u = g->indices[e];
      if (u > v && g->membership[u] != g->membership[v]) x++;
    }
  g->inter_edges = x;
}

/* random permutation of 0..n-1 (Fisher-Yates driven by the counter generator) */
static int32_t *random_perm(int64_t n, uint64_t seed, uint64_t stream) {
  int32_t *p = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  if (!p) return NULL;
  for (int64_t i = 0; i < n; i++) p[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; i--) {
    int64_t j = rngi(seed, stream, (uint64_t)i, i + 1);
    int32_t t = p[i];
    p[i] = p[j];
    p[j] = t;
  }
  return p;
}

/* ================================================================== tiny planted graph
 * n_clusters clusters of csize vertices (all vertices assigned, ids permuted):
 *   - n_bridged clusters: two halves, each ER(p_half), joined by one bridge edge;
 *   - n_pendant clusters: (csize - path_len) ER(p) vertices plus a path of path_len
 *     vertices hanging from one ER vertex;
 *   - the rest: ER(p) on the whole cluster;
 * plus n_noise distinct uniform inter-cluster edges. */
gen_graph *gen_tiny(uint64_t seed, int64_t n_clusters, int64_t csize, double p,
                    int64_t n_bridged, double p_half, int64_t n_pendant, int64_t path_len,
                    int64_t n_noise) {
  int64_t n = n_clusters * csize;
  gen_graph *g = (gen_graph *)calloc(1, sizeof(gen_graph));
  if (!g) return NULL;
  g->n = n;
  g->nclusters = n_clusters;
  g->membership = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  int32_t *perm = random_perm(n, seed, stream_of(ST_PERM, 0));
  ebuf e = {0};
  if (!g->membership || !perm) goto fail;
  for (int64_t c = 0; c < n_clusters; c++) {
    const int32_t *V = perm + c * csize;
    for (int64_t i = 0; i < csize; i++) g->membership[V[i]] = (int32_t)c;
    uint64_t st = stream_of(ST_TINY_ER, (uint64_t)c);
    if (c < n_bridged) {
      int64_t h = csize / 2;
      for (int64_t i = 0; i < csize; i++)
        for (int64_t j = i + 1; j < csize; j++) {
          if ((i < h) != (j < h)) continue;
          if (rngu(seed, st, (uint64_t)(i * csize + j)) < p_half)
            if (eb_push(&e, V[i], V[j])) goto fail;
        }
      int64_t a = rngi(seed, stream_of(ST_BRIDGE, (uint64_t)c), 0, h);
      int64_t b = h + rngi(seed, stream_of(ST_BRIDGE, (uint64_t)c), 1, csize - h);
      if (eb_push(&e, V[a], V[b])) goto fail;
    } else if (c < n_bridged + n_pendant) {
      int64_t core = csize - path_len;
      for (int64_t i = 0; i < core; i++)
        for (int64_t j = i + 1; j < core; j++)
          if (rngu(seed, st, (uint64_t)(i * csize + j)) < p)
            if (eb_push(&e, V[i], V[j])) goto fail;
      int64_t anchor = rngi(seed, stream_of(ST_BRIDGE, (uint64_t)c), 0, core);
      int32_t prev = V[anchor];
      for (int64_t i = core; i < csize; i++) {
        if (eb_push(&e, prev, V[i])) goto fail;
        prev = V[i];
      }
    } else {
      for (int64_t i = 0; i < csize; i++)
        for (int64_t j = i + 1; j < csize; j++)
          if (rngu(seed, st, (uint64_t)(i * csize + j)) < p)
            if (eb_push(&e, V[i], V[j])) goto fail;
    }
  }
  /* distinct uniform inter-cluster noise edges (open-addressing set on the pair key) */
  if (n_noise > 0 && n_clusters > 1) {
    int64_t hcap = 1;
    while (hcap < 4 * n_noise) hcap <<= 1;
    uint64_t *hs = (uint64_t *)calloc((size_t)hcap, sizeof(uint64_t));
    if (!hs) goto fail;
    int64_t got = 0;
    for (uint64_t t = 0; got < n_noise; t++) {
      int64_t a = rngi(seed, stream_of(ST_TINY_NOISE, 0), 2 * t, n);
      int64_t b = rngi(seed, stream_of(ST_TINY_NOISE, 0), 2 * t + 1, n);
      if (g->membership[a] == g->membership[b]) continue;
      int64_t lo = a < b ? a : b, hi = a < b ? b : a;
      uint64_t key = ((uint64_t)lo << 32 | (uint64_t)hi) + 1;
      uint64_t h = mix64(key) & (uint64_t)(hcap - 1);
      int dup = 0;
      while (hs[h]) {
        if (hs[h] == key) {
          dup = 1;
          break;
        }
        h = (h + 1) & (uint64_t)(hcap - 1);
      }
      if (dup) continue;
      hs[h] = key;
      if (eb_push(&e, (int32_t)lo, (int32_t)hi)) {
        free(hs);
        goto fail;
      }
      got++;
    }
    free(hs);
  }
  if (build_csr(n, &e, 1, g)) goto fail;
  eb_free(&e);
  free(perm);
  count_inter(g);
  return g;
fail:
  eb_free(&e);
  free(perm);
  gen_free(g);
  return NULL;
}

/* ================================================================== Chung-Lu planted */
typedef struct {
  int64_t n;          /* vertices */
  double mean_deg;    /* target 2m/n */
  double alpha;       /* Pareto exponent of expected degrees */
  double wmax;        /* truncation of expected degree; <= 0 means sqrt(2m) */
  int64_t smin, smax; /* cluster size range */
  double beta;        /* cluster size power-law exponent */
  double mu;          /* mixing: expected share of a vertex's edges leaving its cluster */
  double f_bridged;   /* share of clusters built as halves joined by bridges */
  double f_disc;      /* share of clusters built as two disconnected blocks */
  int32_t depth_max;  /* bridged clusters nest halving to depth U{1..depth_max} */
  int32_t nthreads;
  double intra_mult;  /* sample-count multipliers that offset duplicate-pair losses */
  double inter_mult;
} gen_cl_params;

typedef struct {
  const gen_cl_params *P;
  uint64_t seed;
  const int32_t *perm;   /* vertex order; clusters are consecutive chunks */
  const int64_t *cstart; /* nclusters+1 */
  const double *w;       /* expected degrees */
  const int32_t *memb;
  const double *cw_all;  /* global cumulative weights (n+1) */
  int64_t inter_samples, inter_chunk;
  int64_t nclusters;
  ebuf *bufs;            /* one per task */
} cl_ctx;

/* draw an index in [0,len) proportionally to the weights behind the cumulative array */
static int64_t draw_cum(const double *cum, int64_t len, double x) {
  double t = x * cum[len];
  int64_t lo = 0, hi = len - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (cum[mid + 1] > t) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

/* Chung-Lu edges inside one block of vertices: round(sum((1-mu) w)/2) samples. */
static int cl_block(cl_ctx *c, ebuf *out, const int32_t *V, int64_t len, uint64_t stream) {
  if (len < 2) return 0;
  double *cum = (double *)malloc((size_t)(len + 1) * sizeof(double));
  if (!cum) return -1;
  cum[0] = 0;
  for (int64_t i = 0; i < len; i++) cum[i + 1] = cum[i] + c->w[V[i]];
  int64_t samples = llround(cum[len] * (1.0 - c->P->mu) * 0.5 * c->P->intra_mult);
  for (int64_t s = 0; s < samples; s++) {
    int64_t a = draw_cum(cum, len, rngu(c->seed, stream, 2 * (uint64_t)s));
    int64_t b = draw_cum(cum, len, rngu(c->seed, stream, 2 * (uint64_t)s + 1));
    if (a == b) continue;
    if (eb_push(out, V[a], V[b])) {
      free(cum);
      return -1;
    }
  }
  free(cum);
  return 0;
}

/* recursive halving with bridges at every level (depth 0 = plain block) */
static int cl_nested(cl_ctx *c, ebuf *out, const int32_t *V, int64_t len, int depth,
                     uint64_t cid, uint64_t path) {
  uint64_t st = stream_of(ST_INTRA, (cid << 8) ^ path);
  if (depth == 0 || len < 2) return cl_block(c, out, V, len, st);
  int64_t h = len / 2;
  if (cl_nested(c, out, V, h, depth - 1, cid, path * 2 + 1)) return -1;
  if (cl_nested(c, out, V + h, len - h, depth - 1, cid, path * 2 + 2)) return -1;
  uint64_t bs = stream_of(ST_BRIDGE, (cid << 8) ^ path);
  int64_t nb = 1 + rngi(c->seed, bs, 0, 3);
  for (int64_t i = 0; i < nb; i++) {
    int64_t a = rngi(c->seed, bs, 1 + 2 * (uint64_t)i, h);
    int64_t b = h + rngi(c->seed, bs, 2 + 2 * (uint64_t)i, len - h);
    if (eb_push(out, V[a], V[b])) return -1;
  }
  return 0;
}

static void t_cluster(void *c_, int64_t t) {
  cl_ctx *c = (cl_ctx *)c_;
  ebuf *out = &c->bufs[t];
  const int32_t *V = c->perm + c->cstart[t];
  int64_t len = c->cstart[t + 1] - c->cstart[t];
  double k = rngu(c->seed, stream_of(ST_KIND, (uint64_t)t), 0);
  if (k < c->P->f_bridged) {
    int depth = 1;
    if (c->P->depth_max > 1)
      depth = 1 + (int)rngi(c->seed, stream_of(ST_DEPTH, (uint64_t)t), 0, c->P->depth_max);
    cl_nested(c, out, V, len, depth, (uint64_t)t, 0);
  } else if (k < c->P->f_bridged + c->P->f_disc) {
    int64_t h = len / 2;
    cl_block(c, out, V, h, stream_of(ST_INTRA, ((uint64_t)t << 8) ^ 1));
    cl_block(c, out, V + h, len - h, stream_of(ST_INTRA, ((uint64_t)t << 8) ^ 2));
  } else {
    cl_block(c, out, V, len, stream_of(ST_INTRA, (uint64_t)t << 8));
  }
}

static void t_inter(void *c_, int64_t t) {
  cl_ctx *c = (cl_ctx *)c_;
  ebuf *out = &c->bufs[c->nclusters + t];
  int64_t a0 = t * c->inter_chunk;
  int64_t a1 = a0 + c->inter_chunk < c->inter_samples ? a0 + c->inter_chunk : c->inter_samples;
  uint64_t st = stream_of(ST_INTER, 0);
  for (int64_t s = a0; s < a1; s++) {
    int64_t a = draw_cum(c->cw_all, c->P->n, rngu(c->seed, st, 2 * (uint64_t)s));
    int64_t b = draw_cum(c->cw_all, c->P->n, rngu(c->seed, st, 2 * (uint64_t)s + 1));
    if (a == b || c->memb[a] == c->memb[b]) continue;
    if (eb_push(out, (int32_t)a, (int32_t)b)) return;
  }
}

gen_graph *gen_chung_lu(const gen_cl_params *P, uint64_t seed) {
  int64_t n = P->n;
  gen_graph *g = (gen_graph *)calloc(1, sizeof(gen_graph));
  if (!g) return NULL;
  g->n = n;
  double *w = (double *)malloc((size_t)(n ? n : 1) * sizeof(double));
  double *cw = (double *)malloc((size_t)(n + 1) * sizeof(double));
  int32_t *perm = random_perm(n, seed, stream_of(ST_PERM, 0));
  int64_t *cstart = NULL;
  ebuf *bufs = NULL;
  int64_t nbufs = 0;
  ebuf all = {0};
  g->membership = (int32_t *)malloc((size_t)(n ? n : 1) * sizeof(int32_t));
  if (!w || !cw || !perm || !g->membership) goto fail;

  /* expected degrees: Pareto(alpha) with mean mean_deg, truncated, rescaled to 2m */
  double two_m = P->mean_deg * (double)n;
  double wmin = P->mean_deg * (P->alpha - 2.0) / (P->alpha - 1.0);
  double wmax = P->wmax > 0 ? P->wmax : sqrt(two_m);
  double tot = 0;
  for (int64_t i = 0; i < n; i++) {
    double u = rngu(seed, stream_of(ST_WEIGHT, 0), (uint64_t)i);
    double x = wmin * pow(1.0 - u, -1.0 / (P->alpha - 1.0));
    if (x > wmax) x = wmax;
    w[i] = x;
    tot += x;
  }
  for (int64_t i = 0; i < n && tot > 0; i++) w[i] *= two_m / tot;

  /* cluster sizes: discrete power law s^-beta on [smin, smax] until the vertices run out */
  int64_t ns = P->smax - P->smin + 1;
  double *scum = (double *)malloc((size_t)(ns + 1) * sizeof(double));
  if (!scum) goto fail;
  scum[0] = 0;
  for (int64_t s = 0; s < ns; s++) scum[s + 1] = scum[s] + pow((double)(P->smin + s), -P->beta);
  int64_t ccap = 1024, nc = 0, used = 0;
  cstart = (int64_t *)malloc((size_t)(ccap + 1) * sizeof(int64_t));
  if (!cstart) {
    free(scum);
    goto fail;
  }
  cstart[0] = 0;
  while (used < n) {
    int64_t s = P->smin + draw_cum(scum, ns, rngu(seed, stream_of(ST_SIZE, 0), (uint64_t)nc));
    if (used + s > n) s = n - used;
    if (s < P->smin && nc > 0) { /* fold a short remainder into the previous cluster */
      cstart[nc] = n;
      used = n;
      break;
    }
    if (nc + 1 >= ccap) {
      ccap *= 2;
      int64_t *ncs = (int64_t *)realloc(cstart, (size_t)(ccap + 1) * sizeof(int64_t));
      if (!ncs) {
        free(scum);
        goto fail;
      }
      cstart = ncs;
    }
    used += s;
    nc++;
    cstart[nc] = used;
  }
  free(scum);
  g->nclusters = nc;
  for (int64_t c = 0; c < nc; c++)
    for (int64_t i = cstart[c]; i < cstart[c + 1]; i++) g->membership[perm[i]] = (int32_t)c;

  /* global cumulative weights for inter-cluster sampling on mu*w */
  cw[0] = 0;
  for (int64_t i = 0; i < n; i++) cw[i + 1] = cw[i] + w[i];

  cl_ctx c;
  memset(&c, 0, sizeof(c));
  c.P = P;
  c.seed = seed;
  c.perm = perm;
  c.cstart = cstart;
  c.w = w;
  c.memb = g->membership;
  c.cw_all = cw;
  c.nclusters = nc;
  c.inter_samples = llround(cw[n] * P->mu * 0.5 * P->inter_mult);
  c.inter_chunk = 1 << 20;
  int64_t ninter = (c.inter_samples + c.inter_chunk - 1) / c.inter_chunk;
  bufs = (ebuf *)calloc((size_t)(nc + ninter + 1), sizeof(ebuf));
  if (!bufs) goto fail;
  nbufs = nc + ninter;
  c.bufs = bufs;
  parallel_for(P->nthreads, nc, t_cluster, &c);
  parallel_for(P->nthreads, ninter, t_inter, &c);

  int64_t total = 0;
  for (int64_t t = 0; t < nc + ninter; t++) total += bufs[t].n;
  all.u = (int32_t *)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
  all.v = (int32_t *)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
  if (!all.u || !all.v) goto fail;
  for (int64_t t = 0; t < nc + ninter; t++) {
    memcpy(all.u + all.n, bufs[t].u, (size_t)bufs[t].n * sizeof(int32_t));
    memcpy(all.v + all.n, bufs[t].v, (size_t)bufs[t].n * sizeof(int32_t));
    all.n += bufs[t].n;
    eb_free(&bufs[t]);
  }
  free(bufs);
  bufs = NULL;
  free(w);
  w = NULL;
  free(cw);
  cw = NULL;
  if (build_csr(n, &all, P->nthreads, g)) goto fail;
  eb_free(&all);
  free(perm);
  free(cstart);
  count_inter(g);
  return g;
fail:
  if (bufs) {
    for (int64_t t = 0; t < nbufs; t++) eb_free(&bufs[t]);
    free(bufs);
  }
  eb_free(&all);
  free(w);
  free(cw);
  free(perm);
  free(cstart);
  gen_free(g);
  return NULL;
}
