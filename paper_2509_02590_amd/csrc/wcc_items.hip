// wcc_items.hip -- one workgroup per queued vertex set ("item"):
//   * CCR for top-level clusters: connected components of the induced subgraph, parts
//     larger than s_pre are queued (Alg. 1);
//   * KCORE mode: peel to the k(n)-core; if vertices were removed, the core's components
//     larger than s_post are queued instead of cutting;
//   * the canonical exact minimum cut capped at k(n) (GetMinCut / MinCutPartition of
//     Alg. 3): degree pre-pass, then rounds of maximum-adjacency scans with capped keys,
//     bulk contraction of every edge whose key reaches the bound, degree check;
//   * acceptance (cut > f(n), i.e. cut >= k(n)) or a split into the cut's two sides,
//     each rebuilt as a compacted induced subgraph in the other arena (Alg. 3).
//
// Per-item state lives in LDS when it fits the launch's dynamic LDS, else in the global
// per-position scratch slices [b, b+n) (items of one launch are disjoint) plus a
// per-workgroup bitmap region; the code reaches both through generic pointers.
//
// The maximum-adjacency scan keeps, for every key level j in 0..bound, a 3-level bitmap
// of the unscanned super-vertices whose key is >= j (level 0 = all unscanned).  The next
// vertex is the smallest id in the highest non-empty level, found in four dependent
// reads; a key increment only ever sets one bit, so concurrent updates commute.
#include "wcc_internal.h"

namespace {

constexpr int IB = 256;  // threads per item workgroup
constexpr int NW = IB / 64;
constexpr int MAX_LEVEL = 62;

struct Sh {
  int red[NW + 1];
  long long red64[NW + 1];
  unsigned long long redu[NW + 1];
  unsigned long long levelmask;
  unsigned long long hsum;
  int vi[8];
};

struct St {
  int32_t *A, *B, *C, *D, *E, *F;  // n each
  uint64_t *bits;              // bitmap area
  int n;
  int nw0, nw1, nw2, ls;       // bitmap geometry per level
};

DEV int uf_find(int32_t *P, int x) {
  for (;;) {
    int p = ld(&P[x]);
    if (p == x) return x;
    int g = ld(&P[p]);
    if (g == p) return p;
    st(&P[x], g);  // path halving: g is an ancestor of x
    x = g;
  }
}

// Hook the larger root under the smaller one; roots end as component minima.
DEV void uf_unite(int32_t *P, int a, int b) {
  for (;;) {
    a = uf_find(P, a);
    b = uf_find(P, b);
    if (a == b) return;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(&P[a], a, b) == a) return;
  }
}

// ---------------------------------------------------------------- bitmap levels
DEV uint64_t *lvl0(const St &s, int j) { return s.bits + (size_t)j * s.ls; }
DEV uint64_t *lvl1(const St &s, int j) { return s.bits + (size_t)j * s.ls + s.nw0; }
DEV uint64_t *lvl2(const St &s, int j) { return s.bits + (size_t)j * s.ls + s.nw0 + s.nw1; }

DEV void bit_set(const St &s, int j, int y, unsigned long long *levelmask) {
  unsigned long long old = atomicOr((unsigned long long *)&lvl0(s, j)[y >> 6], 1ull << (y & 63));
  if (old) return;
  old = atomicOr((unsigned long long *)&lvl1(s, j)[y >> 12], 1ull << ((y >> 6) & 63));
  if (old) return;
  old = atomicOr((unsigned long long *)&lvl2(s, j)[y >> 18], 1ull << ((y >> 12) & 63));
  if (old) return;
  atomicOr(levelmask, 1ull << j);
}

DEV void bit_clear(const St &s, int j, int x, unsigned long long *levelmask) {
  unsigned long long b = 1ull << (x & 63);
  unsigned long long old = atomicAnd((unsigned long long *)&lvl0(s, j)[x >> 6], ~b);
  if (old != b) return;
  b = 1ull << ((x >> 6) & 63);
  old = atomicAnd((unsigned long long *)&lvl1(s, j)[x >> 12], ~b);
  if (old != b) return;
  b = 1ull << ((x >> 12) & 63);
  old = atomicAnd((unsigned long long *)&lvl2(s, j)[x >> 18], ~b);
  if (old != b) return;
  for (int t = 0; t < s.nw2; t++)
    if (ld(&lvl2(s, j)[t])) return;
  atomicAnd(levelmask, ~(1ull << j));
}

DEV bool bit_test(const St &s, int j, int y) { return (ld(&lvl0(s, j)[y >> 6]) >> (y & 63)) & 1ull; }

// smallest id in the highest non-empty level, or -1
DEV int bit_pick(const St &s, unsigned long long lm) {
  if (!lm) return -1;
  int j = 63 - __clzll(lm);
  const uint64_t *L2 = lvl2(s, j);
  uint64_t w = 0;
  int t = 0;
  for (; t < s.nw2; t++) {
    w = ld(&L2[t]);
    if (w) break;
  }
  if (!w) return -1;
  int i1 = t * 64 + __ffsll((long long)w) - 1;
  uint64_t w1 = ld(&lvl1(s, j)[i1]);
  if (!w1) return -2;  // inconsistent summary (never expected)
  int i0 = i1 * 64 + __ffsll((long long)w1) - 1;
  uint64_t w0 = ld(&lvl0(s, j)[i0]);
  if (!w0) return -2;
  int x = i0 * 64 + __ffsll((long long)w0) - 1;
  return x < s.n ? x : -2;
}

// ---------------------------------------------------------------- helpers
DEV void err(const ItemArgs &A, int code) {
  atomicMin((long long *)&A.cnt[CNT_ERR], (long long)code);
}

// Connected components of the item restricted to alive vertices (alive = A[i] >= kmin
// when use_deg, else all).  B[i] = smallest vertex of i's component, -1 if dead.
// Returns the number of components.
DEV int item_cc(const St &s, const Arena &ar, const ItemDesc &d, bool use_deg, int kmin, Sh &sh) {
  int n = s.n;
  for (int i = threadIdx.x; i < n; i += IB) {
    bool al = !use_deg || ld(&s.A[i]) >= kmin;
    st(&s.B[i], al ? i : -1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += IB) {
    if (ld(&s.B[i]) < 0) continue;
    int64_t r0 = ar.rs[d.b + i];
    int rdeg = ar.rd[d.b + i];
    for (int e = 0; e < rdeg; e++) {
      int j = ar.adj[r0 + e];
      if (j < i && ld(&s.B[j]) >= 0) uf_unite(s.B, i, j);
    }
  }
  __syncthreads();
  int roots = 0;
  for (int i = threadIdx.x; i < n; i += IB) {
    if (ld(&s.B[i]) < 0) continue;
    int r = uf_find(s.B, i);
    roots += (r == i);
    st(&s.B[i], r);
  }
  return block_sum<IB>(roots, sh.red);  // includes barriers
}

// ---------------------------------------------------------------- rebuild children
// B[i]: child label (the child's smallest local id) or -1.  Children larger than gate
// are compacted into the other arena inside [b, b+n) / [eb, eb+m) and pushed.
DEV void item_rebuild(const ItemArgs &A, const St &s, const ItemDesc &d, int gate, Sh &sh) {
  const Arena &ar = A.ar[d.depth & 1];
  const Arena &nx = A.ar[(d.depth + 1) & 1];
  int n = s.n;
  for (int i = threadIdx.x; i < n; i += IB) st(&s.A[i], 0);
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += IB) {
    int L = ld(&s.B[i]);
    if (L >= 0) atomicAdd(&s.A[L], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += IB) {
    int L = ld(&s.B[i]);
    if (L >= 0 && ld(&s.A[L]) <= gate) st(&s.B[i], -1);
  }
  __syncthreads();
  // child starts: exclusive scan over representatives
  int carry = 0;
  for (int base = 0; base < n; base += IB) {
    int i = base + threadIdx.x;
    int v = 0;
    if (i < n && ld(&s.B[i]) == i) v = ld(&s.A[i]);
    int tot;
    int pre = block_excl_scan<IB>(v, sh.red, &tot);
    if (i < n) st(&s.D[i], carry + pre);
    carry += tot;
  }
  int K = carry;
  __syncthreads();
  if (K == 0) return;
  // stable new positions: wave 0 walks the item in order (E[i] = new position)
  if (threadIdx.x < 64) {
    for (int base = 0; base < n; base += 64) {
      int i = base + threadIdx.x;
      int L = i < n ? ld(&s.B[i]) : -1;
      uint64_t act = __ballot(L >= 0);
      while (act) {
        int leader = __ffsll((long long)act) - 1;
        int LL = __shfl(L, leader, 64);
        uint64_t peers = __ballot(L == LL) & act;
        int pos0 = 0;
        if ((int)threadIdx.x == leader) pos0 = atomicAdd(&s.D[LL], __popcll(peers));
        pos0 = __shfl(pos0, leader, 64);
        if (L == LL) st(&s.E[i], pos0 + __popcll(peers & lanemask_lt()));
        act &= ~peers;
      }
    }
  }
  __syncthreads();
  // D[L] now holds start + size; restore starts
  for (int i = threadIdx.x; i < n; i += IB)
    if (ld(&s.B[i]) == i) st(&s.D[i], ld(&s.D[i]) - ld(&s.A[i]));
  __syncthreads();
  // new degrees by new position (C)
  for (int i = threadIdx.x; i < n; i += IB) {
    int L = ld(&s.B[i]);
    if (L < 0) continue;
    int64_t r0 = ar.rs[d.b + i];
    int rdeg = ar.rd[d.b + i];
    int c = 0;
    for (int e = 0; e < rdeg; e++) c += ld(&s.B[ar.adj[r0 + e]]) == L;
    st(&s.C[ld(&s.E[i])], c);
  }
  __syncthreads();
  // row offsets by new position (exclusive scan of C, in place)
  long long ecarry = 0;
  for (int base = 0; base < K; base += IB) {
    int p = base + threadIdx.x;
    long long v = p < K ? (long long)ld(&s.C[p]) : 0;
    long long tot;
    long long pre = block_excl_scan64<IB>(v, sh.red64, &tot);
    if (p < K) st(&s.C[p], (int)(ecarry + pre));
    ecarry += tot;
  }
  int M = (int)ecarry;
  __syncthreads();
  // write the children's rows into the other arena
  for (int i = threadIdx.x; i < n; i += IB) {
    int L = ld(&s.B[i]);
    if (L < 0) continue;
    int np = ld(&s.E[i]);
    int o = ld(&s.C[np]);
    int o1 = np + 1 < K ? ld(&s.C[np + 1]) : M;
    int cstart = ld(&s.D[L]);
    nx.vtx[d.b + np] = ar.vtx[d.b + i];
    nx.rs[d.b + np] = d.eb + o;
    nx.rd[d.b + np] = o1 - o;
    int64_t r0 = ar.rs[d.b + i];
    int rdeg = ar.rd[d.b + i];
    int64_t w = d.eb + o;
    for (int e = 0; e < rdeg; e++) {
      int j = ar.adj[r0 + e];
      if (ld(&s.B[j]) == L) nx.adj[w++] = ld(&s.E[j]) - cstart;
    }
  }
  // descriptors of the children
  for (int i = threadIdx.x; i < n; i += IB) {
    if (ld(&s.B[i]) != i) continue;
    int cs = ld(&s.D[i]);
    int sz = ld(&s.A[i]);
    int o = ld(&s.C[cs]);
    int o1 = cs + sz < K ? ld(&s.C[cs + sz]) : M;
    ItemDesc c;
    c.b = d.b + cs;
    c.n = sz;
    c.eb = d.eb + o;
    c.m = o1 - o;
    c.depth = d.depth + 1;
    c.flags = 0;
    int slot = atomicAdd(A.out_count, 1);
    if (slot < A.out_cap) A.out[slot] = c;
    else err(A, WCC_ENOMEM);
  }
  __syncthreads();
}

// ---------------------------------------------------------------- k-core peel
// A[i] ends as i's degree inside the surviving core (alive iff A[i] >= k).
// Returns the number of removed vertices.
DEV int item_peel(const St &s, const Arena &ar, const ItemDesc &d, int k, Sh &sh) {
  int n = s.n;
  if (threadIdx.x == 0) sh.vi[0] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += IB) {
    int dg = ar.rd[d.b + i];
    st(&s.A[i], dg);
    if (dg < k) st(&s.D[atomicAdd(&sh.vi[0], 1)], i);
  }
  __syncthreads();
  int cnt = sh.vi[0];
  int removed = cnt;
  int32_t *cur = s.D, *nxt = s.E;
  while (cnt > 0) {
    __syncthreads();
    if (threadIdx.x == 0) sh.vi[1] = 0;
    __syncthreads();
    for (int f = threadIdx.x; f < cnt; f += IB) {
      int u = ld(&cur[f]);
      int64_t r0 = ar.rs[d.b + u];
      int rdeg = ar.rd[d.b + u];
      for (int e = 0; e < rdeg; e++) {
        int j = ar.adj[r0 + e];
        int old = atomicSub(&s.A[j], 1);
        if (old == k) st(&nxt[atomicAdd(&sh.vi[1], 1)], j);
      }
    }
    __syncthreads();
    cnt = sh.vi[1];
    removed += cnt;
    int32_t *t = cur;
    cur = nxt;
    nxt = t;
  }
  __syncthreads();
  return removed;
}

// ---------------------------------------------------------------- canonical min cut
// Returns the capped cut value; F[i] = 1 for i in S.  steps/rounds are accumulated.
DEV int item_mincut(const ItemArgs &A, const St &s, const Arena &ar, const ItemDesc &d, int cap,
                    Sh &sh, long long *steps_out, long long *rounds_out) {
  int n = s.n;
  // Phase 0: minimum degree and its smallest vertex
  unsigned long long mv = ~0ull;
  for (int i = threadIdx.x; i < n; i += IB) {
    unsigned long long v = ((unsigned long long)(uint32_t)ar.rd[d.b + i] << 32) | (uint32_t)i;
    mv = v < mv ? v : mv;
  }
  mv = block_min_u64<IB>(mv, sh.redu);
  int delta = (int)(mv >> 32), dv = (int)(mv & 0xffffffffu);
  int bound = delta < cap ? delta : cap;
  int s_kind = delta <= cap ? 1 : 0;  // 0 empty, 1 singleton dv, 2 set in F
  long long steps = 0, rounds = 0;
  if (bound > 1 && bound > MAX_LEVEL) {
    err(A, WCC_EUNSUPPORTED);
    bound = 1;  // give up on this item; the error is reported
  }
  if (bound > 1) {
    // super-vertex ids: C[v]; round 1 is the item's own graph
    for (int i = threadIdx.x; i < n; i += IB) st(&s.C[i], i);
    bool first = true;
    for (;;) {
      // ---- round setup: keys, union-find, bitmaps (levels 0..bound)
      int words = (bound + 1) * s.ls;
      for (int w = threadIdx.x; w < words; w += IB) st(&s.bits[w], (uint64_t)0);
      if (threadIdx.x == 0) sh.levelmask = 0;
      for (int x = threadIdx.x; x < n; x += IB) {
        st(&s.A[x], 0);
        st(&s.B[x], x);
      }
      __syncthreads();
      for (int x = threadIdx.x; x < n; x += IB)
        if (ld(&s.C[x]) == x) bit_set(s, 0, x, &sh.levelmask);
      __syncthreads();
      // ---- maximum-adjacency scan
      int round_steps = 0;
      for (;;) {
        if (threadIdx.x < 64) {
          int x = 0;
          if (threadIdx.x == 0) x = bit_pick(s, ld(&sh.levelmask));
          x = __shfl(x, 0, 64);
          if (x >= 0) {
            int top = ld(&s.A[x]);
            top = top < bound ? top : bound;
            if ((int)threadIdx.x <= top) bit_clear(s, threadIdx.x, x, &sh.levelmask);
          }
          if (threadIdx.x == 0) sh.vi[2] = x;
        }
        __syncthreads();
        int x = sh.vi[2];
        if (x == -2 || (x >= 0 && round_steps >= n)) {  // guard: a scan takes at most n steps
          if (threadIdx.x == 0) err(A, WCC_EHIP);
          x = -1;
        }
        if (x < 0) break;
        steps++;
        round_steps++;
        const int32_t *lst;
        int cntx;
        if (first) {
          lst = ar.adj + ar.rs[d.b + x];
          cntx = ar.rd[d.b + x];
        } else {
          lst = A.sEdge + d.eb + ld(&s.E[x]);
          cntx = ld(&s.D[x]);
        }
        for (int e = threadIdx.x; e < cntx; e += IB) {
          int y = first ? lst[e] : ld(&lst[e]);
          if (!bit_test(s, 0, y)) continue;  // already scanned
          int nw = atomicAdd(&s.A[y], 1) + 1;
          if (nw <= bound) bit_set(s, nw, y, &sh.levelmask);
          if (nw >= bound) uf_unite(s.B, x, y);  // contractible: key reached the bound
        }
        __syncthreads();
      }
      rounds++;
      // ---- contraction: new id = smallest member of each merged group
      for (int x = threadIdx.x; x < n; x += IB)
        if (ld(&s.C[x]) == x) st(&s.B[x], uf_find(s.B, x));
      __syncthreads();
      int reps = 0;
      for (int v = threadIdx.x; v < n; v += IB) {
        int c = ld(&s.B[ld(&s.C[v])]);
        st(&s.C[v], c);
        reps += (c == v);
      }
      reps = block_sum<IB>(reps, sh.red);
      if (reps <= 1) break;
      first = false;
      // ---- crossing lists of the contracted graph (D = weighted degree, E = start)
      for (int x = threadIdx.x; x < n; x += IB) st(&s.D[x], 0);
      __syncthreads();
      for (int v = threadIdx.x; v < n; v += IB) {
        int a = ld(&s.C[v]);
        int64_t r0 = ar.rs[d.b + v];
        int rdeg = ar.rd[d.b + v];
        int c = 0;
        for (int e = 0; e < rdeg; e++) c += ld(&s.C[ar.adj[r0 + e]]) != a;
        if (c) atomicAdd(&s.D[a], c);
      }
      __syncthreads();
      int carry = 0;
      for (int base = 0; base < n; base += IB) {
        int x = base + threadIdx.x;
        int v = x < n ? ld(&s.D[x]) : 0;
        int tot;
        int pre = block_excl_scan<IB>(v, sh.red, &tot);
        if (x < n) {
          st(&s.E[x], carry + pre);
          st(&s.A[x], carry + pre);  // fill cursor
        }
        carry += tot;
      }
      __syncthreads();
      for (int v = threadIdx.x; v < n; v += IB) {
        int a = ld(&s.C[v]);
        int64_t r0 = ar.rs[d.b + v];
        int rdeg = ar.rd[d.b + v];
        for (int e = 0; e < rdeg; e++) {
          int bb = ld(&s.C[ar.adj[r0 + e]]);
          if (bb != a) st(&A.sEdge[d.eb + atomicAdd(&s.A[a], 1)], bb);
        }
      }
      __syncthreads();
      // ---- degree check: smallest id of minimum weighted degree, strict improvement
      unsigned long long dm = ~0ull;
      for (int x = threadIdx.x; x < n; x += IB)
        if (ld(&s.C[x]) == x) {
          unsigned long long v = ((unsigned long long)(uint32_t)ld(&s.D[x]) << 32) | (uint32_t)x;
          dm = v < dm ? v : dm;
        }
      dm = block_min_u64<IB>(dm, sh.redu);
      int dmin = (int)(dm >> 32), xmin = (int)(dm & 0xffffffffu);
      if (dmin < bound) {
        bound = dmin;
        s_kind = 2;
        for (int v = threadIdx.x; v < n; v += IB) st(&s.F[v], (int32_t)(ld(&s.C[v]) == xmin));
        __syncthreads();
        if (bound <= 1) break;
      }
    }
  }
  if (s_kind != 2)
    for (int v = threadIdx.x; v < n; v += IB) st(&s.F[v], (int32_t)(s_kind == 1 && v == dv));
  __syncthreads();
  *steps_out += steps;
  *rounds_out += rounds;
  return bound;
}

// ---------------------------------------------------------------- one item
DEV void process_item(const ItemArgs &A, const ItemDesc &d, uint64_t *dyn, int item_index, Sh &sh) {
  const Arena &ar = A.ar[d.depth & 1];
  int n = d.n;
  int k = (int)wcc_k_of(A.crit, n, A.lin_num, A.lin_den);
  int set = A.split_only ? A.split_set[item_index] : -1;
  int cap = A.split_only ? A.split_cap[set] : k;
  int lv = (cap < MAX_LEVEL ? cap : MAX_LEVEL) + 1;
  St s;
  s.n = n;
  s.nw0 = (n + 63) / 64;
  s.nw1 = (s.nw0 + 63) / 64;
  s.nw2 = (s.nw1 + 63) / 64;
  s.ls = s.nw0 + s.nw1 + s.nw2;
  // LDS footprint in 32-bit words: 6 int arrays and the bitmaps (8-byte words)
  long long need = 6LL * n + 2LL * lv * s.ls + 2;
  if (need <= A.lds_words) {
    uint64_t *bits = dyn;
    int32_t *w = (int32_t *)(dyn + (size_t)lv * s.ls);
    s.bits = bits;
    s.A = w;
    s.B = w + n;
    s.C = w + 2 * n;
    s.D = w + 3 * n;
    s.E = w + 4 * n;
    s.F = w + 5 * n;
  } else {
    s.bits = A.gbits + (size_t)blockIdx.x * A.gbits_words;
    if ((long long)lv * s.ls > A.gbits_words) {
      if (threadIdx.x == 0) err(A, WCC_EUNSUPPORTED);
      return;
    }
    s.A = A.sA + d.b;
    s.B = A.sB + d.b;
    s.C = A.sC + d.b;
    s.D = A.sD + d.b;
    s.E = A.sE + d.b;
    s.F = A.sF + d.b;
  }
  long long steps = 0, rounds = 0;

  if (A.split_only) {
    // mincut_split: disconnected -> 0 and the component of the first vertex
    int nc = item_cc(s, ar, d, false, 0, sh);
    int lam;
    if (n < 2) {
      lam = 0;
      for (int i = threadIdx.x; i < n; i += IB) st(&s.F[i], 0);
      __syncthreads();
    } else if (nc > 1) {
      lam = 0;
      for (int i = threadIdx.x; i < n; i += IB) st(&s.F[i], (int32_t)(ld(&s.B[i]) == 0));
      __syncthreads();
    } else {
      lam = item_mincut(A, s, ar, d, cap, sh, &steps, &rounds);
    }
    int64_t p0 = A.split_pos[set];
    for (int i = threadIdx.x; i < n; i += IB) A.split_side[p0 + i] = (uint8_t)ld(&s.F[i]);
    if (threadIdx.x == 0) {
      A.split_lambda[set] = lam;
      atomicAdd(&A.cnt[CNT_STEPS], (unsigned long long)steps);
      atomicAdd(&A.cnt[CNT_ROUNDS], (unsigned long long)rounds);
      atomicAdd(&A.cnt[CNT_MINCUTS], 1ull);
    }
    __syncthreads();
    return;
  }

  if (d.flags & ITEM_CCR) {
    int nc = item_cc(s, ar, d, false, 0, sh);
    if (nc > 1) {
      item_rebuild(A, s, d, A.s_pre, sh);
      return;
    }
    if (n <= A.s_pre) return;
  }
  if (threadIdx.x == 0) atomicAdd(&A.cnt[CNT_ITEMS], 1ull);
  if (A.mode == WCC_PRUNE_KCORE) {
    int removed = item_peel(s, ar, d, k, sh);
    if (removed > 0) {
      if (removed < n) {
        item_cc(s, ar, d, true, k, sh);
        item_rebuild(A, s, d, A.s_post, sh);
      }
      return;
    }
  } else if (d.m == 0) {
    return;  // Alg. 3 tests only sets with at least one edge
  }
  int lam = item_mincut(A, s, ar, d, k, sh, &steps, &rounds);
  // record: |S| and the order-free hash of S's global ids
  int ss = 0;
  unsigned long long hs = 0;
  if (threadIdx.x == 0) sh.hsum = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += IB)
    if (ld(&s.F[i])) {
      ss++;
      hs += vhash(ar.vtx[d.b + i]);
    }
  if (hs) atomicAdd(&sh.hsum, hs);
  ss = block_sum<IB>(ss, sh.red);
  if (threadIdx.x == 0) {
    atomicAdd(&A.cnt[CNT_MINCUTS], 1ull);
    atomicAdd(&A.cnt[CNT_STEPS], (unsigned long long)steps);
    atomicAdd(&A.cnt[CNT_ROUNDS], (unsigned long long)rounds);
    if (A.rec) {
      unsigned long long r = atomicAdd(&A.cnt[CNT_RECORDS], 1ull);
      if ((long long)r < A.rec_cap) {
        wcc_record rc;
        rc.minv = ar.vtx[d.b];
        rc.n = n;
        rc.k = k;
        rc.lambda = lam;
        rc.ssize = ss;
        rc.reserved = 0;
        rc.shash = sh.hsum;
        A.rec[r] = rc;
      }
    }
  }
  if (lam >= k) {  // cut > f(n): save the set under its smallest global id
    int key = ar.vtx[d.b];
    for (int i = threadIdx.x; i < n; i += IB) A.acc[ar.vtx[d.b + i]] = key;
    if (threadIdx.x == 0) atomicAdd(&A.cnt[CNT_ACCEPTED], 1ull);
    __syncthreads();
    return;
  }
  // split along the cut: label each side by its smallest member
  unsigned long long mS = ~0ull, mC = ~0ull;
  for (int i = threadIdx.x; i < n; i += IB) {
    if (ld(&s.F[i])) mS = (unsigned long long)i < mS ? (unsigned long long)i : mS;
    else mC = (unsigned long long)i < mC ? (unsigned long long)i : mC;
  }
  mS = block_min_u64<IB>(mS, sh.redu);
  mC = block_min_u64<IB>(mC, sh.redu);
  for (int i = threadIdx.x; i < n; i += IB) st(&s.B[i], ld(&s.F[i]) ? (int)mS : (int)mC);
  __syncthreads();
  item_rebuild(A, s, d, A.s_post, sh);
}

__global__ void __launch_bounds__(IB) k_items(ItemArgs A) {
  extern __shared__ uint64_t dyn[];
  __shared__ Sh sh;
  __shared__ int cur;
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(A.next, 1);
    __syncthreads();
    int it = cur;
    __syncthreads();
    if (it >= A.nitems) break;
    ItemDesc d = A.items[it];
    process_item(A, d, dyn, it, sh);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- item ordering
// keys for a descending-size sort (largest items first)
__global__ void k_item_keys(const ItemDesc *items, int32_t n, uint32_t *keys, uint32_t *vals) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  keys[i] = 0x7fffffffu - (uint32_t)items[i].n;
  vals[i] = (uint32_t)i;
}
__global__ void k_item_gather(const ItemDesc *in, const uint32_t *order, int32_t n, ItemDesc *out,
                              const int32_t *set_in, int32_t *set_out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = in[order[i]];
  if (set_in) set_out[i] = set_in[order[i]];
}

// ---------------------------------------------------------------- relabel
__global__ void k_mark_mins(const int32_t *acc, int64_t N, int32_t *mark) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < N) mark[v] = acc[v] == v;
}
__global__ void k_relabel(const int32_t *acc, const int32_t *rank, int64_t N, int32_t *out) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  int32_t a = acc[v];
  out[v] = a >= 0 ? rank[a] : -1;
}

}  // namespace

int items_block() { return IB; }
int items_max_level() { return MAX_LEVEL; }

// words of 64-bit bitmap storage one workgroup needs for an item of n vertices
int64_t items_bitmap_words(int64_t n, int cap) {
  int64_t nw0 = (n + 63) / 64, nw1 = (nw0 + 63) / 64, nw2 = (nw1 + 63) / 64;
  int lv = (cap < MAX_LEVEL ? cap : MAX_LEVEL) + 1;
  return (int64_t)lv * (nw0 + nw1 + nw2);
}

int items_launch(const ItemArgs &A, int grid, size_t lds_bytes, hipStream_t s) {
  if (A.nitems <= 0) return WCC_OK;
  hipLaunchKernelGGL(k_items, dim3(grid), dim3(IB), lds_bytes, s, A);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

int items_sort_desc(const ItemDesc *in, int32_t n, ItemDesc *out, const int32_t *set_in, int32_t *set_out,
                    uint32_t *k1, uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes,
                    hipStream_t s, int max_n) {
  if (n <= 0) return WCC_OK;
  hipLaunchKernelGGL(k_item_keys, dim3((n + 255) / 256), dim3(256), 0, s, in, n, k1, v1);
  HIP_TRY(hipGetLastError());
  int bits = 31, alt = 0;
  (void)max_n;
  int rc = prim_radix_sort_pairs(k1, v1, k2, v2, n, bits, tmp, tmp_bytes, s, &alt);
  if (rc) return rc;
  hipLaunchKernelGGL(k_item_gather, dim3((n + 255) / 256), dim3(256), 0, s, in, alt ? v2 : v1, n, out,
                     set_in, set_out);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

int items_relabel(const int32_t *acc, int64_t N, int32_t *mark, int32_t *rank, int32_t *out, void *tmp,
                  size_t tmp_bytes, hipStream_t s) {
  if (N <= 0) return WCC_OK;
  unsigned g = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(k_mark_mins, dim3(g), dim3(256), 0, s, acc, N, mark);
  int rc = prim_excl_scan_i32(mark, rank, N, nullptr, tmp, tmp_bytes, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_relabel, dim3(g), dim3(256), 0, s, acc, (const int32_t *)rank, N, out);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}
