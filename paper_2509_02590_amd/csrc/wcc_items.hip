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
// Placement.  The arrays the scan touches every step (keys A, union-find B, list lengths
// D and starts E, row starts R and the level bitmaps) live in LDS when they fit the
// launch's LDS budget, otherwise in global scratch; the contraction marks, the
// super-vertex ids C and the item's own adjacency (as 16-bit ids) join them in LDS when
// room is left.  The cut side F and the crossing lists of later rounds live in global
// scratch.  Items of one launch are disjoint, so position- and entry-indexed scratch
// slices never overlap.
//
// The maximum-adjacency scan is run by one wavefront.  For every key level j in 0..bound
// a bitmap holds the unscanned super-vertices whose key is >= j (level 0 = all
// unscanned); the next vertex is the smallest id of the highest non-empty level.  A key
// increment sets exactly one bit, so concurrent increments commute; contractible edges
// are only marked during the scan (a store nobody waits for) and merged with a
// union-find pass afterwards.  The list of the likely next vertex is loaded into
// registers while the current one is processed.  Before the scans, a certificate of
// lambda >= bound (edge-disjoint spanning forests) ends most items whose cut reaches the
// bound.
//
// Passes over all edges of an item are entry-parallel: each thread takes 16 consecutive
// entries and finds their owners by a binary search in the LDS copy of the row starts.
#include <mutex>

#include "wcc_internal.h"

// The phases below are compiled as separate functions (not inlined into the three
// placements of process_item_t): one copy each keeps the code object small and the build
// fast, and a phase's registers are not live across the others.
#define NOINL __device__ __attribute__((noinline))

namespace {

// threads per item workgroup: 256, or 512 for launches with one workgroup per CU (more
// loads in flight in the item-wide passes); the loops stride by the launch's block size
constexpr int IB_SMALL = 256;
constexpr int IB_MAX = 512;
constexpr int NW_MAX = IB_MAX / 64;
DEV int ib() { return (int)blockDim.x; }
constexpr int CH = 16;   // entries per thread per chunk in entry-parallel passes
constexpr int RV = 8;    // vertices per thread per round in the rebuild's vertex passes
constexpr int NPACK = 4; // children placed by one packed block scan in the rebuild

struct Sh {
  int red[NW_MAX + 1];
  long long red64[NW_MAX + 1];
  unsigned long long redu[NW_MAX + 1];
  unsigned long long hsum;
  int vi[8];
  int crep[NPACK], cstart[NPACK];  // rebuild: first children's representatives and starts
  int own_lo;                       // entry_rounds: first row of the next round
  int arr[64];                      // low-degree runs: vertices that entered the current class
  ItemDesc keep;  // chained form: the child this workgroup processes next
  int has_keep;
};

struct St {
  int32_t *A, *B, *D, *E, *R;  // LDS or global
  int32_t *C, *F;              // global
  uint64_t *bits;              // LDS or global
  uint64_t *bits1;             // LDS summary levels of global-state items, or nullptr (in bits)
  uint16_t *adj16;             // LDS copy of the item's adjacency, or nullptr
  const int32_t *adjg;         // the item's adjacency in the arena (entry 0 = eb)
  uint8_t *mark;               // global, entry-indexed contraction marks (if no markbits)
  uint32_t *markbits;          // LDS bit array of contraction marks, or nullptr
  int32_t *lists;              // global, entry-indexed crossing lists (rounds >= 2)
  int32_t *own;                // LDS, ib() words: chunk owners of entry rounds, or nullptr
  int n, m;
  int nw0, nw1, nw2, ls;       // bitmap geometry per level
  bool l1;                     // summary level of the bitmaps kept (large items only)
  bool pf;                     // accumulate this item's phase profile
  unsigned long long *prof_cnt; // sub-phase timing slots (profiling runs only)
};

// Pointers that say which memory they address.  The phases are separate functions shared
// by every placement, so a pointer they receive is generic; rebuilding it from its LDS
// offset (low 32 bits) or as a global address lets the compiler emit LDS (ds_*) or
// global (global_*) instructions instead of flat ones.  (A plain cast to the LDS address
// space and back is folded away, hence the integer round trip.)
template <typename T>
DEV T *as_lds(T *p) {
  return (T *)(__attribute__((address_space(3))) T *)(uintptr_t)(uint32_t)(uintptr_t)p;
}
template <typename T>
DEV T *as_glb(T *p) {
  return (T *)(__attribute__((address_space(1))) T *)(uintptr_t)p;
}
// The item state with every pointer typed for its placement: LDS = scan arrays (A, B, D,
// E, R, bitmaps) in LDS, CL = super-vertex ids C in LDS; the optional mark bits and 16-bit
// adjacency are LDS arrays when present.
template <bool LDS, bool CL>
DEV St typed_st(const St &in) {
  St s = in;
  s.F = as_glb(s.F);
  s.adjg = as_glb(s.adjg);
  s.mark = as_glb(s.mark);
  s.lists = as_glb(s.lists);
  s.own = s.own ? as_lds(s.own) : nullptr;
  s.bits1 = s.bits1 ? as_lds(s.bits1) : nullptr;
  if constexpr (LDS) {
    s.A = as_lds(s.A);
    s.B = as_lds(s.B);
    s.D = as_lds(s.D);
    s.E = as_lds(s.E);
    s.R = as_lds(s.R);
    s.bits = as_lds(s.bits);
    s.markbits = s.markbits ? as_lds(s.markbits) : nullptr;
    s.adj16 = s.adj16 ? as_lds(s.adj16) : nullptr;
  } else {
    s.A = as_glb(s.A);
    s.B = as_glb(s.B);
    s.D = as_glb(s.D);
    s.E = as_glb(s.E);
    s.R = as_glb(s.R);
    s.bits = as_glb(s.bits);
  }
  if constexpr (CL) s.C = as_lds(s.C);
  else s.C = as_glb(s.C);
  return s;
}

DEV int row_end(const St &s, int x) { return x + 1 < s.n ? ldr(&s.R[x + 1]) : s.m; }

// contraction marks: one bit per list entry in LDS when it fits, else one byte in global
DEV void mark_set(const St &s, int e) {
  if (s.markbits) atomicOr(&s.markbits[e >> 5], 1u << (e & 31));
  else st(&s.mark[e], 1);
}
DEV bool mark_get(const St &s, int e) {
  return s.markbits ? ((ld(&s.markbits[e >> 5]) >> (e & 31)) & 1u) : ld(&s.mark[e]) != 0;
}
DEV void mark_clear(const St &s, int total) {
  if (s.markbits)
    for (int w = threadIdx.x; w < (total + 31) / 32; w += ib()) st(&s.markbits[w], 0u);
  else
    for (int e = threadIdx.x; e < total; e += ib()) st(&s.mark[e], 0);
}
DEV int adj_at(const St &s, int e) { return s.adj16 ? (int)s.adj16[e] : s.adjg[e]; }

// marks of the 16 entries [base, base + 16) below total as a bit mask (base % 16 == 0)
DEV uint32_t mark_chunk(const St &s, int base, int total) {
  uint32_t mk = 0;
  if (s.markbits) {
    mk = (ld(&s.markbits[base >> 5]) >> (base & 31)) & 0xFFFFu;
  } else {
#pragma unroll
    for (int i = 0; i < 16; i++)
      if (base + i < total && ld(&s.mark[base + i]) != 0) mk |= 1u << i;
  }
  if (total - base < 16) mk &= (1u << (total - base)) - 1u;
  return mk;
}

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

// uf_unite that reports whether this call joined two trees (hooked a root).
DEV bool uf_link(int32_t *P, int a, int b) {
  for (;;) {
    a = uf_find(P, a);
    b = uf_find(P, b);
    if (a == b) return false;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    if (atomicCAS(&P[a], a, b) == a) return true;
  }
}

// a[key] += 1 for every lane with act; the lanes holding the same key as the first active
// lane share one atomic (counts of a few large groups would otherwise serialise on one
// address).  Call with the whole wavefront converged.
DEV void count_agg(int32_t *a, int key, bool act) {
  uint64_t m = __ballot(act);
  if (!m) return;
  int leader = __ffsll((long long)m) - 1;
  int k0 = __shfl(key, leader, 64);
  uint64_t same = __ballot(act && key == k0);
  if (act && key != k0) atomicAdd(&a[key], 1);
  if ((int)__lane_id() == leader) atomicAdd(&a[k0], (int)__popcll(same));
}

// Calls body(base, x) for every thread's chunk of CH consecutive entries [base, base + CH)
// of lists stored in ascending owner order (owner x covers [start[x], end(x)), end(x) =
// start[x+1], or total for the last), x = the owner of entry base.  The chunks of one
// round, ib() * CH entries, belong to the threads in order.  With s.own (an LDS array of
// ib() words; items whose state is in global memory) the rows reaching into a round are
// read by the threads together (consecutive rows, one round trip for most rounds) and
// write the owner of every chunk start they hold into s.own; the row of the round's last
// entry is where the next round's rows begin.  Otherwise each thread finds its owner by
// binary search.  With s.own the call contains barriers: the whole block must make it.
template <typename B>
DEV void entry_rounds(const St &s, Sh &sh, const int32_t *start, int n, int total, B body) {
  if (s.own) {
    int lo = 0;
    for (int blk = 0; blk < total; blk += ib() * CH) {
      const int bend = blk + ib() * CH < total ? blk + ib() * CH : total;
      for (int r = lo + (int)threadIdx.x; r < n; r += ib()) {
        int r0 = ldr(&start[r]);
        if (r0 >= bend) break;
        int r1 = r + 1 < n ? ldr(&start[r + 1]) : total;
        int a = r0 > blk ? r0 : blk, b = r1 < bend ? r1 : bend;
        if (a < b) {
          for (int c = (a - blk + CH - 1) / CH; c < (b - blk + CH - 1) / CH; c++) s.own[c] = r;
          if (b == bend) sh.own_lo = r;
        }
      }
      __syncthreads();
      const int base = blk + (int)threadIdx.x * CH;
      const int x = base < total ? s.own[threadIdx.x] : 0;
      lo = sh.own_lo;
      __syncthreads();
      if (base < total) body(base, x);
    }
  } else {
    for (int base = threadIdx.x * CH; base < total; base += ib() * CH) {
      int lo = 0, hi = n - 1;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (ldr(&start[mid]) <= base) lo = mid;
        else hi = mid - 1;
      }
      body(base, lo);
    }
  }
}

// Calls f(x, e, y) for every entry e in [0, total) of lists stored in ascending owner
// order, y = get(e) (entry_rounds' chunks).
template <typename G, typename F>
DEV void for_entries(const St &s, Sh &sh, const int32_t *start, int n, int total, G get, F f) {
  entry_rounds(s, sh, start, n, total, [&](int base, int x) {
    int yv[CH];
#pragma unroll
    for (int i = 0; i < CH; i++) yv[i] = base + i < total ? get(base + i) : 0;
    int xend = x + 1 < n ? ldr(&start[x + 1]) : total;
#pragma unroll
    for (int i = 0; i < CH; i++) {
      int e = base + i;
      if (e < total) {
        while (e >= xend) {
          x++;
          xend = x + 1 < n ? ldr(&start[x + 1]) : total;
        }
        f(x, e, yv[i]);
      }
    }
  });
}

// for_entries that leaves out the entries of owners x with skip(x): a chunk that lies
// inside skipped rows only is passed over without loading it.
template <typename S, typename G, typename F>
DEV void for_entries_skip(const St &s, Sh &sh, const int32_t *start, int n, int total, S skip, G get, F f) {
  entry_rounds(s, sh, start, n, total, [&](int base, int x) {
    int xend = x + 1 < n ? ldr(&start[x + 1]) : total;
    bool sk = skip(x);
    // the chunk is passed over when every owner it touches is skipped
    bool all = sk;
    for (int z = x, zend = xend; all && zend < base + CH && zend < total;) {
      z++;
      zend = z + 1 < n ? ldr(&start[z + 1]) : total;
      all = skip(z);
    }
    if (all) return;
    int yv[CH];
#pragma unroll
    for (int i = 0; i < CH; i++) yv[i] = base + i < total ? get(base + i) : 0;
#pragma unroll
    for (int i = 0; i < CH; i++) {
      int e = base + i;
      if (e < total) {
        while (e >= xend) {
          x++;
          xend = x + 1 < n ? ldr(&start[x + 1]) : total;
          sk = skip(x);
        }
        if (!sk) f(x, e, yv[i]);
      }
    }
  });
}

// Calls f(x, e, y) for the marked entries e in [0, total) only (lists stored in ascending
// owner order, as for for_entries); chunks without a mark are passed over unread.
template <typename G, typename F>
DEV void for_marked_entries(const St &s, Sh &sh, const int32_t *start, int n, int total, G get, F f) {
  static_assert(CH == 16, "mark_chunk reads 16 entries");
  entry_rounds(s, sh, start, n, total, [&](int base, int x) {
    uint32_t mk = mark_chunk(s, base, total);
    if (!mk) return;
    int xend = x + 1 < n ? ldr(&start[x + 1]) : total;
    int yv[CH];
#pragma unroll
    for (int i = 0; i < CH; i++) yv[i] = (mk >> i) & 1u ? get(base + i) : 0;
#pragma unroll
    for (int i = 0; i < CH; i++) {
      if (!((mk >> i) & 1u)) continue;
      int e = base + i;
      while (e >= xend) {
        x++;
        xend = x + 1 < n ? ldr(&start[x + 1]) : total;
      }
      f(x, e, yv[i]);
    }
  });
}

// ---------------------------------------------------------------- bitmap levels
// (level j < 64 and ls < 2^24: a 24-bit multiply)
DEV uint64_t *lvl0(const St &s, int j) { return s.bits + __umul24((unsigned)j, (unsigned)s.ls); }
// GL (items whose state is in global memory): the summary levels are the LDS array bits1
template <bool GL>
DEV uint64_t *lvl1(const St &s, int j) {
  if constexpr (GL) return s.bits1 + __umul24((unsigned)j, (unsigned)s.nw1);
  else return s.bits + __umul24((unsigned)j, (unsigned)s.ls) + s.nw0;
}

// Level j: a bit per vertex (L0) and, for large items, a summary bit per L0 word (L1)
// that is set whenever a bit of that word is set but only cleared lazily.  Setting and
// clearing need no returned values, so they never stall the scan.
template <bool GL>
DEV void bit_set(const St &s, int j, int y) {
  atomicOr((unsigned long long *)&lvl0(s, j)[y >> 6], 1ull << (y & 63));
  if (s.l1) atomicOr((unsigned long long *)&lvl1<GL>(s, j)[y >> 12], 1ull << ((y >> 6) & 63));
}

DEV void bit_clear(const St &s, int j, int x) {
  atomicAnd((unsigned long long *)&lvl0(s, j)[x >> 6], ~(1ull << (x & 63)));
}

DEV uint64_t readlane64(uint64_t v, int l) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(v >> 32), l) << 32) |
         (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
}

// Wavefront-cooperative search of level j: its smallest member, -1 when it is empty, -2
// on an inconsistent bitmap.  All lanes return it.  Summary words whose L0 words all
// turned empty are reset.
template <bool GL>
DEV int level_first(const St &s, int j) {
  const int lane = __lane_id();
  uint64_t *L1 = lvl1<GL>(s, j);
  const uint64_t *L0 = lvl0(s, j);
  if (!s.l1) {
    // small items keep no summary: a wavefront reads 64 L0 words at a time
    for (int c0 = 0; c0 < s.nw0; c0 += 64) {
      uint64_t w0 = c0 + lane < s.nw0 ? ld(&L0[c0 + lane]) : 0ull;
      uint64_t m0 = __ballot(w0 != 0);
      if (m0) {
        int b = __ffsll((long long)m0) - 1;
        uint64_t wsel = readlane64(w0, b);
        int x = (c0 + b) * 64 + __ffsll((long long)wsel) - 1;
        return x < s.n ? x : -2;
      }
    }
    return -1;
  }
  for (int c0 = 0; c0 < s.nw1; c0 += 64) {
    uint64_t w1 = c0 + lane < s.nw1 ? ld(&L1[c0 + lane]) : 0ull;
    uint64_t m1 = __ballot(w1 != 0);
    while (m1) {
      int l = __ffsll((long long)m1) - 1;
      int i1 = c0 + l;
      int i0 = i1 * 64 + lane;
      uint64_t w0 = i0 < s.nw0 ? ld(&L0[i0]) : 0ull;
      uint64_t m0 = __ballot(w0 != 0);
      if (m0) {
        int b = __ffsll((long long)m0) - 1;
        uint64_t wsel = readlane64(w0, b);
        int x = (i1 * 64 + b) * 64 + __ffsll((long long)wsel) - 1;
        return x < s.n ? x : -2;
      }
      if (lane == 0) st(&L1[i1], 0ull);  // stale summary word
      m1 &= m1 - 1;
    }
  }
  return -1;
}

// The smallest id in the highest non-empty level, searching down from *j (every level
// above *j is empty); -1 when every super-vertex is scanned, -2 on an inconsistency.
// *j receives the level found.
template <bool GL>
DEV int bit_pick(const St &s, int *j) {
  for (int l = *j; l >= 0; l--) {
    int x = level_first<GL>(s, l);
    if (x != -1) {
      *j = l;
      return x;
    }
  }
  *j = 0;
  return -1;
}

// Wavefront reductions without the LDS crossbar: DPP exchanges inside each row of 16
// lanes (xor 1, xor 2, half-row mirror, row mirror), then the four row results are read
// with readlane.  Call with all 64 lanes active; the result is uniform.
template <bool MAX>
DEV int wave_red_i(int v) {
  auto op = [](int a, int b) { return MAX ? (a > b ? a : b) : (a < b ? a : b); };
  v = op(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));  // row_mirror
  int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
  int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
  return op(op(r0, r1), op(r2, r3));
}
DEV int wave_max_i(int v) { return wave_red_i<true>(v); }
DEV int wave_min_i(int v) { return wave_red_i<false>(v); }

// ---------------------------------------------------------------- helpers
// optional phase profile: thread 0 adds the 100 MHz wall-clock time since *t to slot ph
DEV void ph_mark(const ItemArgs &A, const St &s, int ph, unsigned long long *t) {
  (void)A;
  if (!s.pf || threadIdx.x != 0) return;
  unsigned long long now = wall_clock64();
  atomicAdd(&A.cnt[CNT_PH + ph], now - *t);
  *t = now;
}

// sub-phase profile: thread 0 adds the time since *t to CNT_PH slot `slot` (13..15, 16..31)
DEV void sub_mark(const St &s, int slot, unsigned long long *t) {
  if (!s.pf || threadIdx.x != 0) return;
  unsigned long long now = wall_clock64();
  atomicAdd(&s.prof_cnt[slot - 16], now - *t);
  *t = now;
}

DEV void err(const ItemArgs &A, int code) {
  atomicMin((long long *)&A.cnt[CNT_ERR], (long long)code);
}

// Connected components of the item restricted to alive vertices (alive = A[i] >= kmin
// when use_deg, else all).  B[i] = smallest vertex of i's component, -1 if dead.
// Returns the number of components.  Uses E as scratch.
//
// Union-find with roots kept at the smallest id, in two passes over the edges (the
// sampling scheme of Afforest, Sutton et al. 2018): first every alive vertex is united
// with its first two alive neighbours, which already joins most of a connected item into
// one tree; c = the root with the most members.  Then every edge is united from the side
// of an endpoint that is not (yet) a child of c; an edge skipped from both sides joins two
// members of c's tree, so the components are exact.  Rows of c's members are not read.
template <bool LDS, bool CL>
NOINL int item_cc(const St &s_in, bool use_deg, int kmin, Sh &sh_in) {
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  int n = s.n;
  unsigned long long q = s.pf ? wall_clock64() : 0;
  for (int i = threadIdx.x; i < n; i += ib()) {
    bool al = !use_deg || ld(&s.A[i]) >= kmin;
    st(&s.B[i], al ? i : -1);
    st(&s.E[i], 0);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += ib()) {
    if (ld(&s.B[i]) < 0) continue;
    int r1 = row_end(s, i), found = 0;
    for (int e = ldr(&s.R[i]); e < r1 && found < 2; e++) {
      int j = adj_at(s, e);
      if (ld(&s.B[j]) >= 0) {
        uf_unite(s.B, i, j);
        found++;
      }
    }
  }
  __syncthreads();
  sub_mark(s, 16, &q);
  for (int base = 0; base < n; base += ib()) {
    int i = base + threadIdx.x;
    int r = -1;
    if (i < n && ld(&s.B[i]) >= 0) {
      r = uf_find(s.B, i);
      st(&s.B[i], r);
    }
    count_agg(s.E, r, r >= 0);
  }
  __syncthreads();
  sub_mark(s, 17, &q);
  unsigned long long best = ~0ull;
  for (int i = threadIdx.x; i < n; i += ib()) {
    int c = ldr(&s.E[i]);
    if (c > 0) {
      unsigned long long v = ((unsigned long long)(uint32_t)(0x7fffffff - c) << 32) | (uint32_t)i;
      best = v < best ? v : best;
    }
  }
  best = block_min_u64<IB_MAX>(best, sh.redu);
  const int cs = best == ~0ull ? -1 : (int)(best & 0xffffffffu);
  sub_mark(s, 18, &q);
  for_entries_skip(
      s, sh, s.R, n, s.m, [&](int x) { int b = ld(&s.B[x]); return b < 0 || b == cs; },
      [&](int e) { return adj_at(s, e); },
      [&](int i, int, int j) {
        if (ld(&s.B[j]) >= 0) uf_unite(s.B, i, j);
      });
  __syncthreads();
  sub_mark(s, 29, &q);
  int roots = 0;
  for (int i = threadIdx.x; i < n; i += ib()) {
    if (ld(&s.B[i]) < 0) continue;
    int r = uf_find(s.B, i);
    roots += (r == i);
    st(&s.B[i], r);
  }
  int nr = block_sum<IB_MAX>(roots, sh.red);  // includes barriers
  sub_mark(s, 30, &q);
  return nr;
}

// ---------------------------------------------------------------- rebuild children
// B[i]: child label (the child's smallest local id) or -1.  Children larger than gate
// are compacted into the other arena inside [b, b+n) / [eb, eb+m) and pushed.
// Uses A (sizes), D (child starts), E (new positions), C (row offsets by new position)
// and F (write cursors by new position).
template <bool LDS, bool CL>
NOINL void item_rebuild(const ItemArgs &A, const St &s_in, const ItemDesc &d, int gate, Sh &sh_in) {
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  Arena ar = A.ar[d.depth & 1], nx = A.ar[(d.depth + 1) & 1];
  ar.vtx = as_glb(ar.vtx);
  nx.vtx = as_glb(nx.vtx);
  nx.rs = as_glb(nx.rs);
  nx.rd = as_glb(nx.rd);
  nx.adj = as_glb(nx.adj);
  int n = s.n;
  unsigned long long q = s.pf ? wall_clock64() : 0;
  for (int i = threadIdx.x; i < n; i += ib()) st(&s.A[i], 0);
  __syncthreads();
  // child sizes by label (A), then labels of children of gate vertices or fewer dropped;
  // RV vertices per thread and round, their loads issued together
  for (int base = 0; base < n; base += ib() * RV) {
    int L[RV];
#pragma unroll
    for (int k = 0; k < RV; k++) {
      int i = base + k * ib() + threadIdx.x;
      L[k] = i < n ? ldr(&s.B[i]) : -1;
    }
#pragma unroll
    for (int k = 0; k < RV; k++) count_agg(s.A, L[k], L[k] >= 0);
  }
  __syncthreads();
  for (int base = 0; base < n; base += ib() * RV) {
    int L[RV], c[RV];
#pragma unroll
    for (int k = 0; k < RV; k++) {
      int i = base + k * ib() + threadIdx.x;
      L[k] = i < n ? ldr(&s.B[i]) : -1;
    }
#pragma unroll
    for (int k = 0; k < RV; k++) c[k] = L[k] >= 0 ? ldr(&s.A[L[k]]) : gate + 1;
#pragma unroll
    for (int k = 0; k < RV; k++)
      if (c[k] <= gate) st(&s.B[base + k * ib() + threadIdx.x], -1);
  }
  __syncthreads();
  // child starts (D, by representative) and ordinals: one exclusive scan of
  // (1 << 32) + size over the representatives, RV consecutive vertices per thread; the
  // first NPACK children's representatives and starts are kept in sh
  long long carry = 0;
  for (int base = 0; base < n; base += ib() * RV) {
    const int i0 = base + threadIdx.x * RV;
    int sz[RV];
    long long v = 0;
#pragma unroll
    for (int k = 0; k < RV; k++) {
      int i = i0 + k;
      sz[k] = (i < n && ldr(&s.B[i]) == i) ? ldr(&s.A[i]) : 0;
      v += sz[k] ? (1LL << 32) + sz[k] : 0;
    }
    long long tot;
    long long pre = carry + block_excl_scan64<IB_MAX>(v, sh.red64, &tot);
#pragma unroll
    for (int k = 0; k < RV; k++)
      if (sz[k]) {
        int start = (int)(pre & 0xffffffffLL), o = (int)(pre >> 32);
        st(&s.D[i0 + k], start);
        if (o < NPACK) {
          sh.crep[o] = i0 + k;
          sh.cstart[o] = start;
        }
        pre += (1LL << 32) + sz[k];
      }
    carry += tot;
  }
  const int K = (int)(carry & 0xffffffffLL), NC = (int)(carry >> 32);
  __syncthreads();
  if (K == 0) return;
  sub_mark(s, 31, &q);
  // stable new positions (E[i] = new position: the child's start plus the number of its
  // vertices before i)
  if (NC <= NPACK) {
    // at most NPACK children: one block scan of NPACK 16-bit counters per round of
    // ib() * RV consecutive vertices (at most 65535 of one child per round)
    static_assert(NPACK * 16 <= 64 && IB_MAX * RV <= 65535, "packed child counters");
    int crep[NPACK], cnext[NPACK];
#pragma unroll
    for (int c = 0; c < NPACK; c++) {
      crep[c] = c < NC ? sh.crep[c] : -2;
      cnext[c] = c < NC ? sh.cstart[c] : 0;
    }
    for (int base = 0; base < n; base += ib() * RV) {
      const int i0 = base + threadIdx.x * RV;
      int o[RV];
      unsigned long long v = 0;
#pragma unroll
      for (int k = 0; k < RV; k++) {
        int L = i0 + k < n ? ldr(&s.B[i0 + k]) : -1;
        int c = -1;
#pragma unroll
        for (int cc = 0; cc < NPACK; cc++) c = L == crep[cc] ? cc : c;
        o[k] = c;
        if (c >= 0) v += 1ull << (16 * c);
      }
      long long tot;
      unsigned long long pre = (unsigned long long)block_excl_scan64<IB_MAX>((long long)v, sh.red64, &tot);
#pragma unroll
      for (int k = 0; k < RV; k++)
        if (o[k] >= 0) {
          int c = o[k];
          int b = c == 0 ? cnext[0] : c == 1 ? cnext[1] : c == 2 ? cnext[2] : cnext[3];
          st(&s.E[i0 + k], b + (int)((pre >> (16 * c)) & 0xffffu));
          pre += 1ull << (16 * c);
        }
#pragma unroll
      for (int c = 0; c < NPACK; c++) cnext[c] += (int)(((unsigned long long)tot >> (16 * c)) & 0xffffu);
    }
    __syncthreads();
  } else {
    // more children: wave 0 walks the item in order with a cursor per child (D[L] ends
    // at start + size and is restored after)
    if (threadIdx.x < 64) {
      for (int base = 0; base < n; base += 64) {
        int i = base + threadIdx.x;
        int L = i < n ? ldr(&s.B[i]) : -1;
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
    for (int i = threadIdx.x; i < n; i += ib())
      if (ldr(&s.B[i]) == i) st(&s.D[i], ldr(&s.D[i]) - ldr(&s.A[i]));
  }
  // clear new degrees and cursors
  for (int i = threadIdx.x; i < K; i += ib()) {
    st(&s.C[i], 0);
    st(&s.F[i], 0);
  }
  __syncthreads();
  sub_mark(s, 31, &q);
  // new degrees by new position (C): a thread's CH entries are read and their endpoints'
  // labels gathered at once; one atomic per row run inside the chunk
  entry_rounds(s, sh, s.R, n, s.m, [&](int base, int x) {
    int yv[CH], by[CH];
#pragma unroll
    for (int i = 0; i < CH; i++) yv[i] = base + i < s.m ? s.adjg[base + i] : 0;
#pragma unroll
    for (int i = 0; i < CH; i++) by[i] = base + i < s.m ? ldr(&s.B[yv[i]]) : -2;
    int xend = x + 1 < n ? ldr(&s.R[x + 1]) : s.m;
    int Lx = ldr(&s.B[x]), cnt = 0;
#pragma unroll
    for (int i = 0; i < CH; i++) {
      int e = base + i;
      if (e < s.m) {
        if (e >= xend) {
          if (cnt) atomicAdd(&s.C[ldr(&s.E[x])], cnt);
          cnt = 0;
          do {
            x++;
            xend = x + 1 < n ? ldr(&s.R[x + 1]) : s.m;
          } while (e >= xend);
          Lx = ldr(&s.B[x]);
        }
        cnt += (Lx >= 0 && by[i] == Lx);
      }
    }
    if (cnt) atomicAdd(&s.C[ldr(&s.E[x])], cnt);
  });
  __syncthreads();
  sub_mark(s, 13, &q);
  // row offsets by new position (exclusive scan of C, in place; RV consecutive positions
  // per thread)
  long long ecarry = 0;
  for (int base = 0; base < K; base += ib() * RV) {
    const int p0 = base + threadIdx.x * RV;
    int c[RV];
    long long v = 0;
#pragma unroll
    for (int k = 0; k < RV; k++) {
      c[k] = p0 + k < K ? ldr(&s.C[p0 + k]) : 0;
      v += c[k];
    }
    long long tot;
    long long pre = ecarry + block_excl_scan64<IB_MAX>(v, sh.red64, &tot);
#pragma unroll
    for (int k = 0; k < RV; k++)
      if (p0 + k < K) {
        st(&s.C[p0 + k], (int)pre);
        pre += c[k];
      }
    ecarry += tot;
  }
  int M = (int)ecarry;
  __syncthreads();
  // vertex records of the children
  for (int base = 0; base < n; base += ib() * RV) {
    int L[RV], np[RV], o[RV], o1[RV];
#pragma unroll
    for (int k = 0; k < RV; k++) {
      int i = base + k * ib() + threadIdx.x;
      L[k] = i < n ? ldr(&s.B[i]) : -1;
    }
#pragma unroll
    for (int k = 0; k < RV; k++) np[k] = L[k] >= 0 ? ldr(&s.E[base + k * ib() + threadIdx.x]) : 0;
#pragma unroll
    for (int k = 0; k < RV; k++) {
      o[k] = L[k] >= 0 ? ldr(&s.C[np[k]]) : 0;
      o1[k] = L[k] >= 0 && np[k] + 1 < K ? ldr(&s.C[np[k] + 1]) : M;
    }
#pragma unroll
    for (int k = 0; k < RV; k++)
      if (L[k] >= 0) {
        int i = base + k * ib() + threadIdx.x;
        nx.vtx[d.b + np[k]] = ar.vtx[d.b + i];
        nx.rs[d.b + np[k]] = d.eb + o[k];
        nx.rd[d.b + np[k]] = o1[k] - o[k];
      }
  }
  sub_mark(s, 15, &q);
  // rows: the kept entries of a row run inside a thread's chunk take consecutive slots,
  // reserved with one atomic on the row's cursor (order inside a row is free; a slot is
  // bounded by the row's counted length)
  entry_rounds(s, sh, s.R, n, s.m, [&](int base, int x) {
    int yv[CH], by[CH], own[CH];
#pragma unroll
    for (int i = 0; i < CH; i++) yv[i] = base + i < s.m ? s.adjg[base + i] : 0;
#pragma unroll
    for (int i = 0; i < CH; i++) by[i] = base + i < s.m ? ldr(&s.B[yv[i]]) : -2;
    int xend = x + 1 < n ? ldr(&s.R[x + 1]) : s.m;
    int Lx = ldr(&s.B[x]);
    uint32_t keep = 0;
#pragma unroll
    for (int i = 0; i < CH; i++) {
      int e = base + i;
      own[i] = -1;
      if (e < s.m) {
        if (e >= xend) {
          do {
            x++;
            xend = x + 1 < n ? ldr(&s.R[x + 1]) : s.m;
          } while (e >= xend);
          Lx = ldr(&s.B[x]);
        }
        own[i] = x;
        if (Lx >= 0 && by[i] == Lx) keep |= 1u << i;
      }
    }
    // kept entries from i to the end of i's run
    int suf[CH];
    suf[CH - 1] = (int)((keep >> (CH - 1)) & 1u);
#pragma unroll
    for (int i = CH - 2; i >= 0; i--) suf[i] = (int)((keep >> i) & 1u) + (own[i + 1] == own[i] ? suf[i + 1] : 0);
    int slot = 0, lim = 0, o = 0, start = 0;
#pragma unroll
    for (int i = 0; i < CH; i++) {
      if (own[i] < 0) continue;
      if ((i == 0 || own[i] != own[i - 1]) && suf[i] > 0) {
        int np = ldr(&s.E[own[i]]);
        o = ldr(&s.C[np]);
        lim = (np + 1 < K ? ldr(&s.C[np + 1]) : M) - o;
        start = ldr(&s.D[ldr(&s.B[own[i]])]);
        slot = atomicAdd(&s.F[np], suf[i]);
      }
      if ((keep >> i) & 1u) {
        if (slot < lim) nx.adj[d.eb + o + slot] = ldr(&s.E[yv[i]]) - start;
        slot++;
      }
    }
  });
  sub_mark(s, 14, &q);
  // descriptors of the children
  auto child = [&](int i) {
    int cs = ldr(&s.D[i]);
    int sz = ldr(&s.A[i]);
    int o = ldr(&s.C[cs]);
    int o1 = cs + sz < K ? ldr(&s.C[cs + sz]) : M;
    ItemDesc c;
    c.b = d.b + cs;
    c.n = sz;
    c.eb = d.eb + o;
    c.m = o1 - o;
    c.depth = d.depth + 1;
    c.flags = 0;
    return c;
  };
  // chained form: the workgroup keeps its largest child (the smallest start among equal
  // sizes) and processes it next, without waiting for the level to end, when the child has
  // at least chain_min_n vertices (the long chains of nested splits) and belongs to this
  // launch's size bin: a large-bin workgroup keeps large children only (small ones run
  // several to a CU in the small bin), a small-bin workgroup keeps children whose scan
  // state fits its LDS; the other children go to the lists
  int keep = -1;
  if (A.chain) {
    unsigned long long best = 0;
    for (int i = threadIdx.x; i < n; i += ib())
      if (ldr(&s.B[i]) == i) {
        unsigned long long v = ((unsigned long long)(uint32_t)ldr(&s.A[i]) << 32) | (uint32_t)(0x7fffffff - i);
        best = v > best ? v : best;
      }
    best = ~block_min_u64<IB_MAX>(~best, sh.redu);
    if (best) {
      int i = 0x7fffffff - (int)(best & 0xffffffffu);
      ItemDesc c = child(i);
      int ccap = (int)wcc_k_of(A.crit, c.n, A.lin_num, A.lin_den);
      int64_t need = item_state_words(c.n, c.m, ccap);
      bool big_bin = A.lds_words > A.small_words;
      if (c.n >= A.chain_min_n && (big_bin ? need > A.small_words : (need <= A.lds_words || A.gbits_words > 0)))
        keep = i;
    }
  }
  for (int i = threadIdx.x; i < n; i += ib()) {
    if (ldr(&s.B[i]) != i) continue;
    ItemDesc c = child(i);
    atomicAdd(&A.cnt[CNT_ALG_BYTES], (unsigned long long)(16LL * c.n + 4LL * c.m));
    int ccap = (int)wcc_k_of(A.crit, c.n, A.lin_num, A.lin_den);
    if (i == keep) {
      sh.keep = c;
      sh.has_keep = 1;
    } else if (A.out_big && item_state_words(c.n, c.m, ccap) > A.small_words) {
      int slot = atomicAdd(A.out_big_count, 1);
      if (slot < A.out_big_cap) A.out_big[slot] = c;
      else err(A, WCC_ENOMEM);
    } else {
      int slot = atomicAdd(A.out_count, 1);
      if (slot < A.out_cap) A.out[slot] = c;
      else err(A, WCC_ENOMEM);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------- PAPER-mode leaf peel
// An item (connected, n vertices) whose minimum degree is 1 has canonical cut 1 with
// S = {its smallest vertex of degree 1} (Phase 0 stops at bound 1).  When every size on
// the way fails its cut (k >= 2), WCC as printed therefore removes, one item at a time,
// the smallest vertex of degree 1 and continues with the rest, until no vertex of degree
// 1 is left (the 2-core) or the rest has s_post vertices or fewer.  This computes that
// whole sequence at once, with one split record per removal:
//   * synchronous peel rounds of the vertices of degree <= 1 (the hanging trees); round(u)
//     is the height of u's hanging subtree, and M(u) = the largest id in that subtree;
//     a tree is rooted at its largest id, which is never removed;
//   * the one-at-a-time order is the sort by (M(u), round(u)): the smallest leaf goes
//     first, and a subtree is consumed in the order its largest id allows;
//   * a counting sort by M that places the rounds in order (inside one round the M
//     values differ: equal M means one vertex is the other's ancestor).
// Arrays: A degrees then the removal order, B round (-1 never removed), C M, D the rounds'
// vertices in round order then the suffix minima of the order, E round starts, F bucket
// starts.  Writes the records; returns the number of vertices left when the rest goes on
// (the 2-core, B[i] = its smallest vertex for members, -1 otherwise) or 0.
DEV int block_suffix_min(int v, int carry, Sh &sh, int *chunk_min) {
  const int lane = __lane_id(), w = threadIdx.x >> 6, NW = (int)(blockDim.x >> 6);
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int y = __shfl_down(x, d, 64);
    if (lane + d < 64) x = y < x ? y : x;
  }
  if (lane == 0) sh.red[w] = x;
  __syncthreads();
  int later = carry, all = carry;
  for (int j = 0; j < NW; j++) {
    int r = sh.red[j];
    if (j > w) later = r < later ? r : later;
    all = r < all ? r : all;
  }
  __syncthreads();
  *chunk_min = all;
  return x < later ? x : later;
}

template <bool LDS, bool CL>
NOINL int item_leaf_peel(const ItemArgs &A, const St &s_in, const ItemDesc &d, Sh &sh_in) {
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  Arena ar = A.ar[d.depth & 1];
  ar.vtx = as_glb(ar.vtx);
  const int n = s.n;
  // a tree keeps its largest vertex (it is the last one standing)
  const int pin = (long long)s.m == 2LL * (n - 1) ? n - 1 : -1;
  if (threadIdx.x == 0) sh.vi[0] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += ib()) {
    int dg = row_end(s, i) - ldr(&s.R[i]);
    st(&s.A[i], dg);
    bool leaf = dg <= 1 && i != pin;
    st(&s.B[i], leaf ? 0 : -1);
    if (leaf) st(&s.D[atomicAdd(&sh.vi[0], 1)], i);
  }
  __syncthreads();
  int head = 0, tail = sh.vi[0], r = 0;
  while (head < tail) {
    if (threadIdx.x == 0) {
      st(&s.E[r], head);
      sh.vi[1] = tail;
    }
    __syncthreads();
    for (int f = head + (int)threadIdx.x; f < tail; f += ib()) {
      int u = ld(&s.D[f]);
      int mu = u;
      for (int e = ldr(&s.R[u]), e1 = row_end(s, u); e < e1; e++) {
        int j = adj_at(s, e);
        int bj = ld(&s.B[j]);
        if (bj >= 0 && bj < r) {  // a child: removed in an earlier round
          int mj = ld(&s.C[j]);
          mu = mj > mu ? mj : mu;
        } else if (bj < 0 || bj > r) {  // alive: one neighbour fewer
          int old = atomicSub(&s.A[j], 1);
          if (old == 2 && j != pin) {
            st(&s.B[j], r + 1);
            st(&s.D[atomicAdd(&sh.vi[1], 1)], j);
          }
        }
      }
      st(&s.C[u], mu);
    }
    __syncthreads();
    head = tail;
    tail = sh.vi[1];
    r++;
    __syncthreads();
  }
  const int P = tail, R = r;
  if (threadIdx.x == 0) st(&s.E[R], P);
  // bucket sizes by M, then bucket starts (exclusive scan over m)
  for (int i = threadIdx.x; i < n; i += ib()) st(&s.F[i], 0);
  __syncthreads();
  for (int f = threadIdx.x; f < P; f += ib()) atomicAdd(&s.F[ld(&s.C[ld(&s.D[f])])], 1);
  __syncthreads();
  int carry = 0;
  for (int base = 0; base < n; base += ib()) {
    int i = base + threadIdx.x;
    int v = i < n ? ld(&s.F[i]) : 0;
    int tot;
    int pre = block_excl_scan<IB_MAX>(v, sh.red, &tot);
    if (i < n) st(&s.F[i], carry + pre);
    carry += tot;
  }
  __syncthreads();
  // removal order, round by round (A = order; the degrees are no longer needed)
  for (int q = 0; q < R; q++) {
    int f0 = ld(&s.E[q]), f1 = ld(&s.E[q + 1]);
    for (int f = f0 + (int)threadIdx.x; f < f1; f += ib()) {
      int u = ld(&s.D[f]);
      st(&s.A[atomicAdd(&s.F[ld(&s.C[u])], 1)], u);
    }
    __syncthreads();
  }
  // smallest vertex that is never removed, then suffix minima of the order (into D)
  int cm = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += ib())
    if (ld(&s.B[i]) < 0) cm = i < cm ? i : cm;
  cm = (int)block_min_u64<IB_MAX>((unsigned long long)(uint32_t)cm, sh.redu);
  int run = cm;
  for (int top = ((P + ib() - 1) / ib()) * ib(); top > 0; top -= ib()) {
    int i = top - ib() + threadIdx.x;
    int v = i < P ? ld(&s.A[i]) : 0x7fffffff;
    int cmin;
    int suf = block_suffix_min(v, run, sh, &cmin);
    if (i < P) st(&s.D[i], suf);
    run = cmin;
  }
  __syncthreads();
  // steps taken: while the current set is larger than s_post and has a vertex of degree 1
  const int steps = P < n - A.s_post ? P : n - A.s_post;
  for (int i = threadIdx.x; i < steps; i += ib()) {
    int ni = n - i;
    wcc_record rc;
    rc.minv = ar.vtx[d.b + ld(&s.D[i])];
    rc.n = ni;
    rc.k = (int)wcc_k_of(A.crit, ni, A.lin_num, A.lin_den);
    rc.lambda = 1;
    rc.ssize = 1;
    rc.reserved = 0;
    rc.shash = vhash(ar.vtx[d.b + ld(&s.A[i])]);
    if (A.rec) {
      unsigned long long q = atomicAdd(&A.cnt[CNT_RECORDS], 1ull);
      if ((long long)q < A.rec_cap) A.rec[q] = rc;
    }
  }
  if (threadIdx.x == 0) {
    atomicAdd(&A.cnt[CNT_MINCUTS], (unsigned long long)steps);
    if (steps > 1) atomicAdd(&A.cnt[CNT_ITEMS], (unsigned long long)(steps - 1));
  }
  __syncthreads();
  if (steps < P || n - P <= A.s_post) return 0;  // the rest has at most s_post vertices
  for (int i = threadIdx.x; i < n; i += ib()) st(&s.B[i], ld(&s.B[i]) < 0 ? cm : -1);
  __syncthreads();
  return n - P;
}

// ---------------------------------------------------------------- k-core peel
// A[i] ends as i's degree inside the surviving core (alive iff A[i] >= k).
// Returns the number of removed vertices.  D and E hold the frontiers.
template <bool LDS, bool CL>
NOINL int item_peel(const St &s_in, int k, Sh &sh_in) {
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  int n = s.n;
  if (threadIdx.x == 0) sh.vi[0] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += ib()) {
    int dg = row_end(s, i) - ld(&s.R[i]);
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
    for (int f = threadIdx.x; f < cnt; f += ib()) {
      int u = ld(&cur[f]);
      int r0 = ld(&s.R[u]), r1 = row_end(s, u);
      for (int e = r0; e < r1; e++) {
        int j = adj_at(s, e);
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
constexpr int32_t SCANNED = -(1 << 30);  // key of a scanned super-vertex (stays negative)

// Effect of one list entry x -> y whose increment left y's key at nw > 0.
template <bool GL>
DEV void scan_entry(const St &s, int x, int y, int nw, int e, int bound, int *bl, int *by) {
  int lv = nw < bound ? nw : bound;
  if (nw <= bound) bit_set<GL>(s, nw, y);
  if (nw == bound) st(&s.B[y], x);          // contractible, first for y: parent
  else if (nw > bound) mark_set(s, e);      // contractible, extra edge
  if (lv > *bl || (lv == *bl && y < *by)) {
    *bl = lv;
    *by = y;
  }
}

// One round's maximum-adjacency scan, run by wave 0.  Lists: owner x's entries are
// [st[x], st[x]+len[x]) of `list` (LDS u16 when L16).  The contractible entries form a
// forest plus extra edges: when a key first reaches the bound, the scanned vertex becomes
// the parent (B) of the unscanned one; later contractible entries are marked in s.mark.
// Lists of later rounds were written by this workgroup before a barrier, so plain loads
// see them.  Returns the number of steps (< 0 on an inconsistency).
//
// The next vertex usually follows from the step itself, without reading the bitmaps:
// x was the smallest member of the highest non-empty level jx.  If this step raised some
// keys above jx, the new top level holds exactly those vertices, and the next vertex is
// the smallest of them.  Otherwise the top level stays jx and the next vertex is the
// smaller of x's successor in its own bitmap word and the vertices raised to jx now;
// when that successor does not exist, the bitmaps are searched from level jx down
// (every level above jx is empty then).
//
// x's key equals jx (capped at the bound): x lies in level jx, and level jx + 1 is
// empty.  The successor's list start, length and first 64 entries are loaded while the
// current step runs, so a step that continues with the successor issues its first key
// increments at once; only the bitmap word of x is read before them.
// Index of entry i of a list [e0, e0 + cnt), clamped into the list (entry 0 of all lists
// when it is empty), so that list loads need no per-lane branch: lanes past the end load
// a valid entry and ignore it.  (During a scan every list array holds at least one entry.)
DEV int clamp_idx(int e0, int i, int cnt) { return cnt > 0 ? e0 + (i < cnt ? i : cnt - 1) : 0; }

template <bool L16, bool GL>
DEV int scan_round(const St &s, const int32_t *stv, const int32_t *lenv, const int32_t *list,
                   const uint16_t *list16, int bound) {
  const int lane = threadIdx.x;
  auto entry = [&](int e) -> int {
    if constexpr (L16) return (int)list16[e];
    else return list[e];
  };
  // uniform state in scalar registers; this lane's bitmap level offset for clearing
  const int n = __builtin_amdgcn_readfirstlane(s.n);
  const unsigned ls = (unsigned)__builtin_amdgcn_readfirstlane(s.ls);
  bound = __builtin_amdgcn_readfirstlane(bound);
  // (lane's own level; used only for levels up to the bound)
  const unsigned my_lv = __umul24((unsigned)lane, ls);
  int steps = 0;
  int x = -1, jx = 0;      // next vertex when already known, and its level
  bool have = false;       // x's list (start e0, length cnt, first 64 entries y) is loaded
  int e0 = 0, cnt = 0, y = -1;
  for (;;) {
    if (x < 0) {
      x = __builtin_amdgcn_readfirstlane(bit_pick<GL>(s, &jx));
      jx = __builtin_amdgcn_readfirstlane(jx);
      if (x == -2) return -1;
      if (x < 0) break;
      have = false;
    }
    if (steps >= n) return -1;  // guard: a scan takes at most n steps
    steps++;
    const int xw = x >> 6;
    const uint64_t xbit = 1ull << (x & 63);
    uint64_t w0 = ld(&s.bits[__umul24((unsigned)jx, ls) + xw]);
    // GL: the first L0 word after x's that may hold a member of level jx (from the LDS
    // summary; a clear summary bit means an empty word) is loaded with x's word: when x's
    // word holds no other member, the first member there is the successor
    int wnx = -1;
    uint64_t wn = 0;
    if constexpr (GL) {
      if (s.l1) {
        const uint64_t *L1 = lvl1<GL>(s, jx);
        const int i1 = xw >> 6;
        uint64_t m1 = (L1[i1] & (~0ull << (xw & 63))) & ~(1ull << (xw & 63));
        if (m1) {
          wnx = i1 * 64 + __ffsll((long long)m1) - 1;
        } else {
          for (int c0 = i1 + 1; c0 < s.nw1; c0 += 64) {
            uint64_t w1 = c0 + lane < s.nw1 ? L1[c0 + lane] : 0ull;
            uint64_t b = __ballot(w1 != 0);
            if (b) {
              int l = __ffsll((long long)b) - 1;
              wnx = (c0 + l) * 64 + __ffsll((long long)readlane64(w1, l)) - 1;
              break;
            }
          }
        }
        wnx = __builtin_amdgcn_readfirstlane(wnx);
        if (wnx >= 0 && wnx < s.nw0) wn = ld(&s.bits[__umul24((unsigned)jx, ls) + wnx]);
      }
    }
    if (!have) {
      e0 = ldr(&stv[x]);
      cnt = ldr(&lenv[x]);
      y = entry(clamp_idx(e0, lane, cnt));
    }
    // x's bitmap words and list entries are complete before the increments are issued (an
    // empty asm statement that reads them): the compiler then has no earlier load to wait
    // for until the increments' results are needed, and the successor's loads below are
    // issued while the increments are in flight
    asm volatile("" ::"v"(w0), "v"(wn), "v"(y));
    // first 64 increments; their results are used only after the successor's loads
    // below have been issued
    int old = -1;
    if (lane < cnt) old = atomicAdd(&s.A[y], 1);
    // y is complete here; re-defining it in an empty asm statement keeps the compiler from
    // waiting again where y is used below, which would also wait for the prefetch issued
    // in between
    asm volatile("" : "+v"(y));
    uint64_t rest = w0 & ~xbit;
    int cand = rest ? (x & ~63) + __ffsll((long long)rest) - 1
                    : wn ? wnx * 64 + __ffsll((long long)wn) - 1 : -1;
    int ce0 = 0, ccnt = 0;
    if (cand >= 0) {
      ce0 = ldr(&stv[cand]);
      ccnt = ldr(&lenv[cand]);
    }
    // x leaves levels 0..jx (lane l clears level l, and l + 64, ... above 63; one of them
    // marks it scanned)
    if (lane <= jx) {
      atomicAnd((unsigned long long *)&s.bits[my_lv + xw], ~xbit);
      st(&s.A[x], SCANNED);
    }
    for (int lb = 64; lb <= jx; lb += 64)
      if (lb + lane <= jx) atomicAnd((unsigned long long *)&s.bits[__umul24((unsigned)(lb + lane), ls) + xw], ~xbit);
    // longer lists: the next 256 entries are loaded before the prefetch below, so that
    // waiting for them does not wait for it
    int yv[4];
    if (cnt > 64) {
#pragma unroll
      for (int k = 0; k < 4; k++) yv[k] = entry(clamp_idx(e0, 64 + 64 * k + lane, cnt));
    }
    int cy = entry(clamp_idx(ce0, lane, ccnt));
    int bl = -1, by = 0;  // this lane's highest raised level and smallest id there
    if (old >= 0) {
      int nw = old + 1;
      if (nw <= bound) bit_set<GL>(s, nw, y);
      if (nw == bound) st(&s.B[y], x);          // contractible, first for y: parent
      else if (nw > bound) mark_set(s, e0 + lane);  // contractible, extra edge
      bl = nw < bound ? nw : bound;
      by = y;
    }
    if (cnt > 64) {
      // four chunks at a time: loads, then the increments, then their effects
      for (int base = 64; base < cnt; base += 256) {
        if (base > 64) {
#pragma unroll
          for (int k = 0; k < 4; k++) yv[k] = entry(clamp_idx(e0, base + 64 * k + lane, cnt));
        }
        int ov[4];
#pragma unroll
        for (int k = 0; k < 4; k++) ov[k] = base + 64 * k + lane < cnt ? atomicAdd(&s.A[yv[k]], 1) : -1;
#pragma unroll
        for (int k = 0; k < 4; k++)
          if (ov[k] >= 0) scan_entry<GL>(s, x, yv[k], ov[k] + 1, e0 + base + 64 * k + lane, bound, &bl, &by);
      }
    }
    // only keys raised to jx or above can decide the next vertex; when there are any, one
    // reduction of (level + 1, 2^24 - 1 - id) packed finds the highest raised level and,
    // inside it, the smallest id (items have fewer than 2^24 vertices; bounds above 126
    // do not fit the packed level and take two reductions)
    int nx = cand;
    if (__ballot(bl >= jx)) {
      int M, pid;
      if (bound < 127) {
        int P = wave_max_i(bl >= jx ? ((bl + 1) << 24) | (0xFFFFFF - by) : 0);
        M = (P >> 24) - 1;
        pid = 0xFFFFFF - (P & 0xFFFFFF);
      } else {
        M = wave_max_i(bl >= jx ? bl : -1);
        pid = wave_min_i(bl == M ? by : 0x7fffffff);
      }
      if (M > jx) {
        nx = pid;
        jx = M;
      } else if (cand >= 0 && pid < cand) {
        nx = pid;
      }
    }
    have = nx >= 0 && nx == cand;
    e0 = ce0;
    cnt = ccnt;
    y = cy;
    x = __builtin_amdgcn_readfirstlane(nx);
    jx = __builtin_amdgcn_readfirstlane(jx);
  }
  return steps;
}

// Certificate of lambda >= t: t edge-disjoint spanning trees (every cut crosses each of
// them).  Built greedily, one spanning forest per pass over the edges not used by earlier
// forests; an edge belongs to a forest when its union-find link joined two trees, so a
// forest spans the item exactly when n - 1 links succeeded.  Each pass first links every
// vertex with up to two sampled unused larger neighbours and flattens the trees, after
// which most edges join one tree and stop at a single comparison.  Uses B (union-find) and the
// entry marks (used edges); returns false as soon as a forest does not span (the greedy
// choice can fail even when lambda >= t: the caller then runs the scans).
// SUB: the certificate of the subgraph induced by the vertices x with C[x] < 0 (na of
// them); edges with an endpoint outside are left out.
template <bool LDS, bool CL, bool SUB = false>
NOINL bool forest_certificate(const St &s_in, int t, int na, Sh &sh_in) {
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  const int n = s.n;
  auto in = [&](int x) { return !SUB || ld(&s.C[x]) < 0; };
  unsigned long long q = s.pf ? wall_clock64() : 0;
  mark_clear(s, s.m);
  for (int f = 0; f < t; f++) {
    for (int x = threadIdx.x; x < n; x += ib()) st(&s.B[x], x);
    __syncthreads();
    int links = 0;
    for (int x = threadIdx.x; x < n; x += ib()) {
      if (!in(x)) continue;
      // two entries of x's row, at a different place for every forest
      int r0 = ldr(&s.R[x]), dg = row_end(s, x) - r0;
      int e1 = r0 + (2 * f) % dg, e2 = r0 + (2 * f + 1) % dg;
      int y1 = adj_at(s, e1), y2 = adj_at(s, e2);
      if (y1 > x && in(y1) && !mark_get(s, e1) && uf_link(s.B, x, y1)) {
        mark_set(s, e1);
        links++;
      }
      if (e2 != e1 && y2 > x && in(y2) && !mark_get(s, e2) && uf_link(s.B, x, y2)) {
        mark_set(s, e2);
        links++;
      }
    }
    __syncthreads();
    sub_mark(s, 19, &q);
    for (int x = threadIdx.x; x < n; x += ib()) st(&s.B[x], uf_find(s.B, x));
    __syncthreads();
    sub_mark(s, 20, &q);
    for_entries(s, sh, s.R, n, s.m, [&](int e) { return adj_at(s, e); }, [&](int x, int e, int y) {
      if (y > x && ld(&s.B[x]) != ld(&s.B[y]) && in(x) && in(y) && !mark_get(s, e) &&
          uf_link(s.B, x, y)) {
        mark_set(s, e);
        links++;
      }
    });
    links = block_sum<IB_MAX>(links, sh.red);  // includes barriers
    sub_mark(s, 21, &q);
    if (links < na - 1) return false;
  }
  return true;
}

// The same certificate for t <= TMAX <= 4 with all forests built in one pass: forest f
// keeps its union-find in B, A, D or E (free before the rounds, and in LDS for an
// LDS-state item), every vertex first links up to two sampled edges
// per forest, and then every unused edge joins the first forest whose trees it connects.
// One pass over the edges instead of t, but no early stop when a forest cannot span.
template <int TMAX, bool LDS, bool CL, bool SUB = false>
NOINL bool forest_certificate_one(const St &s_in, int t, int na, Sh &sh_in) {
  static_assert(TMAX >= 1 && TMAX <= 4, "forests 0..3 keep their union-finds in B, A, D, E");
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  const int n = s.n;
  auto P = [&](int f) -> int32_t * {
    return f == 0 ? s.B : f == 1 ? s.A : f == 2 ? s.D : s.E;
  };
  auto in = [&](int x) { return !SUB || ld(&s.C[x]) < 0; };  // (as for forest_certificate)
  unsigned long long q = s.pf ? wall_clock64() : 0;
  mark_clear(s, s.m);
  for (int x = threadIdx.x; x < n; x += ib()) {
#pragma unroll
    for (int f = 0; f < TMAX; f++)
      if (f < t) st(&P(f)[x], x);
  }
  __syncthreads();
  int links[TMAX];
#pragma unroll
  for (int f = 0; f < TMAX; f++) links[f] = 0;
  for (int x = threadIdx.x; x < n; x += ib()) {
    if (!in(x)) continue;
    int r0 = ldr(&s.R[x]), dg = row_end(s, x) - r0;
#pragma unroll
    for (int f = 0; f < TMAX; f++) {
      if (f >= t) continue;
      // two entries of x's row, at a different place for every forest
      int e1 = r0 + (2 * f) % dg, e2 = r0 + (2 * f + 1) % dg;
      int y1 = adj_at(s, e1), y2 = adj_at(s, e2);
      if (y1 > x && in(y1) && !mark_get(s, e1) && uf_link(P(f), x, y1)) {
        mark_set(s, e1);
        links[f]++;
      }
      if (e2 != e1 && y2 > x && in(y2) && !mark_get(s, e2) && uf_link(P(f), x, y2)) {
        mark_set(s, e2);
        links[f]++;
      }
    }
  }
  __syncthreads();
  sub_mark(s, 19, &q);
  for (int x = threadIdx.x; x < n; x += ib()) {
#pragma unroll
    for (int f = 0; f < TMAX; f++)
      if (f < t) st(&P(f)[x], uf_find(P(f), x));
  }
  __syncthreads();
  sub_mark(s, 20, &q);
  for_entries(s, sh, s.R, n, s.m, [&](int e) { return adj_at(s, e); }, [&](int x, int e, int y) {
    if (y <= x || mark_get(s, e) || !in(x) || !in(y)) return;
    // (no early exit from the unrolled loop: constant indices keep links[] in registers)
    bool done = false;
#pragma unroll
    for (int f = 0; f < TMAX; f++) {
      if (!done && f < t) {
        int32_t *Pf = P(f);
        if (ld(&Pf[x]) != ld(&Pf[y]) && uf_link(Pf, x, y)) {
          links[f]++;
          done = true;
        }
      }
    }
  });
  bool ok = true;
#pragma unroll
  for (int f = 0; f < TMAX; f++) {
    int l = block_sum<IB_MAX>(links[f], sh.red);  // includes barriers
    if (f < t && l < na - 1) ok = false;
  }
  sub_mark(s, 21, &q);
  return ok;
}

// bounds up to TONE: all forests of the certificate in one pass
constexpr int TONE = 4;

// A second packing of t <= 4 edge-disjoint spanning forests, for sets on which the sampled
// greedy fails: there, vertices of low degree, which need one edge in every forest, lose
// edges to forests that did not need them.  Here every edge is placed by its endpoint with
// the shorter row (ties: the smaller id), rows of at most 2t entries first, and each row's
// edges go to the forests in turn (the next edge starts after the forest the last one
// joined).  Each edge is handled by one thread only, and every link joins two trees of its
// forest, so the forests are edge-disjoint and acyclic whatever the interleaving.  SUB as
// for forest_certificate.  Union-finds in B, A, D, E.
template <bool LDS, bool CL, bool SUB>
NOINL bool forest_certificate_rot(const St &s_in, int t, int na, Sh &sh_in) {
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  const int n = s.n;
  auto P = [&](int f) -> int32_t * {
    return f == 0 ? s.B : f == 1 ? s.A : f == 2 ? s.D : s.E;
  };
  auto in = [&](int x) { return !SUB || ld(&s.C[x]) < 0; };
  for (int x = threadIdx.x; x < n; x += ib())
    for (int f = 0; f < t; f++) st(&P(f)[x], x);
  __syncthreads();
  int l0 = 0, l1 = 0, l2 = 0, l3 = 0;
  for (int phase = 0; phase < 2; phase++) {
    for (int x = threadIdx.x; x < n; x += ib()) {
      if (!in(x)) continue;
      const int r0 = ldr(&s.R[x]), r1 = row_end(s, x), lx = r1 - r0;
      if ((lx <= 2 * t) != (phase == 0)) continue;
      int f0 = 0;
      for (int e = r0; e < r1; e++) {
        const int y = adj_at(s, e);
        if (y == x || !in(y)) continue;
        const int ly = row_end(s, y) - ldr(&s.R[y]);
        if (ly < lx || (ly == lx && y < x)) continue;  // y places this edge
        for (int j = 0; j < t; j++) {
          const int f = f0 + j < t ? f0 + j : f0 + j - t;
          if (uf_link(P(f), x, y)) {
            l0 += f == 0;
            l1 += f == 1;
            l2 += f == 2;
            l3 += f == 3;
            f0 = f + 1 < t ? f + 1 : 0;
            break;
          }
        }
      }
    }
    __syncthreads();
  }
  bool ok = true;
  int l = block_sum<IB_MAX>(l0, sh.red);  // (each includes barriers)
  ok = ok && l >= na - 1;
  l = block_sum<IB_MAX>(l1, sh.red);
  ok = ok && (t < 2 || l >= na - 1);
  l = block_sum<IB_MAX>(l2, sh.red);
  ok = ok && (t < 3 || l >= na - 1);
  l = block_sum<IB_MAX>(l3, sh.red);
  ok = ok && (t < 4 || l >= na - 1);
  return ok;
}

// ---------------------------------------------------------------- PAPER-mode low-degree runs
// An item H (connected, minimum degree delta >= 2, delta < k(|H|)) whose cut value equals
// its minimum degree has canonical cut (delta, {smallest vertex of degree delta}): Phase 0
// sets it and the rounds replace it only by a strictly smaller cut.  The part of size 1 is
// dropped and the rest is the next item.  So while that equality holds, WCC as printed
// removes, one item at a time, the smallest vertex of minimum degree.  This computes such
// a sequence at once and proves the equality for every step:
//   * the run: v_1, v_2, ... with H_0 = H, H_t = H_{t-1} - v_t, v_t the smallest vertex of
//     minimum degree d_t in H_{t-1}; it goes on while d_t < k(|H_{t-1}|), |H_{t-1}| >
//     s_post and d_1 <= d_2 <= ... (a removal that would leave a degree below d_t ends
//     the run before it);
//   * adding back a vertex of degree d to a graph of edge connectivity c gives connectivity
//     at least min(c, d).  Hence lambda(H_{t-1}) >= min(lambda(H_P), d_t, ..., d_P) =
//     d_t for a non-decreasing run of P steps with lambda(H_P) >= d_P, and lambda <= the
//     minimum degree gives equality;
//   * lambda(H_P) >= d_P is certified by d_P edge-disjoint spanning forests of H_P.  If
//     they are not found, the item is cut as usual (the run was only a proposal).
// Ears (degree 2, when k(s_post + 1) >= 2): a removal of v at degree 2 that leaves
// neighbours of degree 1 is kept when those neighbours start paths of degree-2 vertices
// (x_1, x_2, ... up to an end z of degree >= 3) whose ends keep degree >= 2 afterwards.
// The one-at-a-time process then peels both paths right after v, smallest leaf first
// (each a split of cut 1), and stops at the ends; the set before v is the set after the
// paths plus an ear, whose edge connectivity is at least min(its connectivity, 2).  With
// lambda >= 2 at the step after the paths (the same argument from the end of the run,
// where d_max forests certify lambda(H_P) >= d_max, the largest class degree), v's step
// has lambda = 2 and the leaf steps lambda = 1.  A path that returns to v (the set is a
// cycle), an end that would fall below degree 2, or a path that would leave s_post or
// fewer vertices ends the run before v.
// The run is sequential (wave 0).  Degree classes are taken in increasing order: the block
// lists the class's vertices in id order, and vertices whose degree falls into the class
// during it wait in sh.arr (up to 64; when full, the class list is rebuilt).  Path
// vertices removed with an ear leave both (list entries are skipped, the waiting list is
// compacted).
// Arrays: A degrees, C removal step (-1 = still in H), D the class list, then the suffix
// minima of the order, E the removal order, F the degrees d_t (1 for path vertices); B
// ends as the child's labels.
// Returns the number of vertices left when the rest goes on (B[i] = its smallest vertex for
// members, -1 otherwise), 0 when nothing goes on, -1 when no certified run exists.
template <bool LDS, bool CL>
NOINL int item_low_run(const ItemArgs &A, const St &s_in, const ItemDesc &d, int dmin, Sh &sh_in) {
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  Arena ar = A.ar[d.depth & 1];
  ar.vtx = as_glb(ar.vtx);
  const int n = s.n;
  auto kof = [&](int sz) { return (int)wcc_k_of(A.crit, sz, A.lin_num, A.lin_den); };
  for (int i = threadIdx.x; i < n; i += ib()) {
    st(&s.A[i], row_end(s, i) - ldr(&s.R[i]));
    st(&s.C[i], -1);
  }
  int P = 0, dc = dmin, dmax = 0;
  long long edges = s.m / 2;  // edges of the current set
  for (;;) {
    const int size = n - P;
    if (size <= A.s_post || dc >= kof(size)) break;
    // the class list: vertices of the current set with degree dc, in id order
    int carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += ib()) {
      int i = base + threadIdx.x;
      bool f = i < n && ld(&s.C[i]) < 0 && ld(&s.A[i]) == dc;
      int tot;
      int pre = block_excl_scan<IB_MAX>((int)f, sh.red, &tot);
      if (f) st(&s.D[carry + pre], i);
      carry += tot;
    }
    const int len = carry;
    __syncthreads();
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      int cur = 0, na = 0, status = 0;  // 0 class done, 1 list rebuilt, 2 run ends
      int p = P, rem = 0;                // steps so far, edges removed in this pass
      // the first neighbour of x still in the set other than `skip` (-1: none skipped)
      auto next_in_set = [&](int x, int skip) -> int {
        const int r0 = ldr(&s.R[x]), r1 = row_end(s, x);
        for (int b = r0; b < r1; b += 64) {
          int e = b + lane;
          int w = e < r1 ? adj_at(s, e) : -1;
          bool f = w >= 0 && w != skip && ld(&s.C[w]) < 0;
          uint64_t bm = __ballot(f);
          if (bm) return __shfl(w, (int)__builtin_ctzll(bm), 64);
        }
        return -1;
      };
      for (;;) {
        const int sz = n - p;
        if (sz <= A.s_post || dc >= kof(sz)) {
          status = 2;
          break;
        }
        // the first list entry still in the set (path vertices of ears leave it early)
        int head = 0x7fffffff;
        while (cur < len) {
          int h = ld(&s.D[cur]);
          if (ld(&s.C[h]) < 0) {
            head = h;
            break;
          }
          cur++;
        }
        int av = lane < na ? sh.arr[lane] : 0x7fffffff;
        int amin = wave_min_i(av);
        int v = head < amin ? head : amin;
        if (v == 0x7fffffff) break;  // the class is empty
        // the neighbours still in the set lose one: below dc ends the run, dc joins the class
        const int e0 = ldr(&s.R[v]), e1 = row_end(s, v);
        int drop = 0, join = 0;
        for (int b = e0; b < e1; b += 64) {
          int e = b + lane;
          if (e < e1) {
            int w = adj_at(s, e);
            if (ld(&s.C[w]) < 0) {
              int dw = ld(&s.A[w]) - 1;
              drop += dw < dc;
              join += dw == dc;
            }
          }
        }
        const bool from_arr = v != head;
        if (wave_sum(drop)) {
          // an ear: v of degree 2 and the paths of degree-2 vertices that start at its
          // neighbours, checked in full before anything is removed
          if (!A.leaf_batch || dc != 2) {
            status = 2;
            break;
          }
          // (a walk that finds no next vertex or outgrows the item, possible only on
          // input with repeated entries, ends the run)
          const int nb0 = next_in_set(v, -1), nb1 = nb0 < 0 ? -1 : next_in_set(v, nb0);
          int z0 = v, z1 = v, L0 = 0, L1 = 0;
          for (int sd = 0; sd < 2 && nb1 >= 0; sd++) {
            int prev = v, x = sd ? nb1 : nb0, l = 0;
            while (x != v && ld(&s.A[x]) == 2) {
              int nx = next_in_set(x, prev);
              if (nx < 0 || l >= n) {
                x = v;
                break;
              }
              prev = x;
              x = nx;
              l++;
            }
            if (sd) {
              z1 = x;
              L1 = l;
            } else {
              z0 = x;
              L0 = l;
            }
            if (x == v) break;  // the set is a cycle
          }
          bool ok = z0 != v && z1 != v && sz - 1 - L0 - L1 > A.s_post;
          int zj = 0;  // ends that fall to degree 2 (they join the class)
          if (ok) {
            const int a0 = ld(&s.A[z0]), a1 = ld(&s.A[z1]);
            if (z0 == z1) {
              ok = a0 >= 4;
              zj = a0 == 4;
            } else {
              zj = (a0 == 3) + (a1 == 3);
            }
          }
          if (!ok) {
            status = 2;
            break;
          }
          if (na - (int)from_arr + zj > 64) {
            status = 1;
            break;
          }
          if (from_arr) {  // the last waiting vertex takes v's slot
            int slot = wave_min_i(av == v ? lane : 64);
            int last = __shfl(av, na - 1, 64);
            if (lane == slot) sh.arr[slot] = last;
            na--;
          } else {
            cur++;
          }
          if (lane == 0) {
            st(&s.C[v], p);
            st(&s.F[p], 2);
            st(&s.A[nb0], ld(&s.A[nb0]) - 1);
            st(&s.A[nb1], ld(&s.A[nb1]) - 1);
          }
          p++;
          rem += 2;
          __threadfence_block();
          // both paths, smallest leaf first; each path vertex has one neighbour left
          int h0 = L0 ? nb0 : 0x7fffffff, h1 = L1 ? nb1 : 0x7fffffff;
          while (h0 != 0x7fffffff || h1 != 0x7fffffff) {
            const bool first = h0 < h1;
            const int u = first ? h0 : h1;
            const int nx = next_in_set(u, -1);
            if (lane == 0) {
              st(&s.C[u], p);
              st(&s.F[p], 1);
              if (nx >= 0) st(&s.A[nx], ld(&s.A[nx]) - 1);
            }
            p++;
            rem += 1;
            __threadfence_block();
            if (first) h0 = --L0 > 0 && nx >= 0 ? nx : 0x7fffffff;
            else h1 = --L1 > 0 && nx >= 0 ? nx : 0x7fffffff;
          }
          // path vertices leave the waiting list; ends that fell to degree 2 join it
          {
            int w = lane < na ? sh.arr[lane] : -1;
            bool keep = w >= 0 && ld(&s.C[w]) < 0;
            uint64_t km = __ballot(keep);
            if (keep) sh.arr[__popcll(km & lanemask_lt())] = w;
            na = __popcll(km);
          }
          if (ld(&s.A[z0]) == 2) {
            if (lane == 0) sh.arr[na] = z0;
            na++;
          }
          if (z1 != z0 && ld(&s.A[z1]) == 2) {
            if (lane == 0) sh.arr[na] = z1;
            na++;
          }
          __threadfence_block();
          continue;
        }
        if (na - (int)from_arr + wave_sum(join) > 64) {
          status = 1;
          break;
        }
        if (from_arr) {  // the last waiting vertex takes v's slot
          int slot = wave_min_i(av == v ? lane : 64);
          int last = __shfl(av, na - 1, 64);
          if (lane == slot) sh.arr[slot] = last;
          na--;
        } else {
          cur++;
        }
        for (int b = e0; b < e1; b += 64) {
          int e = b + lane;
          bool j = false;
          int w = 0;
          if (e < e1) {
            w = adj_at(s, e);
            if (ld(&s.C[w]) < 0) {
              int dw = ld(&s.A[w]) - 1;
              st(&s.A[w], dw);
              j = dw == dc;
            }
          }
          uint64_t bm = __ballot(j);
          if (j) sh.arr[na + __popcll(bm & lanemask_lt())] = w;
          na += __popcll(bm);
        }
        if (lane == 0) {
          st(&s.C[v], p);
          st(&s.F[p], dc);
        }
        p++;
        rem += dc;
        // (this wave reads these words again in the next step)
        __threadfence_block();
      }
      if (lane == 0) {
        sh.vi[0] = p;
        sh.vi[1] = status;
        sh.vi[2] = rem;
      }
    }
    __syncthreads();
    const int p1 = sh.vi[0], status = sh.vi[1];
    edges -= sh.vi[2];
    if (p1 > P) dmax = dc;
    P = p1;
    if (status == 2) break;
    if (status == 0) dc++;
  }
  __syncthreads();
  if (P == 0) return -1;
  // lambda(H_P) >= d_max: d_max edge-disjoint spanning forests of the vertices left
  const int na = n - P, dP = dmax;
  bool ok = na <= 1;
  if (!ok && edges >= (long long)dP * (na - 1)) {
    ok = dP <= TONE ? forest_certificate_one<TONE, LDS, CL, true>(s_in, dP, na, sh)
                    : forest_certificate<LDS, CL, true>(s_in, dP, na, sh);
    if (!ok && dP <= TONE) ok = forest_certificate_rot<LDS, CL, true>(s_in, dP, na, sh);
  }
  __syncthreads();
  if (!ok) return -1;
  // the removal order (E), then the smallest vertex never removed and the suffix minima
  int cm = 0x7fffffff;
  for (int i = threadIdx.x; i < n; i += ib()) {
    int c = ld(&s.C[i]);
    if (c >= 0) st(&s.E[c], i);
    else cm = i < cm ? i : cm;
  }
  cm = (int)block_min_u64<IB_MAX>((unsigned long long)(uint32_t)cm, sh.redu);
  int run = cm;
  for (int top = ((P + ib() - 1) / ib()) * ib(); top > 0; top -= ib()) {
    int i = top - ib() + threadIdx.x;
    int v = i < P ? ld(&s.E[i]) : 0x7fffffff;
    int cmin;
    int suf = block_suffix_min(v, run, sh, &cmin);
    if (i < P) st(&s.D[i], suf);
    run = cmin;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < P; i += ib()) {
    int ni = n - i;
    wcc_record rc;
    rc.minv = ar.vtx[d.b + ld(&s.D[i])];
    rc.n = ni;
    rc.k = kof(ni);
    rc.lambda = ld(&s.F[i]);
    rc.ssize = 1;
    rc.reserved = 0;
    rc.shash = vhash(ar.vtx[d.b + ld(&s.E[i])]);
    if (A.rec) {
      unsigned long long q = atomicAdd(&A.cnt[CNT_RECORDS], 1ull);
      if ((long long)q < A.rec_cap) A.rec[q] = rc;
    }
  }
  if (threadIdx.x == 0) {
    atomicAdd(&A.cnt[CNT_MINCUTS], (unsigned long long)P);
    if (P > 1) atomicAdd(&A.cnt[CNT_ITEMS], (unsigned long long)(P - 1));
  }
  __syncthreads();
  if (na <= A.s_post) return 0;
  for (int i = threadIdx.x; i < n; i += ib()) st(&s.B[i], ld(&s.C[i]) < 0 ? cm : -1);
  __syncthreads();
  return na;
}

// Returns the capped cut value; F[i] = 1 for i in S.  steps/rounds are accumulated.
template <bool LDS, bool CL>
NOINL int item_mincut(const ItemArgs &A, const St &s_in, const ItemDesc &d, int cap, Sh &sh_in,
                    long long *steps_out, long long *rounds_out) {
  Sh &sh = *as_lds(&sh_in);  // (the workgroup's shared scratch, in LDS)
  const St s = typed_st<LDS, CL>(s_in);  // (a typed local copy: its fields stay in registers)
  int n = s.n;
  unsigned long long pt = s.pf ? wall_clock64() : 0;
  // Phase 0: minimum degree and its smallest vertex
  unsigned long long mv = ~0ull;
  for (int i = threadIdx.x; i < n; i += ib()) {
    unsigned long long dg = (unsigned long long)(uint32_t)(row_end(s, i) - ldr(&s.R[i]));
    unsigned long long v = (dg << 32) | (uint32_t)i;
    mv = v < mv ? v : mv;
  }
  mv = block_min_u64<IB_MAX>(mv, sh.redu);
  int delta = (int)(mv >> 32), dv = (int)(mv & 0xffffffffu);
  int bound = delta < cap ? delta : cap;
  int s_kind = delta <= cap ? 1 : 0;  // 0 empty, 1 singleton dv, 2 set in F
  long long steps = 0, rounds = 0;
  // lambda >= bound: no super-vertex degree can fall below the bound, so the rounds would
  // end with (bound, the Phase-0 set); a certificate of it gives the same result at once
  // (bound spanning trees need bound * (n - 1) edges: sparser items skip the attempt)
  // (one pass for bounds up to 4; above, one pass per forest, which stops at the first
  // forest that does not span: for items split by a small cut that is cheaper than
  // checking every forest per edge, most of all when the union-finds are in global memory)
  if (bound > 1 && (long long)s.m / 2 >= (long long)bound * (n - 1) &&
      (bound <= TONE ? forest_certificate_one<TONE, LDS, CL>(s_in, bound, n, sh)
                      : forest_certificate<LDS, CL>(s_in, bound, n, sh))) {
    if (s.pf && threadIdx.x == 0) atomicAdd(&A.cnt[CNT_PH + 11], 1ull);
    bound = -bound;  // (certified; restored below)
  }
  ph_mark(A, s, 3, &pt);
  if (bound > 1) {
    // super-vertex ids C; round 1 scans the item's own rows (starts R, lengths D)
    for (int i = threadIdx.x; i < n; i += ib()) {
      st(&s.C[i], i);
      st(&s.D[i], row_end(s, i) - ldr(&s.R[i]));
    }
    bool first = true;
    int total = s.m;  // entries in the current lists
    for (;;) {
      ph_mark(A, s, 3, &pt);
      // ---- round setup: keys, marks, bitmaps (levels 0..bound)
      int words = (bound + 1) * s.ls;
      for (int w = threadIdx.x; w < words; w += ib()) st(&s.bits[w], (uint64_t)0);
      if (s.bits1)
        for (int w = threadIdx.x; w < (bound + 1) * s.nw1; w += ib()) s.bits1[w] = 0;
      for (int x = threadIdx.x; x < n; x += ib()) {
        st(&s.A[x], 0);
        st(&s.B[x], x);
      }
      mark_clear(s, total);
      __syncthreads();
      for (int x = threadIdx.x; x < n; x += ib())
        if (ldr(&s.C[x]) == x) bit_set<!LDS>(s, 0, x);
      __syncthreads();
      // ---- maximum-adjacency scan, run by wave 0 alone (no block barrier per step)
      const int32_t *stv = first ? s.R : s.E;
      if (threadIdx.x < 64) {
        int r = !first    ? scan_round<false, !LDS>(s, stv, s.D, s.lists, nullptr, bound)
                : s.adj16 ? scan_round<true, !LDS>(s, stv, s.D, nullptr, s.adj16, bound)
                          : scan_round<false, !LDS>(s, stv, s.D, s.adjg, nullptr, bound);
        if (s.pf && threadIdx.x == 0) {
          atomicAdd(&A.cnt[CNT_PH + 10], (unsigned long long)(r > 0 ? r : 0));
          atomicAdd(&A.cnt[CNT_PH + 12], 1ull);
        }
        if (threadIdx.x == 0) sh.vi[3] = r;
      }
      __syncthreads();
      if (sh.vi[3] < 0) {
        if (threadIdx.x == 0) err(A, WCC_EHIP);
        bound = 1;
        s_kind = 0;
        break;
      }
      steps += sh.vi[3];
      ph_mark(A, s, 4, &pt);
      rounds++;
      unsigned long long q = s.pf ? wall_clock64() : 0;
      // ---- contraction: parent forest, then unions of the extra marked entries; the new
      // id of a merged group is its smallest member (A serves as the group minimum)
      for (int x = threadIdx.x; x < n; x += ib())
        if (ld(&s.C[x]) == x) {
          st(&s.B[x], uf_find(s.B, x));
          st(&s.A[x], 0x7fffffff);
        }
      __syncthreads();
      sub_mark(s, 22, &q);
      // (B holds tree roots here, so most marked entries join one tree and stop at the check)
      auto join = [&](int x, int, int y) {
        if (ld(&s.B[x]) != ld(&s.B[y])) uf_unite(s.B, x, y);
      };
      if (first)
        for_marked_entries(s, sh, stv, n, total, [&](int e) { return adj_at(s, e); }, join);
      else
        for_marked_entries(s, sh, stv, n, total, [&](int e) { return ldr(&s.lists[e]); }, join);
      __syncthreads();
      sub_mark(s, 23, &q);
      for (int x = threadIdx.x; x < n; x += ib())
        if (ld(&s.C[x]) == x) {
          int r = uf_find(s.B, x);
          st(&s.B[x], r);
          atomicMin(&s.A[r], x);
        }
      __syncthreads();
      sub_mark(s, 24, &q);
      int reps = 0;
      for (int v = threadIdx.x; v < n; v += ib()) {
        int c = ldr(&s.A[ldr(&s.B[ldr(&s.C[v])])]);
        st(&s.C[v], c);
        reps += (c == v);
      }
      reps = block_sum<IB_MAX>(reps, sh.red);
      sub_mark(s, 25, &q);
      ph_mark(A, s, 5, &pt);
      if (reps <= 1) break;
      first = false;
      // ---- crossing lists of the contracted graph (D = weighted degree, E = start)
      // (the contraction marks are dead now: they flag the crossing entries instead)
      for (int x = threadIdx.x; x < n; x += ib()) st(&s.D[x], 0);
      mark_clear(s, s.m);
      __syncthreads();
      for_entries(s, sh, s.R, n, s.m, [&](int e) { return adj_at(s, e); }, [&](int v, int e, int u) {
        int a = ldr(&s.C[v]);
        if (ldr(&s.C[u]) != a) {
          atomicAdd(&s.D[a], 1);
          mark_set(s, e);
        }
      });
      __syncthreads();
      sub_mark(s, 26, &q);
      int carry = 0;
      for (int base = 0; base < n; base += ib()) {
        int x = base + threadIdx.x;
        int v = x < n ? ld(&s.D[x]) : 0;
        int tot;
        int pre = block_excl_scan<IB_MAX>(v, sh.red, &tot);
        if (x < n) {
          st(&s.E[x], carry + pre);
          st(&s.A[x], carry + pre);  // fill cursor
        }
        carry += tot;
      }
      total = carry;
      __syncthreads();
      sub_mark(s, 27, &q);
      for_marked_entries(s, sh, s.R, n, s.m, [&](int e) { return adj_at(s, e); }, [&](int v, int, int u) {
        int a = ldr(&s.C[v]);
        int bb = ldr(&s.C[u]);
        int pos = atomicAdd(&s.A[a], 1);
        if (pos < ldr(&s.E[a]) + ldr(&s.D[a])) st(&s.lists[pos], bb);  // within a's segment
      });
      __syncthreads();
      sub_mark(s, 28, &q);
      ph_mark(A, s, 6, &pt);
      // ---- degree check: smallest id of minimum weighted degree, strict improvement
      unsigned long long dm = ~0ull;
      for (int x = threadIdx.x; x < n; x += ib())
        if (ldr(&s.C[x]) == x) {
          unsigned long long v = ((unsigned long long)(uint32_t)ldr(&s.D[x]) << 32) | (uint32_t)x;
          dm = v < dm ? v : dm;
        }
      dm = block_min_u64<IB_MAX>(dm, sh.redu);
      int dmin = (int)(dm >> 32), xmin = (int)(dm & 0xffffffffu);
      if (dmin < bound) {
        bound = dmin;
        s_kind = 2;
        for (int v = threadIdx.x; v < n; v += ib()) st(&s.F[v], (int32_t)(ldr(&s.C[v]) == xmin));
        __syncthreads();
        if (bound <= 1) break;
      }
      ph_mark(A, s, 7, &pt);
    }
  }
  if (bound < 0) bound = -bound;
  if (s_kind != 2)
    for (int v = threadIdx.x; v < n; v += ib()) st(&s.F[v], (int32_t)(s_kind == 1 && v == dv));
  __syncthreads();
  *steps_out += steps;
  *rounds_out += rounds;
  return bound;
}

// ---------------------------------------------------------------- one item
// Geometry and LDS footprint (32-bit words) of an item.
struct Geo {
  int lv, nw0, nw1, nw2, ls;
  long long core;  // bitmaps + A, B, D, E, R
  long long marks; // contraction mark bits
  long long adj;   // 16-bit adjacency copy
};
DEV Geo item_geo(int n, long long m, int cap) {
  Geo g;
  g.lv = (int)item_levels(n, m, cap);
  g.nw0 = (n + 63) / 64;
  g.nw1 = (g.nw0 + 63) / 64;
  g.nw2 = (g.nw1 + 63) / 64;
  g.ls = g.nw0 + g.nw1 + g.nw2;
  g.core = 2LL * g.lv * g.ls + 5LL * n;
  g.marks = (m + 31) / 32 + 1;
  g.adj = n <= 65536 ? (m + 1) / 2 : (1LL << 40);
  return g;
}

// LDS selects where the scan arrays live; instantiating both placements lets the
// compiler emit LDS instructions (not generic ones) when they are in LDS.
// Placement of the optional LDS arrays after the core (bitmaps and A, B, D, E, R): the
// contraction mark bits, then the super-vertex ids C when `with_c`, then the 16-bit
// adjacency copy.  The dispatcher and the item agree on it through this function.
struct LdsPlan {
  bool marks, adj;
  long long c_off, adj_off;  // word offsets after the core
};
DEV LdsPlan lds_plan(const Geo &g, int n, long long lds_words, bool with_c) {
  LdsPlan pl;
  long long used = g.core;
  pl.marks = used + g.marks <= lds_words;
  if (pl.marks) used += g.marks;
  pl.c_off = used - g.core;
  if (with_c) used += n;
  pl.adj_off = used - g.core;
  pl.adj = pl.marks && used + g.adj <= lds_words;
  return pl;
}
// C in LDS when it fits, unless that would cost the adjacency copy (read by every scan step)
DEV bool want_c_in_lds(const Geo &g, int n, long long lds_words) {
  if (g.core > lds_words) return false;
  LdsPlan without = lds_plan(g, n, lds_words, false);
  LdsPlan with = lds_plan(g, n, lds_words, true);
  if (g.core + with.adj_off > lds_words) return false;  // C itself does not fit
  return with.adj || !without.adj;
}

template <bool LDS, bool CL>
DEV void process_item_t(const ItemArgs &A, const ItemDesc &d, uint64_t *dyn, int item_index, Sh &sh) {
  const Arena &ar = A.ar[d.depth & 1];
  int n = d.n;
  int k = (int)wcc_k_of(A.crit, n, A.lin_num, A.lin_den);
  int set = A.split_only ? A.split_set[item_index] : -1;
  int cap = A.split_only ? A.split_cap[set] : k;
  Geo g = item_geo(n, d.m, cap);
  St s;
  s.n = n;
  s.m = (int)d.m;
  s.nw0 = g.nw0;
  s.nw1 = g.nw1;
  s.nw2 = g.nw2;
  s.ls = g.ls;
  s.l1 = n > 16384;
  s.C = A.sC + d.b;
  s.F = A.sF + d.b;
  s.adjg = ar.adj + d.eb;
  s.mark = A.sMark + d.eb;
  s.lists = A.sEdge + d.eb;
  s.adj16 = nullptr;
  s.own = nullptr;
  s.bits1 = nullptr;
  if constexpr (LDS) {
    s.bits = dyn;
    int32_t *w = (int32_t *)(dyn + (size_t)g.lv * g.ls);
    s.A = w;
    s.B = w + n;
    s.D = w + 2 * n;
    s.E = w + 3 * n;
    s.R = w + 4 * n;
    LdsPlan lp = lds_plan(g, n, A.lds_words, CL);
    s.markbits = lp.marks ? (uint32_t *)(w + 5 * n) : nullptr;
    if constexpr (CL) s.C = w + 5 * n + lp.c_off;
    if (lp.adj) s.adj16 = (uint16_t *)(w + 5 * n + lp.adj_off);
  } else {
    s.bits = A.gbits + (size_t)blockIdx.x * A.gbits_words;
    if ((long long)g.lv * g.ls > A.gbits_words) {
      if (threadIdx.x == 0) err(A, WCC_EUNSUPPORTED);
      return;
    }
    s.A = A.sA + d.b;
    s.B = A.sB + d.b;
    s.D = A.sD + d.b;
    s.E = A.sE + d.b;
    s.R = A.sG + d.b;
    s.markbits = nullptr;
    // The launch's LDS is otherwise unused here: it holds the chunk owners of the entry
    // passes, then the bitmaps' summary levels (set by every key raise of a scan) when
    // they fit; items whose summaries do not fit keep none (level searches read L0).
    if (A.lds_words >= IB_MAX) s.own = (int32_t *)dyn;
    if (s.l1 && IB_MAX + 2LL * g.lv * g.nw1 <= A.lds_words) s.bits1 = dyn + IB_MAX / 2;
    else s.l1 = false;
  }
  long long steps = 0, rounds = 0;
  // profile: 1 every item, 2 the first item of each launch, >= 1000 every item with at
  // least that many vertices
  s.pf = A.prof == 1 || (A.prof == 2 && item_index == 0) ||
         (A.prof >= 1000 && n >= A.prof);
  s.prof_cnt = A.cnt + CNT_PH + 16;
  unsigned long long pt = s.pf ? wall_clock64() : 0;
  // every item reads its rows at least once: vtx, rs, rd per vertex and one index per entry
  if (threadIdx.x == 0) atomicAdd(&A.cnt[CNT_ALG_BYTES], (unsigned long long)(16LL * n + 4LL * d.m));
  // row starts relative to eb, and the LDS copy of the adjacency when it fits
  for (int i = threadIdx.x; i < n; i += ib()) st(&s.R[i], (int32_t)(ar.rs[d.b + i] - d.eb));
  if (s.adj16)
    for (int e = threadIdx.x; e < s.m; e += ib()) s.adj16[e] = (uint16_t)s.adjg[e];
  __syncthreads();

  if (A.ccr_out) {
    // components of the cluster's induced subgraph (Alg. 1), labelled by smallest member
    item_cc<LDS, CL>(s, false, 0, sh);
    for (int i = threadIdx.x; i < n; i += ib()) A.ccr_out[ar.vtx[d.b + i]] = ar.vtx[d.b + ld(&s.B[i])];
    __syncthreads();
    return;
  }
  if (A.split_only) {
    // mincut_split: disconnected -> 0 and the component of the first vertex
    int nc = item_cc<LDS, CL>(s, false, 0, sh);
    int lam;
    if (n < 2) {
      lam = 0;
      for (int i = threadIdx.x; i < n; i += ib()) st(&s.F[i], 0);
      __syncthreads();
    } else if (nc > 1) {
      lam = 0;
      for (int i = threadIdx.x; i < n; i += ib()) st(&s.F[i], (int32_t)(ld(&s.B[i]) == 0));
      __syncthreads();
    } else {
      lam = item_mincut<LDS, CL>(A, s, d, cap, sh, &steps, &rounds);
    }
    int64_t p0 = A.split_pos[set];
    for (int i = threadIdx.x; i < n; i += ib()) A.split_side[p0 + i] = (uint8_t)ld(&s.F[i]);
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
    int nc = item_cc<LDS, CL>(s, false, 0, sh);
    ph_mark(A, s, 0, &pt);
    if (nc > 1) {
      item_rebuild<LDS, CL>(A, s, d, A.s_pre, sh);
      ph_mark(A, s, 9, &pt);
      return;
    }
    if (n <= A.s_pre) return;
  }
  if (threadIdx.x == 0) atomicAdd(&A.cnt[CNT_ITEMS], 1ull);
  if (A.mode == WCC_PRUNE_KCORE) {
    int removed = item_peel<LDS, CL>(s, k, sh);
    ph_mark(A, s, 1, &pt);
    if (removed > 0) {
      if (removed < n) {
        item_cc<LDS, CL>(s, true, k, sh);
        item_rebuild<LDS, CL>(A, s, d, A.s_post, sh);
      }
      ph_mark(A, s, 2, &pt);
      return;
    }
  } else if (d.m == 0) {
    return;  // Alg. 3 tests only sets with at least one edge
  } else if (A.leaf_batch || A.low_runs) {
    // Phase 0's minimum degree: 1 means a run of single-vertex splits (peeled at once)
    int dmin = 0x7fffffff;
    for (int i = threadIdx.x; i < n; i += ib()) {
      int dg = row_end(s, i) - ldr(&s.R[i]);
      dmin = dg < dmin ? dg : dmin;
    }
    dmin = (int)block_min_u64<IB_MAX>((unsigned long long)(uint32_t)dmin, sh.redu);
    if (dmin == 1 && A.leaf_batch) {
      if (item_leaf_peel<LDS, CL>(A, s, d, sh) > 0) item_rebuild<LDS, CL>(A, s, d, A.s_post, sh);
      ph_mark(A, s, 9, &pt);
      return;
    }
    // a run of single-vertex splits at the minimum degree, removed at once when certified
    if (A.low_runs && dmin >= 1 && dmin < k && k <= 64) {
      int left = item_low_run<LDS, CL>(A, s, d, dmin, sh);
      if (left >= 0) {
        if (left > 0) item_rebuild<LDS, CL>(A, s, d, A.s_post, sh);
        ph_mark(A, s, 9, &pt);
        return;
      }
    }
  }
  int lam = item_mincut<LDS, CL>(A, s, d, k, sh, &steps, &rounds);
  pt = s.pf ? wall_clock64() : 0;
  // record: |S| and the order-free hash of S's global ids
  int ss = 0;
  unsigned long long hs = 0;
  if (threadIdx.x == 0) sh.hsum = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += ib())
    if (ld(&s.F[i])) {
      ss++;
      hs += vhash(ar.vtx[d.b + i]);
    }
  if (hs) atomicAdd(&sh.hsum, hs);
  ss = block_sum<IB_MAX>(ss, sh.red);
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
    for (int i = threadIdx.x; i < n; i += ib()) A.acc[ar.vtx[d.b + i]] = key;
    if (threadIdx.x == 0) {
      atomicAdd(&A.cnt[CNT_ACCEPTED], 1ull);
      atomicAdd(&A.cnt[CNT_ALG_BYTES], (unsigned long long)(4LL * n));
    }
    __syncthreads();
    return;
  }
  // split along the cut: label each side by its smallest member
  unsigned long long mS = ~0ull, mC = ~0ull;
  for (int i = threadIdx.x; i < n; i += ib()) {
    if (ld(&s.F[i])) mS = (unsigned long long)i < mS ? (unsigned long long)i : mS;
    else mC = (unsigned long long)i < mC ? (unsigned long long)i : mC;
  }
  mS = block_min_u64<IB_MAX>(mS, sh.redu);
  mC = block_min_u64<IB_MAX>(mC, sh.redu);
  for (int i = threadIdx.x; i < n; i += ib()) st(&s.B[i], ld(&s.F[i]) ? (int)mS : (int)mC);
  __syncthreads();
  ph_mark(A, s, 8, &pt);
  item_rebuild<LDS, CL>(A, s, d, A.s_post, sh);
  ph_mark(A, s, 9, &pt);
}

DEV void process_item(const ItemArgs &A, const ItemDesc &d, uint64_t *dyn, int item_index, Sh &sh) {
  int n = d.n;
  int cap = A.split_only ? A.split_cap[A.split_set[item_index]] : (int)wcc_k_of(A.crit, n, A.lin_num, A.lin_den);
  if (n >= (1 << 24)) {  // ids of the scan's packed reduction
    if (threadIdx.x == 0) err(A, WCC_EUNSUPPORTED);
    return;
  }
  Geo g = item_geo(n, d.m, cap);
  if (g.core > A.lds_words) process_item_t<false, false>(A, d, dyn, item_index, sh);
  else if (want_c_in_lds(g, n, A.lds_words)) process_item_t<true, true>(A, d, dyn, item_index, sh);
  else process_item_t<true, false>(A, d, dyn, item_index, sh);
}

__global__ void __launch_bounds__(IB_MAX) k_items(ItemArgs A) {
  extern __shared__ uint64_t dyn[];
  __shared__ Sh sh;
  __shared__ int cur;
  // the count of a device-driven level was written by an earlier launch
  int nit = A.nitems;
  if (A.nitems_dev) {
    int c = *A.nitems_dev;
    nit = c < nit ? c : nit;
  }
  if (threadIdx.x == 0) sh.has_keep = 0;
  __syncthreads();
  for (;;) {
    // a child kept by the previous item first (chained form), else the next list item
    if (threadIdx.x == 0) cur = sh.has_keep ? -1 : atomicAdd(A.next, 1);
    __syncthreads();
    int it = cur;
    ItemDesc d;
    if (it < 0) d = sh.keep;
    else if (it < nit) d = A.items[it];
    __syncthreads();
    if (it >= nit) break;
    if (threadIdx.x == 0) sh.has_keep = 0;
    __syncthreads();
    process_item(A, d, dyn, it, sh);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- device-driven levels
// Per-level control words: counts of the small and large lists of each parity, then the
// work counters of the level being launched.
enum : int32_t { LV_CS0 = 0, LV_CB0, LV_CS1, LV_CB1, LV_NEXT_S, LV_NEXT_B, LV_WORDS };

// Clears the output counts of parity nx and the work counters before a level.
__global__ void k_level_prep(int32_t *ctl, int nx) {
  if (threadIdx.x == 0) {
    ctl[2 * nx] = 0;
    ctl[2 * nx + 1] = 0;
    ctl[LV_NEXT_S] = 0;
    ctl[LV_NEXT_B] = 0;
  }
}

// Splits the sorted initial items into the parity-0 lists: the first *nbig (largest
// first) are large, the rest small.  When g_nitems >= 0 the device-side sizes must equal
// the ones the launch sequence was recorded for (item count, large count, largest n);
// otherwise both lists stay empty and WCC_ECANCELLED is reported.
__global__ void k_route0(const ItemDesc *sorted, int32_t nitems, const int32_t *nbig_p, const FrontCounts *fc,
                         int32_t g_nitems, int32_t g_nbig, int32_t g_top, ItemDesc *lstS, ItemDesc *lstB,
                         int32_t *ctl, unsigned long long *cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int32_t nb = nitems > 0 ? *nbig_p : 0;
  nb = nb < 0 ? 0 : (nb > nitems ? nitems : nb);
  bool bad = g_nitems >= 0 &&
             (fc->nitems != g_nitems || nb != g_nbig || (nitems > 0 && sorted[0].n != g_top));
  if (bad) {
    if (i == 0) {
      ctl[LV_CS0] = 0;
      ctl[LV_CB0] = 0;
      atomicMin((long long *)&cnt[CNT_ERR], (long long)WCC_ECANCELLED);
    }
    return;
  }
  if (i < nitems) {
    if (i < nb) lstB[i] = sorted[i];
    else lstS[i - nb] = sorted[i];
  }
  if (i == 0) {
    ctl[LV_CB0] = nb;
    ctl[LV_CS0] = nitems - nb;
  }
}

// ---------------------------------------------------------------- item ordering
// Keys of a sort by descending scan-state size (largest items first); sz[0] counts the
// items whose state exceeds the small-bin LDS, sz[1..2] (64-bit) receives the largest
// bitmap a global-state item of this list or of its descendants can need.  The cut cap of
// an item is k(n) (descendants: at most k(n), monotone in n), or the caller's cap of its set.
__global__ void k_item_keys(const ItemDesc *items, int32_t n, uint32_t *keys, uint32_t *vals, SortNeed nd,
                            int32_t *sz) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ItemDesc d = items[i];
  int64_t cap = nd.caps ? nd.caps[nd.set[i]] : wcc_k_of(nd.crit, d.n, nd.lin_num, nd.lin_den);
  int64_t need = item_state_words(d.n, d.m, cap);
  keys[i] = 0x7fffffffu - (uint32_t)(need < 0x7ffffffe ? need : 0x7ffffffe);
  vals[i] = (uint32_t)i;
  if (need > nd.small_words) atomicAdd(&sz[0], 1);
  // (the list-entry bound of a descendant is unknown: every vertex pair)
  int64_t bits = nd.caps ? item_bitmap_words(d.n, d.m, cap)
                         : item_bitmap_words(d.n, (int64_t)d.n * (d.n - 1), cap);
  atomicMax((unsigned long long *)(sz + 2), (unsigned long long)bits);
}
// Keys of a largest-first sort of a list whose length is read on the device: entries
// past the count get the largest key and sort last.
__global__ void k_item_keys_dev(const ItemDesc *items, int32_t cap, const int32_t *count, uint32_t *keys,
                                uint32_t *vals) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cap) return;
  int c = *count;
  keys[i] = i < c ? 0x7fffffffu - (uint32_t)items[i].n : 0x7fffffffu;
  vals[i] = (uint32_t)i;
}

__global__ void k_item_gather(const ItemDesc *in, const uint32_t *order, int32_t n, ItemDesc *out,
                              const int32_t *set_in, int32_t *set_out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = in[order[i]];
  if (set_in) set_out[i] = set_in[order[i]];
}

// ---------------------------------------------------------------- CCR labels
// Before the cluster items run: an assigned vertex is its own component (clusters with
// no induced edge have no item), an unassigned one is -1.
__global__ void k_ccr_init(const int32_t *mem, int64_t N, int32_t *out) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < N) out[v] = mem[v] >= 0 ? (int32_t)v : -1;
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

int items_block() { return IB_SMALL; }

int items_launch(const ItemArgs &A, int grid, size_t lds_bytes, hipStream_t s) {
  if (grid <= 0 || (!A.nitems_dev && A.nitems <= 0)) return WCC_OK;
  if (lds_bytes > 65536) {
    // raised once per process to the largest budget any launch uses (threads of the
    // served form launch concurrently)
    static std::once_flag once;
    static hipError_t attr_rc = hipSuccess;
    std::call_once(once, [] {
      attr_rc = hipFuncSetAttribute((const void *)k_items, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(159 * 1024));
    });
    HIP_TRY(attr_rc);
    if (lds_bytes > 159 * 1024) return WCC_EINVAL;
  }
  int block = lds_bytes > 65536 ? IB_MAX : IB_SMALL;
  hipLaunchKernelGGL(k_items, dim3(grid), dim3(block), lds_bytes, s, A);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

int items_level_words() { return LV_WORDS; }

int items_ccr_init(const int32_t *mem, int64_t N, int32_t *out, hipStream_t s) {
  if (N <= 0) return WCC_OK;
  hipLaunchKernelGGL(k_ccr_init, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, mem, N, out);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

int items_level_prep(int32_t *ctl, int nx, hipStream_t s) {
  hipLaunchKernelGGL(k_level_prep, dim3(1), dim3(64), 0, s, ctl, nx);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

int items_route0(const ItemDesc *sorted, int32_t nitems, const int32_t *nbig, const FrontCounts *fc,
                 int32_t g_nitems, int32_t g_nbig, int32_t g_top, ItemDesc *lstS, ItemDesc *lstB, int32_t *ctl,
                 unsigned long long *cnt, hipStream_t s) {
  int blocks = nitems > 0 ? (nitems + 255) / 256 : 1;
  hipLaunchKernelGGL(k_route0, dim3(blocks), dim3(256), 0, s, sorted, nitems, nbig, fc, g_nitems, g_nbig, g_top,
                     lstS, lstB, ctl, cnt);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

int items_sort_desc(const ItemDesc *in, int32_t n, ItemDesc *out, const int32_t *set_in, int32_t *set_out,
                    uint32_t *k1, uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes,
                    hipStream_t s, const SortNeed &nd, int32_t *sz) {
  if (n <= 0) return WCC_OK;
  int rc0 = prim_fill32(sz, 0u, 4, s);
  if (rc0) return rc0;
  SortNeed nd2 = nd;
  nd2.set = set_in;
  hipLaunchKernelGGL(k_item_keys, dim3((n + 255) / 256), dim3(256), 0, s, in, n, k1, v1, nd2, sz);
  HIP_TRY(hipGetLastError());
  int bits = 31, alt = 0;
  int rc = prim_radix_sort_pairs(k1, v1, k2, v2, n, bits, tmp, tmp_bytes, s, &alt);
  if (rc) return rc;
  hipLaunchKernelGGL(k_item_gather, dim3((n + 255) / 256), dim3(256), 0, s, in, alt ? v2 : v1, n, out,
                     set_in, set_out);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

int items_sort_desc_dev(const ItemDesc *in, int32_t cap, const int32_t *count, ItemDesc *out, uint32_t *k1,
                        uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes, hipStream_t s) {
  if (cap <= 0) return WCC_OK;
  hipLaunchKernelGGL(k_item_keys_dev, dim3((cap + 255) / 256), dim3(256), 0, s, in, cap, count, k1, v1);
  HIP_TRY(hipGetLastError());
  int alt = 0;
  int rc = prim_radix_sort_pairs(k1, v1, k2, v2, cap, 31, tmp, tmp_bytes, s, &alt);
  if (rc) return rc;
  hipLaunchKernelGGL(k_item_gather, dim3((cap + 255) / 256), dim3(256), 0, s, in, alt ? v2 : v1, cap, out,
                     (const int32_t *)nullptr, (int32_t *)nullptr);
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
