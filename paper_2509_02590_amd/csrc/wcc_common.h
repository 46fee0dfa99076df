// wcc_common.h -- shared definitions of the gfx950 WCC library (device helpers, item
// descriptors, launch arguments).  Internal header; the public ABI is include/wcc.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wcc.h"

#define WCC_WAVE 64

// ---------------------------------------------------------------- error plumbing
void wcc_note_hip_error(hipError_t e, const char *expr, const char *file, int line);

#define HIP_TRY(expr)                                          \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) {                                    \
      wcc_note_hip_error(_e, #expr, __FILE__, __LINE__);       \
      return WCC_EHIP;                                         \
    }                                                          \
  } while (0)

// ---------------------------------------------------------------- criterion k(n)
// Least integer strictly above f(n) (Sec. 2 criteria; Alg. 3 accepts "cut > f(n)").
__host__ __device__ inline int64_t wcc_k_of(int32_t crit, int64_t n, int32_t num, int32_t den) {
  if (n < 1) return 0;
  if (crit == WCC_CRIT_LOG10) {
    int64_t k = 1, p = 10;
    while (p <= n) {
      p *= 10;
      k++;
    }
    return k;
  }
  if (crit == WCC_CRIT_LOG2) {
    int64_t k = 0;
    while (n >> k) k++;
    return k;
  }
  if (crit == WCC_CRIT_SQRT) {
    // integer square root by bisection on r*r <= n
    int64_t lo = 0, hi = 3037000499LL;
    while (lo < hi) {
      int64_t mid = (lo + hi + 1) >> 1;
      if (mid <= n / mid) lo = mid;
      else hi = mid - 1;
    }
    return lo + 1;
  }
  return ((int64_t)num * n) / den + 1;
}

// ---------------------------------------------------------------- scan-state geometry
// A cut capped at `cap` keeps its keys below bound + 1 levels, bound = min(cap, delta), and
// the minimum degree delta of an item with n vertices and m list entries is at most m / n
// (and n - 1).  The scan holds one bitmap per key level: a bit per vertex (nw0 64-bit
// words) plus two summary levels (nw1, nw2 words).
__host__ __device__ inline int64_t item_levels(int64_t n, int64_t m, int64_t cap) {
  if (n < 2) return 2;
  int64_t d = m / n;
  if (d > n - 1) d = n - 1;
  int64_t b = cap < d ? cap : d;
  return (b < 1 ? 1 : b) + 1;
}
__host__ __device__ inline int64_t item_level_words(int64_t n) {
  int64_t nw0 = (n + 63) / 64, nw1 = (nw0 + 63) / 64, nw2 = (nw1 + 63) / 64;
  return nw0 + nw1 + nw2;
}
// 64-bit bitmap words of the scan (all levels)
__host__ __device__ inline int64_t item_bitmap_words(int64_t n, int64_t m, int64_t cap) {
  return item_levels(n, m, cap) * item_level_words(n);
}
// 32-bit LDS words of the scan state kept in LDS: the bitmaps and five words per vertex
// (keys, union-find, list lengths, list starts, row starts)
__host__ __device__ inline int64_t item_state_words(int64_t n, int64_t m, int64_t cap) {
  return 2 * item_bitmap_words(n, m, cap) + 5 * n;
}

// ---------------------------------------------------------------- item descriptors
// A queued vertex set ("item") lives in one of two arenas (depth & 1): positions
// [b, b+n) hold its vertices in ascending global id (local id = position - b), and its
// induced subgraph's rows occupy entries [eb, eb+m) of that arena.  Children of an item
// are written into the other arena inside the same position and entry ranges.
enum : int32_t { ITEM_CCR = 1 };  // top-level cluster: CCR components first (Alg. 1)

struct ItemDesc {
  int32_t b;
  int32_t n;
  int64_t eb;
  int64_t m;
  int32_t depth;
  int32_t flags;
};
static_assert(sizeof(ItemDesc) == 32, "descriptor layout");

struct Arena {
  int32_t *vtx;  // positions -> global vertex id
  int64_t *rs;   // positions -> row start (absolute entry index)
  int32_t *rd;   // positions -> row length
  int32_t *adj;  // entries -> local id of the neighbour
};

// counters accumulated on the device (int64 each)
enum : int32_t {
  CNT_ITEMS = 0,
  CNT_MINCUTS,
  CNT_ACCEPTED,
  CNT_STEPS,
  CNT_ROUNDS,
  CNT_RECORDS,
  CNT_ERR,  // first error code seen by a kernel (atomicMin of negative codes)
  CNT_ALG_BYTES,  // algorithmic bytes of the item launches (reads + writes)
  CNT_PH,         // 16 slots: optional per-phase clock totals (profiling builds of a run)
  CNT_PH_END = CNT_PH + 32,
  CNT_NUM
};

struct ItemArgs {
  Arena ar[2];
  int32_t *sA, *sB, *sC, *sD, *sE, *sF;  // per-position scratch
  int32_t *sG;                      // per-position scratch (row starts of global-state items)
  int32_t *sEdge;                   // per-entry scratch (crossing lists)
  uint8_t *sMark;                   // per-entry scratch (contraction marks)
  uint64_t *gbits;                  // per-workgroup bitmap regions (large items)
  int64_t gbits_words;              // words per workgroup region
  int32_t *acc;                     // N: smallest global id of the saved set, or -1
  const ItemDesc *items;            // this launch's items
  int32_t nitems;
  int32_t *next;                    // work counter of this launch
  ItemDesc *out;                    // children
  int32_t *out_count;
  int32_t out_cap;
  int32_t crit, lin_num, lin_den, s_pre, s_post, mode;
  int32_t lds_words;                // 32-bit words of dynamic LDS per workgroup
  wcc_record *rec;
  int64_t rec_cap;
  unsigned long long *cnt;          // CNT_* counters
  int32_t prof;                     // accumulate per-phase clock totals into CNT_PH slots
  int32_t split_only;               // mincut_split mode: items are caller sets
  int32_t *split_lambda;            // per set (mincut_split mode)
  uint8_t *split_side;              // per position (mincut_split mode)
  const int32_t *split_set;         // per item: index of the caller's set
  const int32_t *split_cap;         // per set
  const int64_t *split_pos;         // per set: offset of its first vertex in the caller's order
  // device-driven levels (batched form): the item count of the launch is read on the
  // device, and children whose scan state exceeds small_words go to a second list
  const int32_t *nitems_dev;        // when set, the launch's item count (overrides nitems),
                                    // clamped to nitems (the list's capacity)
  ItemDesc *out_big;                // children with a larger state (nullptr: all go to out)
  int32_t *out_big_count;
  int32_t out_big_cap;
  int64_t small_words;              // LDS words of a small-bin workgroup
  // CCR only: each vertex of a processed cluster gets the smallest global id of its
  // component inside the cluster's induced subgraph (no cut, no children)
  int32_t *ccr_out;
  // PAPER mode: items with a vertex of degree 1 are peeled to their 2-core in one batch
  // (every step of the one-at-a-time peel fails its cut: k(s_post + 1) >= 2)
  int32_t leaf_batch;
  // PAPER mode: runs of single-vertex splits at the minimum degree (>= 2) are removed in
  // one batch when a certificate shows that every one of them is the canonical cut
  int32_t low_runs;
  // chained form (batched execution): a workgroup that splits an item processes one of the
  // children itself, next, instead of leaving every child to the next launch
  int32_t chain;
  int32_t chain_min_n;  // only children of at least this many vertices are chained
};

// ---------------------------------------------------------------- device helpers
#ifdef __HIP_DEVICE_COMPILE__
#define DEV __device__ __forceinline__
#else
#define DEV __device__ inline
#endif

// Relaxed agent-scope loads/stores: used for every scratch word other lanes may write
// during a kernel, so that no stale vector-L1 copy is read (they also work on LDS
// addresses through generic pointers).
template <typename T>
DEV T ld(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Plain (cached) load for scratch that only this workgroup writes and that is read after
// a barrier: all waves of a workgroup share one CU's vector L1, which stays coherent with
// their own stores, so the value is current; unlike ld() the compiler may batch and
// reorder these loads.
template <typename T>
DEV T ldr(const T *p) {
  return *p;
}
template <typename T, typename U>
DEV void st(T *p, U v) {
  __hip_atomic_store(p, (T)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

DEV unsigned lane_id() { return __lane_id(); }

DEV uint64_t lanemask_lt() {
  unsigned l = __lane_id();
  return l ? (~0ull >> (64 - l)) : 0ull;
}

DEV int wave_incl_sum(int v) {
  unsigned l = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (l >= (unsigned)d) v += t;
  }
  return v;
}
DEV long long wave_incl_sum64(long long v) {
  unsigned l = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    long long t = __shfl_up(v, d, 64);
    if (l >= (unsigned)d) v += t;
  }
  return v;
}
DEV int wave_sum(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}
DEV unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    unsigned long long t = __shfl_xor(v, d, 64);
    v = t < v ? t : v;
  }
  return v;
}

// Block-wide reductions and scans for blocks of up to BLOCK threads (the block size of the
// launch, a multiple of 64, is read at run time).  red must hold >= BLOCK/64 + 1 entries.
// Block-wide exclusive scan of one int per thread.  Returns the exclusive prefix; *total
// gets the block sum.  Contains barriers.
template <int BLOCK>
DEV int block_excl_scan(int v, int *red, int *total) {
  const int NW = (int)(blockDim.x >> 6);
  int inc = wave_incl_sum(v);
  int w = threadIdx.x >> 6;
  if (__lane_id() == 63) red[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int s = 0;
    for (int i = 0; i < NW; i++) {
      int t = red[i];
      red[i] = s;
      s += t;
    }
    red[NW] = s;
  }
  __syncthreads();
  int r = red[w] + inc - v;
  *total = red[NW];
  __syncthreads();
  return r;
}

template <int BLOCK>
DEV long long block_excl_scan64(long long v, long long *red, long long *total) {
  const int NW = (int)(blockDim.x >> 6);
  long long inc = wave_incl_sum64(v);
  int w = threadIdx.x >> 6;
  if (__lane_id() == 63) red[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    for (int i = 0; i < NW; i++) {
      long long t = red[i];
      red[i] = s;
      s += t;
    }
    red[NW] = s;
  }
  __syncthreads();
  long long r = red[w] + inc - v;
  *total = red[NW];
  __syncthreads();
  return r;
}

template <int BLOCK>
DEV unsigned long long block_min_u64(unsigned long long v, unsigned long long *red) {
  const int NW = (int)(blockDim.x >> 6);
  v = wave_min_u64(v);
  int w = threadIdx.x >> 6;
  if (__lane_id() == 0) red[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = red[0];
    for (int i = 1; i < NW; i++) m = red[i] < m ? red[i] : m;
    red[NW] = m;
  }
  __syncthreads();
  unsigned long long r = red[NW];
  __syncthreads();
  return r;
}

template <int BLOCK>
DEV int block_sum(int v, int *red) {
  int t;
  block_excl_scan<BLOCK>(v, red, &t);
  return t;
}

// order-free set hash term (matches wcc_record.shash)
DEV uint64_t vhash(int32_t v) {
  uint64_t z = (uint64_t)(uint32_t)v + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// ---------------------------------------------------------------- host launch helpers
// (implemented in wcc_prims.hip)
int prim_excl_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total_dev,
                       void *tmp, size_t tmp_bytes, hipStream_t s);
int prim_excl_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev,
                       void *tmp, size_t tmp_bytes, hipStream_t s);
size_t prim_scan_tmp_bytes(int64_t n);
int prim_radix_sort_pairs(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                          int64_t n, int bits, void *tmp, size_t tmp_bytes, hipStream_t s,
                          int *result_in_alt, const int32_t *maxkey_m1 = nullptr);
int prim_fill32(void *p, uint32_t v, int64_t nwords, hipStream_t s);
size_t prim_radix_tmp_bytes(int64_t n);
