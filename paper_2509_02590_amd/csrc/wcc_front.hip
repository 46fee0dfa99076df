// wcc_front.hip -- the front end of the WCC path on gfx950:
//   * CSR validation (optional),
//   * grouping of vertices by input cluster (stable radix sort on the cluster id, so
//     vertices stay in ascending id inside a cluster: local id = rank, Alg. 1 V_c),
//   * membership-filtered CSR compaction: every cluster's induced subgraph
//     E_c = {(u,v) in E : u, v in V_c} (Alg. 1, Alg. 2, Alg. 3) with local ids, laid out
//     cluster-major in arena 0,
//   * the initial item list (clusters with at least one induced edge, Alg. 1).
//
// Entry-parallel passes walk the input CSR in tiles of consecutive entries; each tile
// finds the rows it covers with one binary search and then locates every entry's row in
// LDS, so hub rows and short rows cost the same per entry and index loads are coalesced.
#include "wcc_internal.h"

namespace {

constexpr int FB = 256;             // block
constexpr int FITEMS = 8;           // entries per thread per tile
constexpr int FTILE = FB * FITEMS;  // entries per tile
constexpr int FROWS = FTILE + 1;    // row offsets cached per tile

template <typename OT>
DEV int64_t row_of(const OT *off, int64_t lo, int64_t hi, int64_t e) {
  // largest r in [lo, hi] with off[r] <= e
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if ((int64_t)off[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Per tile: the range of rows [r0, r1] covering entries [e0, e1) and, when it fits, their
// offsets in LDS.  Returns true when cached.
template <typename OT>
DEV bool tile_rows(const OT *off, int64_t N, int64_t e0, int64_t e1, int64_t *sh_r, int64_t *cache) {
  if (threadIdx.x == 0) sh_r[0] = row_of(off, 0, N - 1, e0);
  if (threadIdx.x == 1) sh_r[1] = row_of(off, 0, N - 1, e1 - 1);
  __syncthreads();
  int64_t r0 = sh_r[0], r1 = sh_r[1];
  bool cached = (r1 - r0 + 2) <= FROWS;
  if (cached)
    for (int64_t i = threadIdx.x; i < r1 - r0 + 2; i += FB) cache[i] = (int64_t)off[r0 + i];
  __syncthreads();
  return cached;
}

DEV int64_t row_in_cache(const int64_t *cache, int64_t nr, int64_t e) {
  int64_t lo = 0, hi = nr - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi + 1) >> 1;
    if (cache[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- validation
template <typename OT>
__global__ void __launch_bounds__(FB) k_validate_offsets(const OT *off, int64_t N, int64_t nnz,
                                                         unsigned long long *bad) {
  int64_t i = (int64_t)blockIdx.x * FB + threadIdx.x;
  if (i > N) return;
  bool b = false;
  if (i == 0) b = off[0] != 0;
  else b = off[i] < off[i - 1];
  if (i == N) b = b || (int64_t)off[N] != nnz;
  if (b) atomicAdd(&bad[0], 1ull);
}

DEV uint64_t pair_mix(uint64_t a, uint64_t b) {
  uint64_t z = a * 0x9E3779B97F4A7C15ULL + b + 0x632BE59BD9B4E019ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// bad[1]: out-of-range or self-loop entries; bad[2]: sum of h(v,u) - h(u,v) over all
// entries (zero for a symmetric entry multiset, up to a 2^-64 collision chance).
template <typename OT>
__global__ void __launch_bounds__(FB) k_validate_entries(const OT *off, const int32_t *idx, int64_t N,
                                                         int64_t nnz, unsigned long long *bad) {
  __shared__ int64_t sh_r[2];
  __shared__ int64_t cache[FROWS];
  int64_t e0 = (int64_t)blockIdx.x * FTILE, e1 = e0 + FTILE < nnz ? e0 + FTILE : nnz;
  bool cached = tile_rows(off, N, e0, e1, sh_r, cache);
  int64_t r0 = sh_r[0], r1 = sh_r[1];
  unsigned long long nb = 0, h = 0;
  for (int i = 0; i < FITEMS; i++) {
    int64_t e = e0 + (int64_t)i * FB + threadIdx.x;
    if (e >= e1) break;
    int64_t v = cached ? r0 + row_in_cache(cache, r1 - r0 + 2, e) : row_of(off, r0, r1, e);
    int32_t u = idx[e];
    if (u < 0 || u >= N || u == v) nb++;
    h += pair_mix((uint64_t)v, (uint64_t)(uint32_t)u) - pair_mix((uint64_t)(uint32_t)u, (uint64_t)v);
  }
  if (nb) atomicAdd(&bad[1], nb);
  if (h) atomicAdd(&bad[2], h);
}

// bad[3]: entries whose neighbour id already occurs earlier in the same row (parallel
// edges).  Row v owns the open-addressing table slots [2*off[v], 2*off[v+1]) (twice its
// length, so linear probing always finds a free slot), split over two scratch arrays of
// nnz words each (tabA: slots below nnz, tabB: the rest), filled with -1 beforehand.  An
// insertion that meets its own id counts one duplicate; exact for any row length.
template <typename OT>
__global__ void __launch_bounds__(FB) k_validate_dups(const OT *off, const int32_t *idx, int64_t N, int64_t nnz,
                                                      int32_t *tabA, int32_t *tabB, unsigned long long *bad) {
  __shared__ int64_t sh_r[2];
  __shared__ int64_t cache[FROWS];
  int64_t e0 = (int64_t)blockIdx.x * FTILE, e1 = e0 + FTILE < nnz ? e0 + FTILE : nnz;
  bool cached = tile_rows(off, N, e0, e1, sh_r, cache);
  int64_t r0 = sh_r[0], r1 = sh_r[1];
  unsigned long long nd = 0;
  for (int i = 0; i < FITEMS; i++) {
    int64_t e = e0 + (int64_t)i * FB + threadIdx.x;
    if (e >= e1) break;
    int64_t v = cached ? r0 + row_in_cache(cache, r1 - r0 + 2, e) : row_of(off, r0, r1, e);
    int64_t b = (int64_t)off[v], len = (int64_t)off[v + 1] - b;
    int32_t u = idx[e];
    int64_t size = 2 * len, base = 2 * b;
    int64_t h = (int64_t)(pair_mix((uint64_t)(uint32_t)u, 0x5bd1e995ull) % (uint64_t)size);
    for (int64_t t = 0; t < size; t++) {
      int64_t slot = base + h;
      int32_t *p = slot < nnz ? &tabA[slot] : &tabB[slot - nnz];
      int32_t old = atomicCAS(p, -1, u);
      if (old == -1) break;
      if (old == u) {
        nd++;
        break;
      }
      h = h + 1 == size ? 0 : h + 1;
    }
  }
  if (nd) atomicAdd(&bad[3], nd);
}

// ---------------------------------------------------------------- grouping
// Every size the front end produces (assigned vertices na, clusters K, intra entries E,
// initial items) stays in device counters (FrontCounts), so the whole front end runs
// without a host synchronisation and can be captured in a graph.
__global__ void k_member_stats(const int32_t *mem, int64_t N, FrontCounts *fc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t m = -1;
  int c = 0;
  if (i < N) {
    m = mem[i];
    c = m >= 0;
  }
  __shared__ int ws[16], wm[16];
  int s = wave_sum(c);
  int32_t mx = m;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    int32_t t = __shfl_xor(mx, d, 64);
    mx = t > mx ? t : mx;
  }
  if (__lane_id() == 0) {
    ws[threadIdx.x >> 6] = s;
    wm[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // one pair of atomics per block
    int ts = 0, tm = -1;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) {
      ts += ws[w];
      tm = wm[w] > tm ? wm[w] : tm;
    }
    if (ts) atomicAdd((unsigned long long *)&fc->na, (unsigned long long)ts);
    if (tm >= 0) atomicMax(&fc->maxid, tm);
  }
}

// unassigned vertices get key maxid + 1, so they sort after every cluster
__global__ void k_sort_init(const int32_t *mem, int64_t N, const FrontCounts *fc, uint32_t *keys,
                            uint32_t *vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int32_t m = mem[i];
  keys[i] = m >= 0 ? (uint32_t)m : (uint32_t)(fc->maxid + 1);
  vals[i] = (uint32_t)i;
}

__global__ void k_cluster_flags(const uint32_t *keys, int64_t N, const FrontCounts *fc, int32_t *flag) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  int64_t na = fc->na;
  flag[p] = (p < na && (p == 0 || keys[p] != keys[p - 1])) ? 1 : 0;
}

// cid = exclusive-scan(flag) + flag - 1 ; record cluster starts and per-vertex tables
__global__ void k_cluster_tables(const uint32_t *keys, const uint32_t *vals, const int32_t *flag,
                                 const int32_t *flag_scan, int64_t N, const FrontCounts *fc,
                                 int64_t *cl_start, int32_t *cl_ids, int32_t *cidv, int32_t *vtx0) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t na = fc->na;
  if (p >= na) return;
  int32_t c = flag_scan[p] + flag[p] - 1;
  uint32_t v = vals[p];
  if (flag[p]) {
    cl_start[c] = p;
    if (cl_ids) cl_ids[c] = (int32_t)keys[p];
  }
  if (p == na - 1) cl_start[c + 1] = na;
  cidv[v] = c;
  vtx0[p] = (int32_t)v;
}

// posv[v] = v's cluster-major position (its local id plus its cluster's start), -1 for an
// unassigned vertex (filled beforehand).  u is in cluster c exactly when posv[u] lies in
// [cl_start[c], cl_start[c+1]), so the staging pass gathers one word per entry (the test and
// the local id at once).
__global__ void k_cluster_pos(const int32_t *vtx0, const FrontCounts *fc, int32_t *posv) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= fc->na) return;
  posv[vtx0[p]] = (int32_t)p;
}

// ---------------------------------------------------------------- compaction
// Two passes, one gather: the staging pass reads every entry and gathers the neighbour's
// cluster-major position once (the membership test and the local id at once), writing
// each row's intra entries to the start of the row's own CSR range in a staging array
// (deg_in[v] counts them and is the row's cursor); the copy pass streams the rows, in
// cluster-major order, from there into arena 0.  Inside a tile a row's intra entries are
// counted in LDS first, so each (row, tile) pair reserves its slots with one global atomic.
template <typename OT>
__global__ void __launch_bounds__(FB) k_stage_intra(const OT *off, const int32_t *idx, int64_t N, int64_t nnz,
                                                    const int32_t *cidv, const int32_t *posv,
                                                    const int64_t *cl_start, int32_t *deg_in, int32_t *stage) {
  __shared__ int64_t sh_r[2];
  __shared__ int64_t cache[FROWS];
  __shared__ int cnt[FROWS];
  int64_t e0 = (int64_t)blockIdx.x * FTILE, e1 = e0 + FTILE < nnz ? e0 + FTILE : nnz;
  bool cached = tile_rows(off, N, e0, e1, sh_r, cache);
  int64_t r0 = sh_r[0], r1 = sh_r[1];
  if (!cached) {
    for (int i = 0; i < FITEMS; i++) {
      int64_t e = e0 + (int64_t)i * FB + threadIdx.x;
      if (e >= e1) break;
      int64_t v = row_of(off, r0, r1, e);
      int32_t cv = cidv[v];
      if (cv < 0) continue;
      int64_t lo = cl_start[cv];
      int32_t pu = posv[idx[e]];
      if (pu < lo || pu >= cl_start[cv + 1]) continue;
      int32_t slot = atomicAdd(&deg_in[v], 1);
      stage[(int64_t)off[v] + slot] = (int32_t)(pu - lo);
    }
    return;
  }
  int nr = (int)(r1 - r0 + 1);
  for (int i = threadIdx.x; i < nr; i += FB) cnt[i] = 0;
  __syncthreads();
  int val[FITEMS], slot[FITEMS], row[FITEMS];
#pragma unroll
  for (int i = 0; i < FITEMS; i++) {
    val[i] = -1;
    int64_t e = e0 + (int64_t)i * FB + threadIdx.x;
    if (e >= e1) continue;
    int r = (int)row_in_cache(cache, nr + 1, e);
    row[i] = r;
    int32_t cv = cidv[r0 + r];
    if (cv < 0) continue;
    int64_t lo = cl_start[cv];
    int32_t pu = posv[idx[e]];
    if (pu < lo || pu >= cl_start[cv + 1]) continue;
    val[i] = (int32_t)(pu - lo);
    slot[i] = atomicAdd(&cnt[r], 1);
  }
  __syncthreads();
  // one reservation per row of the tile; cache[] (the row starts) becomes the write base
  for (int r = threadIdx.x; r < nr; r += FB) {
    int c = cnt[r];
    if (c) cache[r] += atomicAdd(&deg_in[r0 + r], c);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < FITEMS; i++)
    if (val[i] >= 0) stage[cache[row[i]] + slot[i]] = val[i];
}

__global__ void k_gather_deg(const int32_t *vtx0, const int32_t *deg_in, int64_t N, const FrontCounts *fc,
                             int32_t *rd0, int64_t *rs0) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  int32_t d = p < fc->na ? deg_in[vtx0[p]] : 0;
  rd0[p] = d;
  rs0[p] = d;
}

// adj0[d] for every entry d < E of arena 0: the row of position p (tile rows from rs0,
// rs0[N] = E) is v = vtx0[p], whose intra entries start at off[v] in the staging array.
// Grid sized for nnz; tiles at or beyond E exit.
template <typename OT>
__global__ void __launch_bounds__(FB) k_copy_intra(const OT *off, const int32_t *vtx0, const int64_t *rs0,
                                                   int64_t N, const FrontCounts *fc, const int32_t *stage,
                                                   int32_t *adj0) {
  __shared__ int64_t sh_r[2];
  __shared__ int64_t cache[FROWS];
  __shared__ int64_t src[FROWS];
  const int64_t E = fc->E;
  int64_t e0 = (int64_t)blockIdx.x * FTILE;
  if (e0 >= E) return;
  int64_t e1 = e0 + FTILE < E ? e0 + FTILE : E;
  bool cached = tile_rows(rs0, N, e0, e1, sh_r, cache);
  int64_t r0 = sh_r[0], r1 = sh_r[1];
  if (!cached) {
    for (int i = 0; i < FITEMS; i++) {
      int64_t d = e0 + (int64_t)i * FB + threadIdx.x;
      if (d >= e1) break;
      int64_t p = row_of(rs0, r0, r1, d);
      adj0[d] = stage[(int64_t)off[vtx0[p]] + (d - rs0[p])];
    }
    return;
  }
  int nr = (int)(r1 - r0 + 1);
  for (int i = threadIdx.x; i < nr; i += FB) src[i] = (int64_t)off[vtx0[r0 + i]] - cache[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < FITEMS; i++) {
    int64_t d = e0 + (int64_t)i * FB + threadIdx.x;
    if (d >= e1) break;
    adj0[d] = stage[src[row_in_cache(cache, nr + 1, d)] + d];
  }
}

__global__ void k_make_items(const int64_t *cl_start, const int32_t *cl_ids, int64_t N, const FrontCounts *fc,
                             const int64_t *rs0, ItemDesc *items, int32_t *item_set, bool all) {
  int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t K = fc->K, na = fc->na, E = fc->E;
  if (c >= K) return;
  int64_t b = cl_start[c];
  int64_t e = cl_start[c + 1];
  int64_t eb = rs0[b];
  int64_t ee = e < na ? rs0[e] : E;
  if (!all && ee == eb) return;  // Alg. 1: clusters without induced edges are not refined
  ItemDesc d;
  d.b = (int32_t)b;
  d.n = (int32_t)(e - b);
  d.eb = eb;
  d.m = ee - eb;
  d.depth = 0;
  d.flags = all ? 0 : ITEM_CCR;
  int32_t slot = all ? (int32_t)c : atomicAdd((int32_t *)&fc->nitems, 1);
  items[slot] = d;
  if (item_set) item_set[slot] = cl_ids ? cl_ids[c] : (int32_t)c;
}

__global__ void k_finish_counts(FrontCounts *fc, int64_t *rs0, int64_t N) {
  fc->K = fc->K32;
  rs0[N] = fc->E;  // (row starts of arena 0 end with the entry count)
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------- host wrappers
int front_validate(const FrontBufs &f, hipStream_t s, int *ok) {
  int rc0 = prim_fill32(f.dcnt, 0u, 8, s);
  if (rc0) return rc0;
  unsigned gb = nblk(f.N + 1, FB), ge = nblk(f.nnz, FTILE);
  if (f.obits == 32) {
    hipLaunchKernelGGL(k_validate_offsets<int32_t>, dim3(gb), dim3(FB), 0, s, (const int32_t *)f.off,
                       f.N, f.nnz, f.dcnt);
  } else {
    hipLaunchKernelGGL(k_validate_offsets<int64_t>, dim3(gb), dim3(FB), 0, s, (const int64_t *)f.off,
                       f.N, f.nnz, f.dcnt);
  }
  unsigned long long h[4];
  HIP_TRY(hipMemcpyAsync(h, f.dcnt, sizeof(h), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (h[0]) {
    *ok = 0;
    return WCC_OK;
  }
  if (f.nnz > 0 && f.N > 0) {
    if (f.obits == 32)
      hipLaunchKernelGGL(k_validate_entries<int32_t>, dim3(ge), dim3(FB), 0, s,
                         (const int32_t *)f.off, f.idx, f.N, f.nnz, f.dcnt);
    else
      hipLaunchKernelGGL(k_validate_entries<int64_t>, dim3(ge), dim3(FB), 0, s,
                         (const int64_t *)f.off, f.idx, f.N, f.nnz, f.dcnt);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(h, f.dcnt, sizeof(h), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // parallel edges: only once ids and offsets are known to be valid
    if (h[1] == 0 && h[2] == 0) {
      int rc = prim_fill32(f.vtab_a, 0xffffffffu, f.nnz, s);
      if (!rc) rc = prim_fill32(f.vtab_b, 0xffffffffu, f.nnz, s);
      if (rc) return rc;
      if (f.obits == 32)
        hipLaunchKernelGGL(k_validate_dups<int32_t>, dim3(ge), dim3(FB), 0, s, (const int32_t *)f.off, f.idx, f.N,
                           f.nnz, f.vtab_a, f.vtab_b, f.dcnt);
      else
        hipLaunchKernelGGL(k_validate_dups<int64_t>, dim3(ge), dim3(FB), 0, s, (const int64_t *)f.off, f.idx, f.N,
                           f.nnz, f.vtab_a, f.vtab_b, f.dcnt);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(h, f.dcnt, sizeof(h), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    }
  }
  *ok = (h[1] == 0 && h[2] == 0 && h[3] == 0);
  return WCC_OK;
}

// Groups vertices by cluster and compacts every cluster's induced subgraph into arena 0:
// vtx0 (global ids, cluster-major, ascending inside a cluster), cl_start (K+1), cl_ids
// (nullable), rd0/rs0 (row lengths and starts), adj0 (local ids) and the initial items
// (clusters with at least one induced edge; with all_items, every cluster in order and
// item_set[i] = i).  Sizes end in *fc; nothing is read back to the host.
int front_build(const FrontBufs &f, FrontCounts *fc, int32_t *vtx0, int64_t *cl_start, int32_t *cl_ids,
                int32_t *rd0, int64_t *rs0, int32_t *adj0, ItemDesc *items, int32_t *item_set, bool all_items,
                hipStream_t s) {
  int64_t N = f.N;
  int rc;
  if ((rc = prim_fill32(fc, 0u, (int64_t)(sizeof(FrontCounts) / 4), s))) return rc;
  if ((rc = prim_fill32(&fc->maxid, 0xffffffffu, 1, s))) return rc;
  if ((rc = prim_fill32(f.cidv, 0xffffffffu, N, s))) return rc;
  if ((rc = prim_fill32(f.posv, 0xffffffffu, N, s))) return rc;  // cluster-major positions
  if ((rc = prim_fill32(cl_start, 0u, 2, s))) return rc;
  if (N > 0) hipLaunchKernelGGL(k_member_stats, dim3(nblk(N, 1024)), dim3(1024), 0, s, f.mem, N, fc);
  hipLaunchKernelGGL(k_sort_init, dim3(nblk(N, 256)), dim3(256), 0, s, f.mem, N, (const FrontCounts *)fc,
                     f.keys, f.vals);
  HIP_TRY(hipGetLastError());
  int alt = 0;
  // four 8-bit passes; the passes above the key range copy through (decided on the device)
  rc = prim_radix_sort_pairs(f.keys, f.vals, f.keys2, f.vals2, N, 32, f.tmp, f.tmp_bytes, s, &alt, &fc->maxid);
  if (rc) return rc;
  const uint32_t *keys = alt ? f.keys2 : f.keys;
  const uint32_t *vals = alt ? f.vals2 : f.vals;
  hipLaunchKernelGGL(k_cluster_flags, dim3(nblk(N, 256)), dim3(256), 0, s, keys, N, (const FrontCounts *)fc, f.flag);
  rc = prim_excl_scan_i32(f.flag, f.flag_scan, N, &fc->K32, f.tmp, f.tmp_bytes, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_cluster_tables, dim3(nblk(N, 256)), dim3(256), 0, s, keys, vals, f.flag, f.flag_scan, N,
                     (const FrontCounts *)fc, cl_start, cl_ids, f.cidv, vtx0);
  hipLaunchKernelGGL(k_cluster_pos, dim3(nblk(N, 256)), dim3(256), 0, s, vtx0, (const FrontCounts *)fc,
                     f.posv);
  HIP_TRY(hipGetLastError());
  // staging pass: intra entries at the start of each row's own range (arena 1 is free
  // until the first split and sized for every entry), intra degree per vertex
  if ((rc = prim_fill32(f.deg_in, 0u, N, s))) return rc;
  if (f.nnz > 0) {
    unsigned g = nblk(f.nnz, FTILE);
    if (f.obits == 32)
      hipLaunchKernelGGL(k_stage_intra<int32_t>, dim3(g), dim3(FB), 0, s, (const int32_t *)f.off, f.idx, f.N,
                         f.nnz, f.cidv, f.posv, cl_start, f.deg_in, f.stage);
    else
      hipLaunchKernelGGL(k_stage_intra<int64_t>, dim3(g), dim3(FB), 0, s, (const int64_t *)f.off, f.idx, f.N,
                         f.nnz, f.cidv, f.posv, cl_start, f.deg_in, f.stage);
  }
  // row starts by position
  hipLaunchKernelGGL(k_gather_deg, dim3(nblk(N, 256)), dim3(256), 0, s, vtx0, f.deg_in, N,
                     (const FrontCounts *)fc, rd0, rs0);
  HIP_TRY(hipGetLastError());
  rc = prim_excl_scan_i64(rs0, rs0, N, &fc->E, f.tmp, f.tmp_bytes, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_finish_counts, dim3(1), dim3(1), 0, s, fc, rs0, N);
  // copy pass: rows in cluster-major order into arena 0
  if (f.nnz > 0) {
    unsigned g = nblk(f.nnz, FTILE);
    if (f.obits == 32)
      hipLaunchKernelGGL(k_copy_intra<int32_t>, dim3(g), dim3(FB), 0, s, (const int32_t *)f.off, vtx0, rs0, N,
                         (const FrontCounts *)fc, f.stage, adj0);
    else
      hipLaunchKernelGGL(k_copy_intra<int64_t>, dim3(g), dim3(FB), 0, s, (const int64_t *)f.off, vtx0, rs0, N,
                         (const FrontCounts *)fc, f.stage, adj0);
  }
  if (items)
    hipLaunchKernelGGL(k_make_items, dim3(nblk(N, 256)), dim3(256), 0, s, cl_start, (const int32_t *)cl_ids, N,
                       (const FrontCounts *)fc, rs0, items, item_set, all_items);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

namespace {

// membership for caller sets: mem[v] = set index; bad counts unsorted, duplicate,
// out-of-range or overlapping entries and malformed offsets
__global__ void k_split_membership(const int32_t *verts, const int64_t *so, int32_t ns, int64_t nv, int64_t N,
                                   int32_t *mem, unsigned long long *bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ns) {
    if (so[i + 1] < so[i]) atomicAdd(bad, 1ull);
    if (i == 0 && so[0] != 0) atomicAdd(bad, 1ull);
  }
  if (i >= nv) return;
  int64_t lo = 0, hi = ns - 1;
  while (lo < hi) {  // set containing entry i: largest s with so[s] <= i
    int64_t mid = (lo + hi + 1) >> 1;
    if (so[mid] <= i) lo = mid;
    else hi = mid - 1;
  }
  int32_t v = verts[i];
  if (v < 0 || v >= N) {
    atomicAdd(bad, 1ull);
    return;
  }
  if (i > so[lo] && verts[i - 1] >= v) atomicAdd(bad, 1ull);
  if (atomicCAS(&mem[v], -1, (int32_t)lo) != -1) atomicAdd(bad, 1ull);
}

}  // namespace

int front_split_membership(const int32_t *verts, const int64_t *set_offsets, int32_t num_sets, int64_t nv,
                           int64_t N, int32_t *mem, unsigned long long *bad, hipStream_t s) {
  int rc;
  if ((rc = prim_fill32(mem, 0xffffffffu, N, s))) return rc;
  if ((rc = prim_fill32(bad, 0u, 2, s))) return rc;
  int64_t work = nv > num_sets ? nv : num_sets;
  if (work > 0)
    hipLaunchKernelGGL(k_split_membership, dim3(nblk(work, 256)), dim3(256), 0, s, verts, set_offsets, num_sets,
                       nv, N, mem, bad);
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

