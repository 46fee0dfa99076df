// wcc_cm.hip -- device kernels of the Connectivity Modifier (CM, Alg. 4, and its check
// CMC, Alg. 5) on gfx950.  CM keeps WCC's structure (CCR, then a minimum cut per set,
// accept when the cut exceeds the criterion, otherwise split along the cut) and adds a
// community detection step (GetCommunities with a CDA) on every side of a failing cut.
//
// A level of the CM driver works on a per-vertex label array `cur` (the smallest vertex
// id of the vertex's current set, -1 for none):
//   * the sets are grouped by a stable radix sort of the vertex ids on `cur`, giving the
//     concatenated, ascending vertex lists that mincut_split_batch takes;
//   * k_cm_outcome* turn the cuts into saved sets, split records and the two parts of every
//     failing set (each part labelled by its smallest vertex, parts of at most s_post
//     vertices dropped);
//   * the CDA labels the vertices of every part with a community;
//   * k_cm_next* group the vertices by (part, community) and choose the next sets: every
//     community larger than s_post when a part has several, the whole part when it has one.
// The label-propagation CDA runs on the parts' compacted induced subgraphs (the WCC
// front end's cluster-major arena): per round, the neighbours' labels of every row are
// sorted (two stable radix sorts: by label, then by row) and each row takes its longest
// run, the smallest label on ties.
#include "wcc_internal.h"

namespace {

constexpr int CB = 256;
inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ---------------------------------------------------------------- sets of a level
// keys: the set label (N for vertices in no set, so they sort last); vals: the vertex id
__global__ void k_cm_keys(const int32_t *cur, int64_t N, uint32_t *keys, uint32_t *vals, int32_t *nv) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  int32_t c = cur[v];
  keys[v] = c >= 0 ? (uint32_t)c : (uint32_t)N;
  vals[v] = (uint32_t)v;
  if (c >= 0) atomicAdd(nv, 1);
}

// flag[i] = 1 where a new set starts in the sorted order (i < nv)
__global__ void k_cm_flags(const uint32_t *keys, const int32_t *nv, int32_t *flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int n = *nv;
  if (i >= n) return;
  flag[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1 : 0;
}

// set index of every sorted position; set starts; the vertex lists; caps k(n) per set;
// set of every vertex
__global__ void k_cm_sets(const uint32_t *vals, const int32_t *flag, const int32_t *fscan, const int32_t *nv,
                          int64_t *set_off, int32_t *verts, int32_t *setidx, int32_t *setof) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int n = *nv;
  if (i >= n) return;
  int32_t s = fscan[i] + flag[i] - 1;
  int32_t v = (int32_t)vals[i];
  setidx[i] = s;
  verts[i] = v;
  setof[v] = s;
  if (flag[i]) set_off[s] = i;
  if (i == n - 1) set_off[s + 1] = n;
}

__global__ void k_cm_caps(const int64_t *set_off, const int32_t *nsets, int32_t crit, int32_t lin_num,
                          int32_t lin_den, int32_t *caps, int32_t *has_edge, int32_t *ssize,
                          unsigned long long *shash, int32_t *psize, int32_t *pmin) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *nsets) return;
  int64_t n = set_off[s + 1] - set_off[s];
  int64_t k = wcc_k_of(crit, n, lin_num, lin_den);
  caps[s] = (int32_t)(k < 0x7fffffff ? k : 0x7fffffff);
  has_edge[s] = 0;
  ssize[s] = 0;
  shash[s] = 0;
  psize[2 * s] = psize[2 * s + 1] = 0;
  pmin[2 * s] = pmin[2 * s + 1] = 0x7fffffff;
}

// has_edge[s] = 1 when some vertex of set s has a neighbour in s (Alg. 5 tests only sets
// with at least one edge).  One thread per set member; a row stops at its first hit.
template <typename OT>
__global__ void k_cm_edges(const OT *off, const int32_t *idx, const int32_t *verts, const int32_t *setidx,
                           const int32_t *setof, const int32_t *nv, int32_t *has_edge) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *nv) return;
  int32_t v = verts[i], s = setidx[i];
  if (has_edge[s]) return;
  for (int64_t e = (int64_t)off[v]; e < (int64_t)off[v + 1]; e++) {
    int32_t u = idx[e];
    if (setof[u] == s) {
      has_edge[s] = 1;
      return;
    }
  }
}

// ---------------------------------------------------------------- outcome of the cuts
// per member: side sizes, part minima, |S| and the hash of S (sets with an edge only)
__global__ void k_cm_outcome_a(const int32_t *verts, const int32_t *setidx, const uint8_t *sides, const int32_t *nv,
                               const int32_t *has_edge, int32_t *ssize, unsigned long long *shash, int32_t *psize,
                               int32_t *pmin) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *nv) return;
  int32_t s = setidx[i];
  if (!has_edge[s]) return;
  int32_t v = verts[i];
  int sd = sides[i] ? 1 : 0;
  atomicAdd(&psize[2 * s + sd], 1);
  atomicMin(&pmin[2 * s + sd], v);
  if (sd) {
    atomicAdd(&ssize[s], 1);
    atomicAdd(&shash[s], (unsigned long long)vhash(v));
  }
}

// per set with an edge: one split record; counts of cuts and saved sets
__global__ void k_cm_outcome_b(const int64_t *set_off, const int32_t *verts, const int32_t *nsets,
                               const int32_t *has_edge, const int32_t *caps, const int32_t *lam,
                               const int32_t *ssize, const unsigned long long *shash, wcc_record *rec,
                               int64_t rec_cap, unsigned long long *cnt) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= *nsets || !has_edge[s]) return;
  atomicAdd(&cnt[CNT_MINCUTS], 1ull);
  if (lam[s] >= caps[s]) atomicAdd(&cnt[CNT_ACCEPTED], 1ull);
  unsigned long long r = atomicAdd(&cnt[CNT_RECORDS], 1ull);
  if (rec && (long long)r < rec_cap) {
    wcc_record rc;
    rc.minv = verts[set_off[s]];
    rc.n = (int32_t)(set_off[s + 1] - set_off[s]);
    rc.k = caps[s];
    rc.lambda = lam[s];
    rc.ssize = ssize[s];
    rc.reserved = 0;
    rc.shash = shash[s];
    rec[r] = rc;
  }
}

// per member: saved sets go to acc (their smallest vertex); members of a failing set get
// their part (the smallest vertex of their side) when the part is larger than s_post
__global__ void k_cm_outcome_c(const int64_t *set_off, const int32_t *verts, const int32_t *setidx,
                               const uint8_t *sides, const int32_t *nv, const int32_t *has_edge, const int32_t *caps,
                               const int32_t *lam, const int32_t *psize, const int32_t *pmin, int32_t s_post,
                               int32_t *acc, int32_t *part_of, int32_t *nparts) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *nv) return;
  int32_t s = setidx[i], v = verts[i];
  if (!has_edge[s]) return;
  if (lam[s] >= caps[s]) {
    acc[v] = verts[set_off[s]];
    return;
  }
  int sd = sides[i] ? 1 : 0;
  if (psize[2 * s + sd] > s_post) {
    part_of[v] = pmin[2 * s + sd];
    if (v == pmin[2 * s + sd]) atomicAdd(nparts, 1);
  }
}

// ---------------------------------------------------------------- next sets
// The vertices in a part as a list in ascending id (slot = rank among part members, from
// an exclusive scan of the membership flags): keys = community, vals = vertex.  The stable
// sorts that follow rely on the ascending order.
__global__ void k_cm_comm_keys(const int32_t *part_of, const int32_t *comm, int64_t N, const int32_t *rank,
                               uint32_t *keys, uint32_t *vals) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < N && part_of[v] >= 0) {
    int32_t slot = rank[v];
    keys[slot] = (uint32_t)comm[v];
    vals[slot] = (uint32_t)v;
  }
}

__global__ void k_cm_in_part(const int32_t *part_of, int64_t N, int32_t *flag) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < N) flag[v] = part_of[v] >= 0 ? 1 : 0;
}

// after sorting by community, then stably by part: keys2[i] = part of the i-th vertex
__global__ void k_cm_part_keys(const uint32_t *vals, const int32_t *part_of, const int32_t *np, uint32_t *keys) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *np) return;
  keys[i] = (uint32_t)part_of[vals[i]];
}

// runs of equal (part, community) in the sorted order: the first member of a run is the
// community's smallest vertex; count communities per part and record each run's start
__global__ void k_cm_runs(const uint32_t *vals, const int32_t *np, const int32_t *part_of, const int32_t *comm,
                          int32_t *ncomm, int32_t *run_flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int n = *np;
  if (i >= n) return;
  int32_t v = (int32_t)vals[i];
  bool start = i == 0;
  if (!start) {
    int32_t u = (int32_t)vals[i - 1];
    start = part_of[u] != part_of[v] || comm[u] != comm[v];
  }
  run_flag[i] = start ? 1 : 0;
  if (start) atomicAdd(&ncomm[part_of[v]], 1);
}

// run index of every sorted position (scan of run_flag) -> run start and size
__global__ void k_cm_run_bounds(const int32_t *run_flag, const int32_t *run_scan, const int32_t *np,
                                int32_t *run_start, int32_t *run_size) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int n = *np;
  if (i >= n) return;
  int32_t r = run_scan[i] + run_flag[i] - 1;
  if (run_flag[i]) run_start[r] = (int32_t)i;
  atomicAdd(&run_size[r], 1);
}

// next sets: the part itself when it has one community, else each community larger than
// s_post (labelled by its smallest vertex)
__global__ void k_cm_next(const uint32_t *vals, const int32_t *run_flag, const int32_t *run_scan,
                          const int32_t *run_start, const int32_t *run_size, const int32_t *np,
                          const int32_t *part_of, const int32_t *ncomm, int32_t s_post, int32_t *cur) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *np) return;
  int32_t v = (int32_t)vals[i];
  int32_t p = part_of[v];
  if (ncomm[p] <= 1) {
    cur[v] = p;
    return;
  }
  int32_t r = run_scan[i] + run_flag[i] - 1;
  cur[v] = run_size[r] > s_post ? (int32_t)vals[run_start[r]] : -1;
}

// ---------------------------------------------------------------- CCR sizes (Alg. 4 step 1)
__global__ void k_cm_count(const int32_t *lab, int64_t N, int32_t *cnt) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < N && lab[v] >= 0) atomicAdd(&cnt[lab[v]], 1);
}
__global__ void k_cm_gate(const int32_t *lab, const int32_t *cnt, int64_t N, int32_t gate, int32_t *cur) {
  int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  int32_t l = lab[v];
  cur[v] = (l >= 0 && cnt[l] > gate) ? l : -1;
}

// ---------------------------------------------------------------- label propagation
// Per entry of the parts' arena: its row (position) and its neighbour's position.
__global__ void k_lp_entries(const int64_t *rs0, const int32_t *rd0, const int32_t *vtx0, const int32_t *cidv,
                             const int64_t *cl_start, const int32_t *adj0, const int64_t *na_p, int32_t *erow,
                             int32_t *enb) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *na_p) return;
  int64_t base = cl_start[cidv[vtx0[p]]];
  int64_t e0 = rs0[p];
  int32_t d = rd0[p];
  for (int32_t j = 0; j < d; j++) {
    erow[e0 + j] = (int32_t)p;
    enb[e0 + j] = (int32_t)(base + adj0[e0 + j]);
  }
}

__global__ void k_lp_init(const int32_t *vtx0, const int64_t *na_p, int32_t *lab) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < *na_p) lab[p] = vtx0[p];
}

// keys: the neighbour's label, vals: the row
__global__ void k_lp_keys(const int32_t *erow, const int32_t *enb, const int32_t *lab, const int64_t *E_p,
                          uint32_t *keys, uint32_t *vals) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= *E_p) return;
  keys[e] = (uint32_t)lab[enb[e]];
  vals[e] = (uint32_t)erow[e];
}

// after the label sort: keys become the rows (sorted stably next), vals the labels
__global__ void k_lp_swap(const uint32_t *k_in, const uint32_t *v_in, const int64_t *E_p, uint32_t *k_out,
                          uint32_t *v_out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= *E_p) return;
  k_out[e] = v_in[e];
  v_out[e] = k_in[e];
}

// Every row's neighbour labels are now ascending in [rs0[p], rs0[p] + rd0[p]): the
// longest run wins, the first (smallest) label on ties; a row without entries keeps its
// label.
__global__ void k_lp_mode(const int64_t *rs0, const int32_t *rd0, const uint32_t *sorted_lab, const int64_t *na_p,
                          const int32_t *lab, int32_t *lab_new) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *na_p) return;
  int32_t d = rd0[p];
  if (d == 0) {
    lab_new[p] = lab[p];
    return;
  }
  const uint32_t *L = sorted_lab + rs0[p];
  uint32_t best = L[0], cur = L[0];
  int32_t best_len = 0, len = 0;
  for (int32_t j = 0; j < d; j++) {
    uint32_t x = L[j];
    if (x == cur) {
      len++;
    } else {
      cur = x;
      len = 1;
    }
    if (len > best_len) {
      best_len = len;
      best = cur;
    }
  }
  lab_new[p] = (int32_t)best;
}

__global__ void k_lp_out(const int32_t *vtx0, const int32_t *lab, const int64_t *na_p, int32_t *comm) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < *na_p) comm[vtx0[p]] = lab[p];
}

}  // namespace

// ---------------------------------------------------------------- host launchers
#define LAUNCH(kern, n, ...)                                                      \
  do {                                                                          \
    if ((n) > 0) hipLaunchKernelGGL(kern, dim3(nblk((n), CB)), dim3(CB), 0, s, __VA_ARGS__); \
    HIP_TRY(hipGetLastError());                                                 \
  } while (0)

int cm_set_keys(const int32_t *cur, int64_t N, uint32_t *keys, uint32_t *vals, int32_t *nv, hipStream_t s) {
  LAUNCH(k_cm_keys, N, cur, N, keys, vals, nv);
  return WCC_OK;
}
int cm_sets(const uint32_t *skeys, const uint32_t *svals, int64_t cap, const int32_t *nv, int32_t *flag,
            int32_t *fscan, int32_t *nsets, int64_t *set_off, int32_t *verts, int32_t *setidx, int32_t *setof,
            void *tmp, size_t tmp_bytes, hipStream_t s) {
  LAUNCH(k_cm_flags, cap, skeys, nv, flag);
  int rc = prim_excl_scan_i32(flag, fscan, cap, nsets, tmp, tmp_bytes, s);
  if (rc) return rc;
  LAUNCH(k_cm_sets, cap, svals, flag, fscan, nv, set_off, verts, setidx, setof);
  return WCC_OK;
}
int cm_caps(const int64_t *set_off, const int32_t *nsets, int64_t cap, const wcc_params &p, int32_t *caps,
            int32_t *has_edge, int32_t *ssize, unsigned long long *shash, int32_t *psize, int32_t *pmin,
            hipStream_t s) {
  LAUNCH(k_cm_caps, cap, set_off, nsets, p.criterion, p.lin_num, p.lin_den, caps, has_edge, ssize, shash, psize,
         pmin);
  return WCC_OK;
}
int cm_edges(const wcc_csr *g, const int32_t *verts, const int32_t *setidx, const int32_t *setof,
             const int32_t *nv, int64_t cap, int32_t *has_edge, hipStream_t s) {
  if (g->offset_bits == 32)
    LAUNCH(k_cm_edges<int32_t>, cap, (const int32_t *)g->row_offsets, g->col_indices, verts, setidx, setof, nv,
           has_edge);
  else
    LAUNCH(k_cm_edges<int64_t>, cap, (const int64_t *)g->row_offsets, g->col_indices, verts, setidx, setof, nv,
           has_edge);
  return WCC_OK;
}
int cm_outcome(const int64_t *set_off, const int32_t *verts, const int32_t *setidx, const uint8_t *sides,
               const int32_t *nv, const int32_t *nsets, int64_t cap, const int32_t *has_edge, const int32_t *caps,
               const int32_t *lam, int32_t *ssize, unsigned long long *shash, int32_t *psize, int32_t *pmin,
               int32_t s_post, int32_t *acc, int32_t *part_of, int32_t *nparts, wcc_record *rec, int64_t rec_cap,
               unsigned long long *cnt, hipStream_t s) {
  LAUNCH(k_cm_outcome_a, cap, verts, setidx, sides, nv, has_edge, ssize, shash, psize, pmin);
  LAUNCH(k_cm_outcome_b, cap, set_off, verts, nsets, has_edge, caps, lam, ssize, shash, rec, rec_cap, cnt);
  LAUNCH(k_cm_outcome_c, cap, set_off, verts, setidx, sides, nv, has_edge, caps, lam, psize, pmin, s_post, acc,
         part_of, nparts);
  return WCC_OK;
}
// np = number of vertices in a part; fscan = their ranks
int cm_part_count(const int32_t *part_of, int64_t N, int32_t *flag, int32_t *fscan, int32_t *np, void *tmp,
                  size_t tmp_bytes, hipStream_t s) {
  LAUNCH(k_cm_in_part, N, part_of, N, flag);
  return prim_excl_scan_i32(flag, fscan, N, np, tmp, tmp_bytes, s);
}

// Next sets from the parts (part_of) and their communities (comm, labels below 2^comm_bits).
// ncomm (N) and run_size (np_host) must be zero on entry.
int cm_next(const int32_t *part_of, const int32_t *comm, int64_t N, int32_t s_post, int comm_bits, int32_t *cur,
            const int32_t *fscan, const int32_t *np, int np_host, uint32_t *k1, uint32_t *v1, uint32_t *k2,
            uint32_t *v2, int32_t *ncomm, int32_t *run_flag, int32_t *run_scan, int32_t *run_start,
            int32_t *run_size, int32_t *nruns, void *tmp, size_t tmp_bytes, hipStream_t s) {
  int rc;
  if (np_host <= 0) return WCC_OK;
  LAUNCH(k_cm_comm_keys, N, part_of, comm, N, fscan, k1, v1);
  int bits = 1;
  while (bits < 31 && (1LL << bits) < N) bits++;
  int alt = 0;
  if ((rc = prim_radix_sort_pairs(k1, v1, k2, v2, np_host, comm_bits, tmp, tmp_bytes, s, &alt))) return rc;
  uint32_t *sv = alt ? v2 : v1;             // vertices sorted by community
  uint32_t *pk = alt ? k1 : k2;             // free key buffer
  uint32_t *pv = alt ? v1 : v2;             // free value buffer
  LAUNCH(k_cm_part_keys, np_host, sv, part_of, np, pk);
  // stable sort of (part, vertex) pairs keeps the community order inside a part
  HIP_TRY(hipMemcpyAsync(pv, sv, (size_t)np_host * 4, hipMemcpyDeviceToDevice, s));
  uint32_t *ok = alt ? k2 : k1;             // the other free pair
  uint32_t *ov = sv;
  int alt2 = 0;
  if ((rc = prim_radix_sort_pairs(pk, pv, ok, ov, np_host, bits, tmp, tmp_bytes, s, &alt2))) return rc;
  const uint32_t *fin = alt2 ? ov : pv;     // vertices sorted by (part, community)
  LAUNCH(k_cm_runs, np_host, fin, np, part_of, comm, ncomm, run_flag);
  if ((rc = prim_excl_scan_i32(run_flag, run_scan, np_host, nruns, tmp, tmp_bytes, s))) return rc;
  LAUNCH(k_cm_run_bounds, np_host, run_flag, run_scan, np, run_start, run_size);
  LAUNCH(k_cm_next, np_host, fin, run_flag, run_scan, run_start, run_size, np, part_of, ncomm, s_post, cur);
  return WCC_OK;
}
int cm_ccr_gate(const int32_t *comp, int64_t N, int32_t gate, int32_t *cnt, int32_t *cur, hipStream_t s) {
  int rc = prim_fill32(cnt, 0u, N, s);
  if (rc) return rc;
  LAUNCH(k_cm_count, N, comp, N, cnt);
  LAUNCH(k_cm_gate, N, comp, cnt, N, gate, cur);
  return WCC_OK;
}

int lp_prepare(const int64_t *rs0, const int32_t *rd0, const int32_t *vtx0, const int32_t *cidv,
               const int64_t *cl_start, const int32_t *adj0, const int64_t *na_p, int64_t na_cap, int32_t *erow,
               int32_t *enb, int32_t *lab, hipStream_t s) {
  LAUNCH(k_lp_entries, na_cap, rs0, rd0, vtx0, cidv, cl_start, adj0, na_p, erow, enb);
  LAUNCH(k_lp_init, na_cap, vtx0, na_p, lab);
  return WCC_OK;
}
int lp_round(const int64_t *rs0, const int32_t *rd0, const int32_t *erow, const int32_t *enb, const int64_t *na_p,
             int64_t na_cap, const int64_t *E_p, int64_t E_host, int bits, int32_t *lab, int32_t *lab_new,
             uint32_t *k1, uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes, hipStream_t s) {
  int rc;
  LAUNCH(k_lp_keys, E_host, erow, enb, lab, E_p, k1, v1);
  int alt = 0;
  if (E_host > 0 && (rc = prim_radix_sort_pairs(k1, v1, k2, v2, E_host, bits, tmp, tmp_bytes, s, &alt))) return rc;
  uint32_t *sk = alt ? k2 : k1, *sv = alt ? v2 : v1;
  uint32_t *ok = alt ? k1 : k2, *ov = alt ? v1 : v2;
  LAUNCH(k_lp_swap, E_host, sk, sv, E_p, ok, ov);  // keys: rows, vals: labels
  int alt2 = 0;
  if (E_host > 0 && (rc = prim_radix_sort_pairs(ok, ov, sk, sv, E_host, bits, tmp, tmp_bytes, s, &alt2))) return rc;
  const uint32_t *lab_sorted = alt2 ? sv : ov;
  LAUNCH(k_lp_mode, na_cap, rs0, rd0, lab_sorted, na_p, lab, lab_new);
  return WCC_OK;
}
int lp_out(const int32_t *vtx0, const int32_t *lab, const int64_t *na_p, int64_t na_cap, int32_t *comm,
           hipStream_t s) {
  LAUNCH(k_lp_out, na_cap, vtx0, lab, na_p, comm);
  return WCC_OK;
}
