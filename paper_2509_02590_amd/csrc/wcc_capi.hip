// wcc_capi.hip -- C ABI (include/wcc.h) and host drivers of the gfx950 WCC path.
//
// Plain driver (level-synchronous): front end (validate, group, compaction), then one
// item launch per recursion depth.  Items of a depth are disjoint, so every launch reads
// one arena and writes the children into the other; the host only learns how many
// children there are between launches.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <string>
#include <vector>

#include "wcc_internal.h"

namespace {

// ---------------------------------------------------------------- workspace
// Bumped whenever any workspace buffer moves: a recorded launch sequence (HIP graph)
// holds raw buffer addresses and is only replayed while this value is unchanged.
std::atomic<unsigned long long> g_alloc_gen{1};

// A fixed device region that buffers are carved from in call order (the allocation-free
// entry point): a buffer that must grow takes a new slice, nothing is ever freed, and the
// carve restarts at the next call.
struct Carver {
  char *base = nullptr;
  size_t size = 0, used = 0;
};

struct Buf {
  void *p = nullptr;
  size_t bytes = 0;
  Carver *carve = nullptr;
  int ensure(size_t b) {
    if (b <= bytes) return WCC_OK;
    if (carve) {
      size_t off = (carve->used + 255) & ~(size_t)255;
      if (off > carve->size || b > carve->size - off) return WCC_ENOMEM;
      p = carve->base + off;
      bytes = b;
      carve->used = off + b;
      return WCC_OK;
    }
    g_alloc_gen++;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    size_t nb = b + b / 8 + 256;
    if (hipMalloc(&p, nb) != hipSuccess) {
      (void)hipGetLastError();
      return WCC_ENOMEM;
    }
    bytes = nb;
    return WCC_OK;
  }
  void release() {
    if (p && !carve) {
      g_alloc_gen++;
      (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
  }
  template <typename T>
  T *as() const {
    return (T *)p;
  }
};

enum BufId {
  B_KEYS, B_VALS, B_KEYS2, B_VALS2, B_FLAG, B_FLAGSCAN, B_CIDV, B_POSV, B_DEGIN,
  B_ACC, B_MARK, B_RANK, B_TMP, B_DCNT, B_CLSTART, B_CLIDS,
  B_VTX0, B_VTX1, B_RS0, B_RS1, B_RD0, B_RD1, B_ADJ0, B_ADJ1,
  B_SA, B_SB, B_SC, B_SD, B_SE, B_SF, B_SG, B_SEDGE, B_SMARK, B_GBITS,
  B_ITEMS0, B_ITEMS1, B_ITEMS_SORTED, B_SET0, B_SET_SORTED, B_IKEYS, B_IVALS, B_IKEYS2, B_IVALS2,
  B_SPLITMEM, B_SMALL, B_LVCTL, B_LB0, B_LB1, B_LBS,
  // Connectivity Modifier: per vertex, per set, per run, and label propagation per entry
  B_CM_CUR, B_CM_PART, B_CM_COMM, B_CM_ACC, B_CM_SETOF, B_CM_VERTS, B_CM_SETIDX, B_CM_FLAG, B_CM_FSCAN,
  B_CM_K1, B_CM_V1, B_CM_K2, B_CM_V2, B_CM_NCOMM, B_CM_SO, B_CM_CAPS, B_CM_HASE, B_CM_SSZ, B_CM_SHASH,
  B_CM_LAM, B_CM_PSZ, B_CM_PMIN, B_CM_SIDES, B_CM_RUNF, B_CM_RUNS, B_CM_RUNSTART, B_CM_RUNSIZE, B_CM_CTL,
  B_CM_TMP, B_LP_EROW, B_LP_ENB, B_LP_LAB, B_LP_LAB2, B_LP_K1, B_LP_V1, B_LP_K2, B_LP_V2, B_LP_TMP,
  B_NUM
};

// Launch shape of the item kernels: the size-bin boundary follows from the small-bin LDS
// budget (an item goes to the large bin when its scan state does not fit it).
struct ExecCfg : wcc_exec_config {
  ExecCfg() {
    small_lds_kb = 32;
    wg_per_cu = 0;
    big_lds_kb = 159;
    big_max_pct = 100;
    chain_min_n = -1;
  }
};
bool cfg_valid(const wcc_exec_config &c) {
  return c.small_lds_kb >= 4 && c.small_lds_kb <= 64 && c.wg_per_cu >= 0 && c.wg_per_cu <= 8 &&
         c.big_lds_kb >= c.small_lds_kb && c.big_lds_kb <= 159 && c.big_max_pct >= 0 && c.big_max_pct <= 100 &&
         c.chain_min_n >= -1;
}

// Identity of a recorded batched run: replayed only for the same buffers and parameters.
struct GraphKey {
  const void *off, *idx, *mem, *out, *rec;
  int64_t N, nnz, rec_cap;
  int32_t obits, pad;
  wcc_params p;
  wcc_exec_config cfg;
};

// Sizes a batched run was planned with (host side).
struct BatchPlan {
  int32_t nitems = 0, nbig = 0, top_n = 0;
  int64_t small_words = 0;
  size_t lds_bytes = 0, big_bytes = 0;
  int g_big = 0, g_small = 0;
  int64_t gbits_words = 0;
  int64_t capS = 0, capB = 0;  // list capacities (items)
  int32_t chain_min_n = 0x7fffffff;  // chained form: least child size kept by its workgroup
  int levels = 0;              // levels launched (a multiple of the chunk size)
};

constexpr int LEVEL_CHUNK = 4;  // levels launched between two looks at the remaining work
constexpr int MAX_TIMED_LEVELS = 64;
struct Workspace {
  Buf b[B_NUM];
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evj = nullptr, evf = nullptr, evg = nullptr;
  hipEvent_t evb0 = nullptr, evb1 = nullptr, evs0 = nullptr, evs1 = nullptr;  // per-launch timing
  hipEvent_t lev[MAX_TIMED_LEVELS][4] = {};  // batched form: per-level launch timing
  hipStream_t s2 = nullptr;  // second stream (default priority) for the large-item launch
  hipStream_t sg = nullptr;  // stream the recorded batched run is captured on and replayed on
  int cus = 0;
  int dev = 0;
  double tick_khz = 100000.0;  // device wall clock
  ExecCfg cfg;
  hipGraphExec_t gexec = nullptr;
  GraphKey gkey;
  GraphKey last_key;  // key of the previous eager batched call (recorded when seen twice)
  bool last_valid = false;
  unsigned long long ggen = 0;
  BatchPlan gplan;
  bool gtimed = false;  // the recorded sequence carries the per-launch timing events
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  }
  void release() {
    drop_graph();
    for (auto &x : b) x.release();
  }
  int64_t bytes() const {
    int64_t t = 0;
    for (auto &x : b) t += (int64_t)x.bytes;
    return t;
  }
  // streams and events (the served form creates and destroys whole workspaces)
  void destroy() {
    release();
    for (hipEvent_t e : {ev0, ev1, evj, evf, evg, evb0, evb1, evs0, evs1})
      if (e) (void)hipEventDestroy(e);
    for (auto &l : lev)
      for (auto &e : l)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : {s2, sg})
      if (st) (void)hipStreamDestroy(st);
  }
};

std::mutex g_lock;

// device FrontCounts live in the counter block, after the 128 words used by the drivers
FrontCounts *front_counts(Workspace &w) { return (FrontCounts *)(w.b[B_DCNT].as<unsigned long long>() + 128); }
std::vector<Workspace *> g_ws;

int env_int(const char *name, int dflt);

int ws_init(Workspace &w, int dev, const hipDeviceProp_t &prop) {
  w.dev = dev;
  w.cus = prop.multiProcessorCount;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
    w.tick_khz = khz;
  HIP_TRY(hipEventCreate(&w.ev0));
  HIP_TRY(hipEventCreate(&w.ev1));
  HIP_TRY(hipEventCreateWithFlags(&w.evj, hipEventDisableTiming));
  for (hipEvent_t *e : {&w.evb0, &w.evb1, &w.evs0, &w.evs1}) HIP_TRY(hipEventCreate(e));
  for (auto &l : w.lev)
    for (auto &e : l) HIP_TRY(hipEventCreate(&e));
  HIP_TRY(hipEventCreateWithFlags(&w.evf, hipEventDisableTiming));
  HIP_TRY(hipEventCreateWithFlags(&w.evg, hipEventDisableTiming));
  HIP_TRY(hipStreamCreateWithFlags(&w.s2, hipStreamNonBlocking));
  HIP_TRY(hipStreamCreateWithFlags(&w.sg, hipStreamNonBlocking));
  w.cfg.small_lds_kb = env_int("WCC_LDS_KB", w.cfg.small_lds_kb);
  w.cfg.big_lds_kb = env_int("WCC_BIG_LDS_KB", w.cfg.big_lds_kb);
  w.cfg.wg_per_cu = env_int("WCC_WG_PER_CU", w.cfg.wg_per_cu);
  w.cfg.big_max_pct = env_int("WCC_BIG_PCT", w.cfg.big_max_pct);
  w.cfg.chain_min_n = env_int("WCC_CHAIN_MIN", w.cfg.chain_min_n);
  return WCC_OK;
}

int get_ws(Workspace **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1, nullptr);
  if (!g_ws[dev]) {
    Workspace *w = new Workspace();
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    int rc = ws_init(*w, dev, prop);
    if (rc) {
      delete w;
      return rc;
    }
    g_ws[dev] = w;
  }
  *out = g_ws[dev];
  return WCC_OK;
}

#define TRY(x)                \
  do {                        \
    int _r = (x);             \
    if (_r != WCC_OK) return _r; \
  } while (0)

int env_int(const char *name, int dflt) {
  const char *v = getenv(name);
  if (!v || !*v) return dflt;
  return atoi(v);
}

int check_params(const wcc_params &p) {
  if (p.criterion < WCC_CRIT_LOG10 || p.criterion > WCC_CRIT_LINEAR) return WCC_EINVAL;
  if (p.criterion == WCC_CRIT_LINEAR && (p.lin_den < 1 || p.lin_num < 0)) return WCC_EINVAL;
  if (p.s_pre < 0 || p.s_post < 0) return WCC_EINVAL;
  if (p.prune_mode != WCC_PRUNE_PAPER && p.prune_mode != WCC_PRUNE_KCORE) return WCC_EINVAL;
  if (p.mincut_rule != 1) return WCC_EINVAL;
  if (p.exec_mode != WCC_EXEC_PLAIN && p.exec_mode != WCC_EXEC_BATCHED) return WCC_EINVAL;
  return WCC_OK;
}

int check_csr(const wcc_csr *g) {
  if (!g) return WCC_EINVAL;
  if (g->num_vertices < 0 || g->num_entries < 0) return WCC_EINVAL;
  if (g->offset_bits != 32 && g->offset_bits != 64) return WCC_EINVAL;
  if (g->num_vertices > 0 && !g->row_offsets) return WCC_EINVAL;
  if (g->num_entries > 0 && !g->col_indices) return WCC_EINVAL;
  if (g->num_vertices >= (1LL << 31) - 1) return WCC_EUNSUPPORTED;
  if (g->offset_bits == 32 && g->num_entries >= (1LL << 31)) return WCC_EINVAL;
  return WCC_OK;
}

// Front end shared by every entry point.  Buffers are sized for the worst case (every
// vertex assigned, every entry intra-cluster), so no size has to be read back before the
// compaction; the sizes it produced stay on the device in FrontCounts.
int ensure_items(Workspace &w, int64_t cap, bool with_sets);

int run_front(Workspace &w, const wcc_csr *g, const int32_t *mem, bool want_ids, bool all_items,
              hipStream_t s) {
  int64_t N = g->num_vertices;
  size_t n4 = (size_t)(N > 0 ? N : 1) * 4;
  for (int id : {B_KEYS, B_VALS, B_KEYS2, B_VALS2, B_FLAG, B_FLAGSCAN, B_CIDV, B_POSV, B_DEGIN,
                 B_ACC, B_MARK, B_RANK, B_VTX0, B_VTX1, B_RD0, B_RD1, B_SA, B_SB, B_SC, B_SD, B_SE, B_SF,
                 B_SG})
    TRY(w.b[id].ensure(n4));
  TRY(w.b[B_RS0].ensure(2 * n4 + 8));
  TRY(w.b[B_RS1].ensure(2 * n4 + 8));
  TRY(w.b[B_CLSTART].ensure(2 * n4 + 16));
  TRY(w.b[B_CLIDS].ensure(n4));
  size_t tmpb = prim_radix_tmp_bytes(N > 0 ? N : 1);
  size_t sb = prim_scan_tmp_bytes(N > 0 ? N : 1);
  TRY(w.b[B_TMP].ensure(tmpb > sb ? tmpb : sb));
  TRY(w.b[B_DCNT].ensure(256 * sizeof(unsigned long long)));
  size_t e4 = (size_t)(g->num_entries > 0 ? g->num_entries : 1) * 4;
  TRY(w.b[B_ADJ0].ensure(e4));
  TRY(w.b[B_ADJ1].ensure(e4));
  TRY(w.b[B_SEDGE].ensure(e4));
  TRY(w.b[B_SMARK].ensure(e4 / 4 + 64));
  TRY(ensure_items(w, N + 1, all_items));

  FrontBufs f;
  f.off = g->row_offsets;
  f.obits = g->offset_bits;
  f.idx = g->col_indices;
  f.mem = mem;
  f.N = N;
  f.nnz = g->num_entries;
  f.keys = w.b[B_KEYS].as<uint32_t>();
  f.vals = w.b[B_VALS].as<uint32_t>();
  f.keys2 = w.b[B_KEYS2].as<uint32_t>();
  f.vals2 = w.b[B_VALS2].as<uint32_t>();
  f.flag = w.b[B_FLAG].as<int32_t>();
  f.flag_scan = w.b[B_FLAGSCAN].as<int32_t>();
  f.cidv = w.b[B_CIDV].as<int32_t>();
  f.posv = w.b[B_POSV].as<int32_t>();
  f.deg_in = w.b[B_DEGIN].as<int32_t>();
  f.stage = w.b[B_ADJ1].as<int32_t>();
  f.tmp = w.b[B_TMP].p;
  f.tmp_bytes = w.b[B_TMP].bytes;
  f.dcnt = w.b[B_DCNT].as<unsigned long long>();
  f.dmax = (int32_t *)(f.dcnt + 8);
  if (w.b[B_DCNT].bytes == 0) return WCC_EINVAL;
  return front_build(f, front_counts(w), w.b[B_VTX0].as<int32_t>(), w.b[B_CLSTART].as<int64_t>(),
                     want_ids ? w.b[B_CLIDS].as<int32_t>() : nullptr, w.b[B_RD0].as<int32_t>(),
                     w.b[B_RS0].as<int64_t>(), w.b[B_ADJ0].as<int32_t>(), w.b[B_ITEMS0].as<ItemDesc>(),
                     all_items ? w.b[B_SET0].as<int32_t>() : nullptr, all_items, s);
}

// CSR checks only (symmetric, simple, ids in range): WCC_EGRAPH when malformed.
int run_validate(Workspace &w, const wcc_csr *g, hipStream_t s) {
  TRY(w.b[B_DCNT].ensure(256 * sizeof(unsigned long long)));
  // the duplicate tables borrow the second arena and the crossing-list scratch (sized as
  // the front end sizes them anyway)
  size_t e4 = (size_t)(g->num_entries > 0 ? g->num_entries : 1) * 4;
  TRY(w.b[B_ADJ1].ensure(e4));
  TRY(w.b[B_SEDGE].ensure(e4));
  FrontBufs f;
  memset(&f, 0, sizeof(f));
  f.off = g->row_offsets;
  f.obits = g->offset_bits;
  f.idx = g->col_indices;
  f.N = g->num_vertices;
  f.nnz = g->num_entries;
  f.dcnt = w.b[B_DCNT].as<unsigned long long>();
  f.vtab_a = w.b[B_ADJ1].as<int32_t>();
  f.vtab_b = w.b[B_SEDGE].as<int32_t>();
  int ok = 1;
  TRY(front_validate(f, s, &ok));
  return ok ? WCC_OK : WCC_EGRAPH;
}

int read_counts(Workspace &w, FrontCounts *h, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(h, front_counts(w), sizeof(FrontCounts), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return WCC_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Smallest n whose scan state can exceed `words` 32-bit LDS words: an item of n vertices
// has at most n(n-1) list entries, and its cut cap is k(n) of the criterion (WCC) or any
// caller's cap (mincut_split).  Items of one level are disjoint, so at most N / that many
// of them are large.
int min_big_n(int64_t words, const wcc_params &p, bool split) {
  int64_t lo = 1, hi = 1 << 24;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    int64_t cap = split ? (int64_t)INT32_MAX : wcc_k_of(p.criterion, mid, p.lin_num, p.lin_den);
    if (item_state_words(mid, mid * (mid - 1), cap) > words) hi = mid;
    else lo = mid + 1;
  }
  return (int)lo;
}

// Device words of a level's sort: [0] large-item count, [2..3] largest bitmap (64-bit)
int32_t *sort_sizes(Workspace &w) { return (int32_t *)(w.b[B_DCNT].as<unsigned long long>() + 20); }

SortNeed sort_need(const wcc_params &p, const ItemArgs &base, int64_t small_words) {
  SortNeed nd;
  nd.crit = p.criterion;
  nd.lin_num = p.lin_num;
  nd.lin_den = p.lin_den;
  nd.caps = base.split_only ? base.split_cap : nullptr;
  nd.set = nullptr;
  nd.small_words = small_words;
  return nd;
}

struct SortSizes {
  int32_t nbig, pad;
  int64_t maxbits;
};

// Processes item lists level by level until no children remain.  Each level is sorted
// by size (largest first) and split into two launches that run concurrently: the items
// whose state does not fit the small LDS budget go to a workgroup per CU with the full
// 160 KB of LDS on a second stream, the rest to many small-LDS workgroups.
struct Shape {
  size_t lds_bytes, big_bytes;
  int per_cu;
  int big_max;  // batched form: most CUs given to large-bin workgroups
};
int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
Shape exec_shape(const Workspace &w) {
  Shape sh;
  int lds_kb = clampi(w.cfg.small_lds_kb, 4, 64);
  int big_kb = clampi(w.cfg.big_lds_kb, lds_kb, 159);
  int fit = 160 / lds_kb;
  int per_cu = w.cfg.wg_per_cu > 0 ? w.cfg.wg_per_cu : (fit > 8 ? 8 : fit);
  sh.per_cu = clampi(per_cu, 1, fit < 8 ? fit : 8);
  sh.lds_bytes = (size_t)lds_kb * 1024;
  sh.big_bytes = (size_t)big_kb * 1024;
  // 0 turns the large-bin launch of the batched form off (large items then run from
  // global memory in small-bin workgroups)
  sh.big_max = w.cfg.big_max_pct <= 0 ? 0 : clampi(w.cus * clampi(w.cfg.big_max_pct, 1, 100) / 100, 1, w.cus);
  return sh;
}

void print_phases(const unsigned long long *ph);

int run_levels(Workspace &w, ItemArgs base, int32_t nitems0, int max_cap_crit, const wcc_params &p,
               int64_t *levels, double *ms_kernel, int64_t *launches, hipStream_t s) {
  Shape shp = exec_shape(w);
  size_t lds_bytes = shp.lds_bytes;
  size_t big_bytes = shp.big_bytes;
  int per_cu = shp.per_cu;
  int gmax = w.cus * per_cu;
  int32_t nitems = nitems0;
  int cur = 0;  // items in B_ITEMS0 (cur==0) or B_ITEMS1
  int32_t *dcount = (int32_t *)(w.b[B_DCNT].as<unsigned long long>() + 16);
  int32_t *dnext = dcount + 1;
  int32_t *dnext_big = dcount + 2;
  int32_t *dsz = sort_sizes(w);
  ItemDesc *sorted = w.b[B_ITEMS_SORTED].as<ItemDesc>();
  int32_t *set_sorted = base.split_only ? w.b[B_SET_SORTED].as<int32_t>() : nullptr;
  const int32_t *set_in = base.split_only ? w.b[B_SET0].as<int32_t>() : nullptr;
  SortNeed nd = sort_need(p, base, (int64_t)(lds_bytes / 4));
  (void)max_cap_crit;
  *levels = 0;
  *ms_kernel = 0;
  *launches = 0;
  while (nitems > 0) {
    ItemDesc *in = w.b[cur ? B_ITEMS1 : B_ITEMS0].as<ItemDesc>();
    ItemDesc *out = w.b[cur ? B_ITEMS0 : B_ITEMS1].as<ItemDesc>();
    TRY(items_sort_desc(in, nitems, sorted, set_in, set_sorted, w.b[B_IKEYS].as<uint32_t>(),
                        w.b[B_IVALS].as<uint32_t>(), w.b[B_IKEYS2].as<uint32_t>(), w.b[B_IVALS2].as<uint32_t>(),
                        w.b[B_TMP].p, w.b[B_TMP].bytes, s, nd, dsz));
    ItemDesc top;
    SortSizes hs;
    HIP_TRY(hipMemcpyAsync(&top, sorted, sizeof(top), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hs, dsz, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t nbig = hs.nbig;
    int32_t nsmall = nitems - nbig;
    int grid_small = nsmall < gmax ? nsmall : gmax;
    int grid_big = nbig < w.cus ? nbig : w.cus;
    // bitmap regions of the large-bin workgroups (small-bin items keep their state in LDS)
    int64_t words = hs.maxbits > 0 ? hs.maxbits : 1;
    Carver *cv = w.b[B_GBITS].carve;
    if (cv && grid_big > 1) {
      // a fixed region: fewer large-bin workgroups (each loops over the large items)
      size_t left = cv->size > cv->used + 512 ? cv->size - cv->used - 512 : 0;
      int64_t fit = (int64_t)(left / ((size_t)words * 8 + 64));
      if (fit < grid_big) grid_big = fit > 1 ? (int)fit : 1;
    }
    TRY(w.b[B_GBITS].ensure((size_t)(grid_big > 0 ? grid_big : 1) * words * 8 + 64));
    ItemArgs A = base;
    A.gbits = w.b[B_GBITS].as<uint64_t>();
    A.gbits_words = words;
    A.out = out;
    A.out_count = dcount;
    if (base.split_only) A.split_set = set_sorted;
    TRY(prim_fill32(dcount, 0u, 3, s));
    // the large bin goes first on the caller's stream: its workgroups each need a whole
    // CU's LDS and would otherwise wait for small-bin workgroups to drain; the small bin
    // follows on the second stream
    HIP_TRY(hipEventRecord(w.evf, s));
    if (nbig > 0) {
      ItemArgs Bg = A;
      Bg.items = sorted;
      Bg.nitems = nbig;
      Bg.next = dnext_big;
      Bg.lds_words = (int32_t)(big_bytes / 4);
      if (base.prof == 3) Bg.prof = 2;  // profile: the largest item of each level only
      if (base.prof == 4) Bg.prof = 0;  // profile: the small-bin items only
      HIP_TRY(hipEventRecord(w.evb0, s));
      TRY(items_launch(Bg, grid_big, big_bytes, s));
      HIP_TRY(hipEventRecord(w.evb1, s));
    }
    if (nsmall > 0) {
      ItemArgs Sm = A;
      Sm.items = sorted + nbig;
      Sm.nitems = nsmall;
      Sm.next = dnext;
      Sm.lds_words = (int32_t)(lds_bytes / 4);
      Sm.gbits_words = 0;  // (small-bin items keep their scan state in LDS)
      if (base.split_only) Sm.split_set = set_sorted + nbig;
      if (base.prof == 3) Sm.prof = nbig > 0 ? 0 : 2;
      if (base.prof == 4) Sm.prof = 1;
      HIP_TRY(hipStreamWaitEvent(w.s2, w.evf, 0));
      HIP_TRY(hipEventRecord(w.evs0, w.s2));
      TRY(items_launch(Sm, grid_small, lds_bytes, w.s2));
      HIP_TRY(hipEventRecord(w.evs1, w.s2));
      HIP_TRY(hipEventRecord(w.evj, w.s2));
      HIP_TRY(hipStreamWaitEvent(s, w.evj, 0));
    }
    int32_t nout = 0;
    HIP_TRY(hipMemcpyAsync(&nout, dcount, sizeof(nout), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    float ms_b = 0, ms_s = 0;
    if (nbig > 0) {
      HIP_TRY(hipEventElapsedTime(&ms_b, w.evb0, w.evb1));
      *ms_kernel += ms_b;
      (*launches)++;
    }
    if (nsmall > 0) {
      HIP_TRY(hipEventElapsedTime(&ms_s, w.evs0, w.evs1));
      *ms_kernel += ms_s;
      (*launches)++;
    }
    (*levels)++;
    if (env_int("WCC_VERBOSE", 0)) {
      fprintf(stderr, "[wcc] level %lld: %d items (%d large, largest n=%d m=%lld) -> %d children; large bin "
              "%.2f ms, small bin %.2f ms\n", (long long)*levels, nitems, nbig, top.n, (long long)top.m, nout, ms_b,
              ms_s);
      if (base.prof) {
        // this level's phase totals, then cleared for the next level
        unsigned long long ph[CNT_PH_END - CNT_PH];
        HIP_TRY(hipMemcpyAsync(ph, base.cnt + CNT_PH, sizeof(ph), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        print_phases(ph);
        TRY(prim_fill32((uint32_t *)(base.cnt + CNT_PH), 0u, 2 * (CNT_PH_END - CNT_PH), s));
      }
    }
    if (nout > A.out_cap) return WCC_ENOMEM;
    long long errc = 0;
    HIP_TRY(hipMemcpyAsync(&errc, base.cnt + CNT_ERR, sizeof(errc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (errc < 0) return (int)errc;
    if (base.split_only) break;  // sets are not split further
    nitems = nout;
    cur ^= 1;
  }
  return WCC_OK;
}

// ---------------------------------------------------------------- batched form
// Device-driven levels: every recursion depth is one launch per size bin whose item
// count is read on the device, children go straight into the next level's small or
// large list, and the host does not synchronise inside a run, so the whole run can be
// recorded as one HIP graph.  Lists of parity p: small = B_ITEMS<p>, large = B_LB<p>.

ItemDesc *list_small(Workspace &w, int p) { return w.b[p ? B_ITEMS1 : B_ITEMS0].as<ItemDesc>(); }
ItemDesc *list_big(Workspace &w, int p) { return w.b[p ? B_LB1 : B_LB0].as<ItemDesc>(); }
int32_t *level_ctl(Workspace &w) { return w.b[B_LVCTL].as<int32_t>(); }

// Plans a batched run: sorts the initial items (largest first), reads back how many need
// the large LDS budget and the largest size, and sizes grids, lists and bitmap regions.
int plan_batched(Workspace &w, const wcc_params &p, int64_t N, int32_t nitems, BatchPlan *pl, hipStream_t s) {
  Shape shp = exec_shape(w);
  pl->nitems = nitems;
  pl->lds_bytes = shp.lds_bytes;
  pl->big_bytes = shp.big_bytes;
  pl->small_words = (int64_t)(shp.lds_bytes / 4);
  int32_t *dsz = sort_sizes(w);
  ItemDesc *sorted = w.b[B_ITEMS_SORTED].as<ItemDesc>();
  pl->nbig = 0;
  pl->top_n = 0;
  int64_t maxbits = 1;
  if (nitems > 0) {
    ItemArgs none;
    memset(&none, 0, sizeof(none));
    TRY(items_sort_desc(w.b[B_ITEMS0].as<ItemDesc>(), nitems, sorted, nullptr, nullptr,
                        w.b[B_IKEYS].as<uint32_t>(), w.b[B_IVALS].as<uint32_t>(), w.b[B_IKEYS2].as<uint32_t>(),
                        w.b[B_IVALS2].as<uint32_t>(), w.b[B_TMP].p, w.b[B_TMP].bytes, s,
                        sort_need(p, none, pl->small_words), dsz));
    ItemDesc top;
    SortSizes hs;
    HIP_TRY(hipMemcpyAsync(&top, sorted, sizeof(top), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hs, dsz, sizeof(hs), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    pl->top_n = top.n;
    pl->nbig = hs.nbig;
    maxbits = hs.maxbits > 0 ? hs.maxbits : 1;
  }
  // Both bins are launched oversubscribed, as in the plain form: a workgroup leaves as soon
  // as its list is empty, so CUs freed by one bin go to the other.  Large-bin workgroups:
  // one per initial large item, at most the configured share of the CUs; with no
  // large-bin launch every item stays in the small lists (large ones then run from
  // global memory in small-bin workgroups).
  int cap_big = shp.big_max;
  pl->g_big = pl->nbig < cap_big ? pl->nbig : cap_big;
  if (pl->g_big == 0) pl->nbig = 0;
  pl->g_small = w.cus * shp.per_cu;
  // chained form: with few large items per large-bin workgroup the level time is one long
  // chain of splits, which chaining shortens; with many, chaining only holds back the
  // children left for the next level
  pl->chain_min_n = w.cfg.chain_min_n >= 0 ? w.cfg.chain_min_n
                    : (pl->nbig <= 4 * (int64_t)(pl->g_big > 0 ? pl->g_big : 1) ? 0 : 0x7fffffff);
  // (the bitmap bound of the initial items covers their descendants: smaller sets with
  // caps no larger)
  pl->gbits_words = maxbits;
  pl->capS = N + 1;
  pl->capB = N / min_big_n(pl->small_words, p, false) + 1;
  TRY(w.b[B_LVCTL].ensure((size_t)items_level_words() * 4));
  TRY(w.b[B_LB0].ensure((size_t)pl->capB * sizeof(ItemDesc)));
  TRY(w.b[B_LB1].ensure((size_t)pl->capB * sizeof(ItemDesc)));
  TRY(w.b[B_LBS].ensure((size_t)pl->capB * sizeof(ItemDesc)));
  // global-state items run in large-bin workgroups only (children whose state exceeds the
  // small-bin LDS go to the large lists), unless there is no large-bin launch
  TRY(w.b[B_GBITS].ensure((size_t)(pl->g_big > 0 ? pl->g_big : pl->g_small) * pl->gbits_words * 8 + 64));
  return WCC_OK;
}

// Level 0 input: the sorted initial items split into the parity-0 lists.  guard: the
// device checks its sizes against the plan (a recorded sequence replayed on new data).
int route_level0(Workspace &w, const ItemArgs &base, const BatchPlan &pl, bool sort, bool guard, hipStream_t s) {
  int32_t *dnbig = sort_sizes(w);
  ItemDesc *sorted = w.b[B_ITEMS_SORTED].as<ItemDesc>();
  if (sort && pl.nitems > 0) {
    wcc_params p;
    wcc_default_params(&p);
    p.criterion = base.crit;
    p.lin_num = base.lin_num;
    p.lin_den = base.lin_den;
    TRY(items_sort_desc(w.b[B_ITEMS0].as<ItemDesc>(), pl.nitems, sorted, nullptr, nullptr,
                        w.b[B_IKEYS].as<uint32_t>(), w.b[B_IVALS].as<uint32_t>(), w.b[B_IKEYS2].as<uint32_t>(),
                        w.b[B_IVALS2].as<uint32_t>(), w.b[B_TMP].p, w.b[B_TMP].bytes, s,
                        sort_need(p, base, pl.small_words), dnbig));
  }
  if (pl.g_big == 0 && pl.nitems > 0) TRY(prim_fill32(dnbig, 0u, 1, s));  // everything small
  return items_route0(sorted, pl.nitems, dnbig, front_counts(w), guard ? pl.nitems : -1, pl.nbig, pl.top_n,
                      list_small(w, 0), list_big(w, 0), level_ctl(w), base.cnt, s);
}

// Launches levels [L0, L1): per level, the large list on the second stream and the small
// list on s, both writing the children into the lists of the other parity.
int launch_levels(Workspace &w, const ItemArgs &base, const BatchPlan &pl, int L0, int L1, bool timed,
                  hipStream_t s) {
  int32_t *ctl = level_ctl(w);
  uint64_t *gb = w.b[B_GBITS].as<uint64_t>();
  for (int L = L0; L < L1; L++) {
    int cur = L & 1, nx = cur ^ 1;
    bool t = timed && L < MAX_TIMED_LEVELS;
    TRY(items_level_prep(ctl, nx, s));
    ItemArgs A = base;
    A.out = list_small(w, nx);
    A.out_count = ctl + 2 * nx;
    A.out_cap = (int32_t)pl.capS;
    A.out_big = pl.g_big > 0 ? list_big(w, nx) : nullptr;
    A.out_big_count = ctl + 2 * nx + 1;
    A.out_big_cap = (int32_t)pl.capB;
    A.small_words = pl.small_words;
    A.chain = 1;
    A.chain_min_n = pl.chain_min_n;
    A.gbits_words = pl.gbits_words;
    if (pl.g_big > 0) {
      // largest first (level 0 is sorted already) so that the longest items start at once;
      // worth its launches only when the large list can hold thousands of items
      ItemDesc *big_in = list_big(w, cur);
      if (L > 0 && pl.capB >= 4096) {
        TRY(items_sort_desc_dev(big_in, (int32_t)pl.capB, ctl + 2 * cur + 1, w.b[B_LBS].as<ItemDesc>(),
                                w.b[B_IKEYS].as<uint32_t>(), w.b[B_IVALS].as<uint32_t>(),
                                w.b[B_IKEYS2].as<uint32_t>(), w.b[B_IVALS2].as<uint32_t>(), w.b[B_TMP].p,
                                w.b[B_TMP].bytes, s));
        big_in = w.b[B_LBS].as<ItemDesc>();
      }
      // large bin first on s, small bin on the second stream (see run_levels)
      HIP_TRY(hipEventRecord(w.evf, s));
      ItemArgs Bg = A;
      Bg.items = big_in;
      Bg.nitems_dev = ctl + 2 * cur + 1;
      Bg.nitems = (int32_t)pl.capB;
      Bg.next = ctl + items_level_words() - 1;
      Bg.lds_words = (int32_t)(pl.big_bytes / 4);
      Bg.gbits = gb;
      if (t) HIP_TRY(hipEventRecord(w.lev[L][0], s));
      TRY(items_launch(Bg, pl.g_big, pl.big_bytes, s));
      if (t) HIP_TRY(hipEventRecord(w.lev[L][1], s));
    }
    ItemArgs Sm = A;
    Sm.items = list_small(w, cur);
    Sm.nitems_dev = ctl + 2 * cur;
    Sm.nitems = (int32_t)pl.capS;
    Sm.next = ctl + items_level_words() - 2;
    Sm.lds_words = (int32_t)(pl.lds_bytes / 4);
    Sm.gbits = gb;
    if (pl.g_big > 0) Sm.gbits_words = 0;  // (small-bin items keep their scan state in LDS)
    hipStream_t ss = pl.g_big > 0 ? w.s2 : s;
    if (pl.g_big > 0) HIP_TRY(hipStreamWaitEvent(w.s2, w.evf, 0));
    if (t) HIP_TRY(hipEventRecord(w.lev[L][2], ss));
    TRY(items_launch(Sm, pl.g_small, pl.lds_bytes, ss));
    if (t) HIP_TRY(hipEventRecord(w.lev[L][3], ss));
    if (pl.g_big > 0) {
      HIP_TRY(hipEventRecord(w.evj, w.s2));
      HIP_TRY(hipStreamWaitEvent(s, w.evj, 0));
    }
  }
  return WCC_OK;
}

// Items left in the input lists of level L (after the stream has been synchronised).
int level_pending(Workspace &w, int L, int64_t *left, hipStream_t s) {
  int32_t c[2];
  HIP_TRY(hipMemcpyAsync(c, level_ctl(w) + 2 * (L & 1), sizeof(c), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *left = (int64_t)c[0] + c[1];
  return WCC_OK;
}

// Runs levels in chunks until a level's input is empty; *L is the next level index.
int finish_levels(Workspace &w, const ItemArgs &base, BatchPlan &pl, int *L, bool timed, hipStream_t s) {
  for (;;) {
    int64_t left = 0;
    TRY(level_pending(w, *L, &left, s));
    unsigned long long errc = 0;
    HIP_TRY(hipMemcpyAsync(&errc, base.cnt + CNT_ERR, sizeof(errc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if ((long long)errc < 0) return (int)(long long)errc;
    if (env_int("WCC_VERBOSE", 0))
      fprintf(stderr, "[wcc] batched: %lld items left after %d levels\n", (long long)left, *L);
    if (left == 0) return WCC_OK;
    TRY(launch_levels(w, base, pl, *L, *L + LEVEL_CHUNK, timed, s));
    *L += LEVEL_CHUNK;
  }
}

// Summed durations and count of the item launches of levels [0, L) (after completion).
// Timing is informative: if an event cannot be read, 0 launches are reported.
int levels_kernel_ms(Workspace &w, const BatchPlan &pl, int L, double *ms, int64_t *launches) {
  double tot = 0;
  int64_t n = 0;
  bool verbose = env_int("WCC_VERBOSE", 0) != 0;
  for (int l = 0; l < L && l < MAX_TIMED_LEVELS; l++) {
    float a = 0, b = 0;
    if (pl.g_big > 0) {
      if (hipEventElapsedTime(&a, w.lev[l][0], w.lev[l][1]) != hipSuccess) goto fail;
      tot += a;
      n++;
    }
    if (hipEventElapsedTime(&b, w.lev[l][2], w.lev[l][3]) != hipSuccess) goto fail;
    tot += b;
    n++;
    if (verbose) fprintf(stderr, "[wcc] batched level %d: large bin %.2f ms, small bin %.2f ms\n", l + 1, a, b);
  }
  *ms = tot;
  *launches = n;
  return WCC_OK;
fail:
  (void)hipGetLastError();
  *ms = 0;
  *launches = 0;
  return WCC_OK;
}

ItemArgs base_args(Workspace &w, const wcc_params &p, int32_t item_cap) {
  ItemArgs A;
  memset(&A, 0, sizeof(A));
  A.ar[0].vtx = w.b[B_VTX0].as<int32_t>();
  A.ar[0].rs = w.b[B_RS0].as<int64_t>();
  A.ar[0].rd = w.b[B_RD0].as<int32_t>();
  A.ar[0].adj = w.b[B_ADJ0].as<int32_t>();
  A.ar[1].vtx = w.b[B_VTX1].as<int32_t>();
  A.ar[1].rs = w.b[B_RS1].as<int64_t>();
  A.ar[1].rd = w.b[B_RD1].as<int32_t>();
  A.ar[1].adj = w.b[B_ADJ1].as<int32_t>();
  A.sA = w.b[B_SA].as<int32_t>();
  A.sB = w.b[B_SB].as<int32_t>();
  A.sC = w.b[B_SC].as<int32_t>();
  A.sD = w.b[B_SD].as<int32_t>();
  A.sE = w.b[B_SE].as<int32_t>();
  A.sF = w.b[B_SF].as<int32_t>();
  A.sG = w.b[B_SG].as<int32_t>();
  A.sMark = w.b[B_SMARK].as<uint8_t>();
  A.sEdge = w.b[B_SEDGE].as<int32_t>();
  A.acc = w.b[B_ACC].as<int32_t>();
  A.out_cap = item_cap;
  A.crit = p.criterion;
  A.lin_num = p.lin_num;
  A.lin_den = p.lin_den;
  A.s_pre = p.s_pre;
  A.s_post = p.s_post;
  A.mode = p.prune_mode;
  A.leaf_batch = p.prune_mode == WCC_PRUNE_PAPER && wcc_k_of(p.criterion, (int64_t)p.s_post + 1, p.lin_num,
                                                              p.lin_den) >= 2;
  A.low_runs = p.prune_mode == WCC_PRUNE_PAPER;
  A.cnt = w.b[B_DCNT].as<unsigned long long>() + 32;
  return A;
}

int ensure_items(Workspace &w, int64_t cap, bool with_sets) {
  size_t ib = (size_t)(cap > 0 ? cap : 1) * sizeof(ItemDesc);
  TRY(w.b[B_ITEMS0].ensure(ib));
  TRY(w.b[B_ITEMS1].ensure(ib));
  TRY(w.b[B_ITEMS_SORTED].ensure(ib));
  size_t i4 = (size_t)(cap > 0 ? cap : 1) * 4;
  for (int id : {B_IKEYS, B_IVALS, B_IKEYS2, B_IVALS2}) TRY(w.b[id].ensure(i4));
  if (with_sets) {
    TRY(w.b[B_SET0].ensure(i4));
    TRY(w.b[B_SET_SORTED].ensure(i4));
  }
  return WCC_OK;
}

// Prints the per-phase clock totals (CNT_PH slots; the wall clock runs at 100 MHz).
void print_phases(const unsigned long long *ph) {
  static const char *names[] = {"ccr-cc", "peel", "prune-children", "cut-setup", "scan", "contract",
                                "lists", "degree", "record", "split-rebuild", "steps", "certified", "rounds"};
  fprintf(stderr, "[wcc phase ms, summed over workgroups]");
  for (int i = 0; i < 13; i++)
    fprintf(stderr, " %s=%.2f", names[i], i >= 10 ? (double)ph[i] : ph[i] / 1e5);
  fprintf(stderr, "\n[wcc cc ms] sample=%.2f compress=%.2f pick=%.2f; certificate: sample=%.2f compress=%.2f pass=%.2f\n",
          ph[16] / 1e5, ph[17] / 1e5, ph[18] / 1e5, ph[19] / 1e5, ph[20] / 1e5, ph[21] / 1e5);
  fprintf(stderr, "[wcc sub-phases ms] forest=%.2f unions=%.2f finds=%.2f relabel=%.2f lists-count=%.2f "
          "lists-scan=%.2f lists-fill=%.2f cc-unite=%.2f cc-roots=%.2f rebuild-head=%.2f "
          "rebuild-degrees=%.2f rebuild-offsets=%.2f rebuild-fill=%.2f\n",
          ph[22] / 1e5, ph[23] / 1e5, ph[24] / 1e5, ph[25] / 1e5, ph[26] / 1e5, ph[27] / 1e5, ph[28] / 1e5,
          ph[29] / 1e5, ph[30] / 1e5, ph[31] / 1e5, ph[13] / 1e5, ph[15] / 1e5, ph[14] / 1e5);
}

// Reads the device counters of a finished run into stats (and the record count).
int collect_counts(Workspace &w, wcc_stats *st, int64_t *nrec, bool prof, hipStream_t s) {
  unsigned long long hc[CNT_NUM];
  FrontCounts fc;
  unsigned long long *cnt = w.b[B_DCNT].as<unsigned long long>() + 32;
  HIP_TRY(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&fc, front_counts(w), sizeof(fc), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if ((long long)hc[CNT_ERR] < 0) return (int)(long long)hc[CNT_ERR];
  st->clusters = fc.K;
  st->intra_entries = fc.E;
  st->items = (int64_t)hc[CNT_ITEMS];
  st->mincuts = (int64_t)hc[CNT_MINCUTS];
  st->accepted = (int64_t)hc[CNT_ACCEPTED];
  st->scan_steps = (int64_t)hc[CNT_STEPS];
  st->scan_rounds = (int64_t)hc[CNT_ROUNDS];
  st->item_alg_bytes = (int64_t)hc[CNT_ALG_BYTES];
  if (nrec) *nrec = (int64_t)hc[CNT_RECORDS];
  if (prof) print_phases(hc + CNT_PH);
  return WCC_OK;
}

GraphKey make_key(Workspace &w, const wcc_csr *g, const int32_t *mem_in, const wcc_params &p, int32_t *out,
                  wcc_record *rec, int64_t rec_cap) {
  GraphKey k;
  memset(&k, 0, sizeof(k));
  k.off = g->row_offsets;
  k.idx = g->col_indices;
  k.mem = mem_in;
  k.out = out;
  k.rec = rec;
  k.N = g->num_vertices;
  k.nnz = g->num_entries;
  k.rec_cap = rec_cap;
  k.obits = g->offset_bits;
  k.p = p;
  k.p.flags &= ~WCC_FLAG_VALIDATE;  // validation runs outside the recorded sequence
  k.cfg = w.cfg;
  return k;
}

// The whole batched run after validation, all on stream s with no host synchronisation:
// front end, resets, sort, guarded routing, pl.levels levels, relabel.
int batched_sequence(Workspace &w, const wcc_csr *g, const int32_t *mem_in, const ItemArgs &A,
                     const BatchPlan &pl, int32_t *out, bool timed, hipStream_t s) {
  int64_t N = g->num_vertices;
  TRY(run_front(w, g, mem_in, false, false, s));
  TRY(prim_fill32(w.b[B_ACC].p, 0xffffffffu, N, s));
  TRY(prim_fill32(A.cnt, 0u, 2 * CNT_NUM, s));
  TRY(route_level0(w, A, pl, true, true, s));
  TRY(launch_levels(w, A, pl, 0, pl.levels, timed, s));
  TRY(items_relabel(w.b[B_ACC].as<int32_t>(), N, w.b[B_MARK].as<int32_t>(), w.b[B_RANK].as<int32_t>(), out,
                    w.b[B_TMP].p, w.b[B_TMP].bytes, s));
  return WCC_OK;
}

// Records batched_sequence as a HIP graph on the workspace's own stream (with the
// per-launch timing events when the runtime records them, else without).
int capture_batched(Workspace &w, const wcc_csr *g, const int32_t *mem_in, const ItemArgs &A,
                    const BatchPlan &pl, int32_t *out, const GraphKey &key) {
  w.drop_graph();
  unsigned long long gen0 = g_alloc_gen.load();
  for (int timed = 1; timed >= 0; timed--) {
    HIP_TRY(hipStreamBeginCapture(w.sg, hipStreamCaptureModeRelaxed));
    int rc = batched_sequence(w, g, mem_in, A, pl, out, timed != 0, w.sg);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(w.sg, &graph);
    if (rc != WCC_OK || e != hipSuccess || !graph || g_alloc_gen.load() != gen0) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      if (rc != WCC_OK && rc != WCC_EHIP) return rc;
      continue;
    }
    e = hipGraphInstantiate(&w.gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      w.gexec = nullptr;
      (void)hipGetLastError();
      continue;
    }
    w.gkey = key;
    w.ggen = gen0;
    w.gplan = pl;
    w.gtimed = timed != 0;
    return WCC_OK;
  }
  return WCC_EHIP;
}

int wcc_run_impl(Workspace &w, const wcc_csr *g, const int32_t *mem_in, const wcc_params *pp, int32_t *out,
                 wcc_stats *stats, wcc_record *rec, int64_t rec_cap, int64_t *nrec, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  wcc_params p;
  if (pp) p = *pp;
  else wcc_default_params(&p);
  TRY(check_params(p));
  TRY(check_csr(g));
  if (g->num_vertices > 0 && (!mem_in || !out)) return WCC_EINVAL;
  if (rec_cap < 0 || (rec_cap > 0 && !rec)) return WCC_EINVAL;
  int64_t N = g->num_vertices;
  wcc_stats st;
  memset(&st, 0, sizeof(st));
  if (nrec) *nrec = 0;
  if (N == 0) {
    if (stats) *stats = st;
    return WCC_OK;
  }
  bool validate = (p.flags & WCC_FLAG_VALIDATE) != 0;
  bool batched = p.exec_mode == WCC_EXEC_BATCHED;
  int prof = env_int("WCC_PROF", 0);
  bool use_graph = batched && !(p.flags & WCC_FLAG_NO_GRAPH) && env_int("WCC_GRAPH", 1) != 0 && prof == 0;
  GraphKey key = make_key(w, g, mem_in, p, out, rec, rec_cap);

  if (use_graph && w.gexec && w.ggen == g_alloc_gen.load() && memcmp(&key, &w.gkey, sizeof(key)) == 0) {
    // replay of the recorded batched run
    if (validate) TRY(run_validate(w, g, s));
    HIP_TRY(hipEventRecord(w.evf, s));
    HIP_TRY(hipStreamWaitEvent(w.sg, w.evf, 0));
    auto t1 = std::chrono::steady_clock::now();
    HIP_TRY(hipGraphLaunch(w.gexec, w.sg));
    HIP_TRY(hipEventRecord(w.evg, w.sg));
    HIP_TRY(hipStreamWaitEvent(s, w.evg, 0));
    BatchPlan pl = w.gplan;
    int L = pl.levels;
    unsigned long long errc = 0;
    HIP_TRY(hipMemcpyAsync(&errc, w.b[B_DCNT].as<unsigned long long>() + 32 + CNT_ERR, sizeof(errc),
                           hipMemcpyDeviceToHost, s));
    int64_t left = 0;
    TRY(level_pending(w, L, &left, s));
    if ((long long)errc == WCC_ECANCELLED) {
      // the device-side sizes differ from the recorded ones: run eagerly, record again
      w.drop_graph();
    } else {
      ItemArgs A = base_args(w, p, (int32_t)(N + 1));
      A.rec = rec;
      A.rec_cap = rec_cap;
      if (left > 0) {
        // deeper recursion than recorded: finish eagerly, then relabel again
        TRY(finish_levels(w, A, pl, &L, false, s));
        TRY(items_relabel(w.b[B_ACC].as<int32_t>(), N, w.b[B_MARK].as<int32_t>(), w.b[B_RANK].as<int32_t>(),
                          out, w.b[B_TMP].p, w.b[B_TMP].bytes, s));
      }
      TRY(collect_counts(w, &st, nrec, false, s));
      st.ms_items = ms_since(t1);
      st.levels = L;
      if (w.gtimed && left == 0) TRY(levels_kernel_ms(w, pl, L, &st.ms_item_kernel, &st.item_launches));
      st.graph_replays = 1;
      st.ms_total = ms_since(t0);
      if (stats) *stats = st;
      return WCC_OK;
    }
  }

  HIP_TRY(hipEventRecord(w.ev0, s));
  if (validate) TRY(run_validate(w, g, s));
  TRY(run_front(w, g, mem_in, false, false, s));
  HIP_TRY(hipEventRecord(w.ev1, s));
  // (the counter block exists once run_front has sized the workspace)
  unsigned long long *cnt = w.b[B_DCNT].as<unsigned long long>() + 32;
  TRY(prim_fill32(w.b[B_ACC].p, 0xffffffffu, N, s));
  TRY(prim_fill32(cnt, 0u, 2 * CNT_NUM, s));
  FrontCounts fc;
  TRY(read_counts(w, &fc, s));
  float fms = 0;
  HIP_TRY(hipEventElapsedTime(&fms, w.ev0, w.ev1));
  st.ms_front = fms;
  int32_t nitems = fc.nitems;
  ItemArgs A = base_args(w, p, (int32_t)(N + 1));
  A.rec = rec;
  A.rec_cap = rec_cap;
  A.prof = prof;
  auto t1 = std::chrono::steady_clock::now();
  BatchPlan pl;
  if (batched) {
    TRY(plan_batched(w, p, N, nitems, &pl, s));
    TRY(route_level0(w, A, pl, false, false, s));
    int L = 0;
    TRY(launch_levels(w, A, pl, 0, LEVEL_CHUNK, true, s));
    L = LEVEL_CHUNK;
    TRY(finish_levels(w, A, pl, &L, true, s));
    pl.levels = L;
    st.levels = L;
  } else {
    TRY(run_levels(w, A, nitems, p.criterion, p, &st.levels, &st.ms_item_kernel, &st.item_launches, s));
  }
  TRY(items_relabel(w.b[B_ACC].as<int32_t>(), N, w.b[B_MARK].as<int32_t>(), w.b[B_RANK].as<int32_t>(), out,
                    w.b[B_TMP].p, w.b[B_TMP].bytes, s));
  TRY(collect_counts(w, &st, nrec, prof != 0, s));
  if (batched) TRY(levels_kernel_ms(w, pl, pl.levels, &st.ms_item_kernel, &st.item_launches));
  st.ms_items = ms_since(t1);
  if (use_graph) {
    // record once the same call has been seen twice; a failed recording only means later
    // calls run eagerly too
    if (w.last_valid && memcmp(&key, &w.last_key, sizeof(key)) == 0) {
      HIP_TRY(hipStreamSynchronize(s));
      if (capture_batched(w, g, mem_in, A, pl, out, key) != WCC_OK) w.drop_graph();
    }
    w.last_key = key;
    w.last_valid = true;
  }
  st.ms_total = ms_since(t0);
  if (stats) *stats = st;
  return WCC_OK;
}

int split_batch_impl(const wcc_csr *g, const int32_t *verts, const int64_t *set_offsets, int32_t num_sets,
                     const int32_t *caps, int32_t *lambdas, uint8_t *sides, int64_t nv, hipStream_t s) {
  TRY(check_csr(g));
  if (num_sets < 0) return WCC_EINVAL;
  if (num_sets == 0) return WCC_OK;
  if (!set_offsets || !caps || !lambdas) return WCC_EINVAL;
  Workspace *wp;
  TRY(get_ws(&wp));
  Workspace &w = *wp;
  int64_t N = g->num_vertices;
  TRY(w.b[B_SPLITMEM].ensure((size_t)(N > 0 ? N : 1) * 4));
  TRY(w.b[B_DCNT].ensure(256 * sizeof(unsigned long long)));
  TRY(prim_fill32(lambdas, 0u, num_sets, s));
  if (nv == 0) {
    HIP_TRY(hipStreamSynchronize(s));
    return WCC_OK;
  }
  if (!verts || !sides) return WCC_EINVAL;
  TRY(prim_fill32(sides, 0u, nv / 4, s));
  if (nv % 4) HIP_TRY(hipMemcpyAsync(sides + (nv / 4) * 4, "\0\0\0", (size_t)(nv % 4), hipMemcpyHostToDevice, s));
  int32_t *mem = w.b[B_SPLITMEM].as<int32_t>();
  unsigned long long *bad = w.b[B_DCNT].as<unsigned long long>() + 100;
  TRY(front_split_membership(verts, set_offsets, num_sets, nv, N, mem, bad, s));
  unsigned long long hb = 0;
  HIP_TRY(hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (hb) return WCC_EINVAL;
  TRY(run_front(w, g, mem, true, true, s));
  FrontCounts fc;
  TRY(read_counts(w, &fc, s));
  wcc_params p;
  wcc_default_params(&p);
  ItemArgs A = base_args(w, p, (int32_t)(fc.K + 1));
  unsigned long long *cnt = w.b[B_DCNT].as<unsigned long long>() + 32;
  TRY(prim_fill32(cnt, 0u, 2 * CNT_NUM, s));
  A.split_only = 1;
  A.split_lambda = lambdas;
  A.split_side = sides;
  A.split_cap = caps;
  A.split_pos = set_offsets;
  int64_t lv;
  double ms;
  int64_t launches;
  TRY(run_levels(w, A, (int32_t)fc.K, WCC_CRIT_LOG10, p, &lv, &ms, &launches, s));
  HIP_TRY(hipStreamSynchronize(s));
  return WCC_OK;
}

// ---------------------------------------------------------------- autotuner
// Candidate shapes: every small-bin LDS budget (the size-bin boundary), the workgroups
// per CU that budget allows, and the large-bin CU share.
std::vector<ExecCfg> tune_candidates() {
  std::vector<ExecCfg> c;
  for (int kb : {8, 16, 24, 32, 48, 64}) {
    int fit = 160 / kb;
    for (int per : {0, 2, 4}) {
      if (per > fit || (per == 0 && fit <= 4 && kb != 32)) continue;
      for (int pct : {25, 50, 100}) {
        ExecCfg e;
        e.small_lds_kb = kb;
        e.wg_per_cu = per;
        e.big_max_pct = pct;
        c.push_back(e);
      }
    }
  }
  return c;
}

std::string tune_key(const Workspace &w, const wcc_csr *g, const wcc_params &p) {
  hipDeviceProp_t prop;
  char name[300] = "gpu";
  if (hipGetDeviceProperties(&prop, w.dev) == hipSuccess) snprintf(name, sizeof(name), "%s", prop.gcnArchName);
  for (char *c = name; *c; c++)
    if (*c == ' ' || *c == '|') *c = '_';
  char k[512];
  snprintf(k, sizeof(k), "%s|cus=%d|N=%lld|E=%lld|crit=%d/%d/%d|s=%d/%d|prune=%d", name, w.cus,
           (long long)g->num_vertices, (long long)g->num_entries, p.criterion, p.lin_num, p.lin_den, p.s_pre,
           p.s_post, p.prune_mode);
  return k;
}

bool tune_cache_lookup(const char *path, const std::string &key, ExecCfg *c) {
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    char k[600];
    int a, b, d, e, cm = c->chain_min_n;
    int got = sscanf(line, "%599s %d %d %d %d %d", k, &a, &b, &d, &e, &cm);
    if (got >= 5 && key == k) {
      c->small_lds_kb = a;
      c->wg_per_cu = b;
      c->big_lds_kb = d;
      c->big_max_pct = e;
      c->chain_min_n = cm;
      found = cfg_valid(*c);  // the last valid entry for the key wins
    }
  }
  fclose(f);
  return found;
}

int autotune_impl(const wcc_csr *g, const int32_t *mem_in, const wcc_params *pp, int reps, wcc_exec_config *best,
                  double *best_ms, int32_t *tried, hipStream_t s) {
  wcc_params p;
  if (pp) p = *pp;
  else wcc_default_params(&p);
  p.exec_mode = WCC_EXEC_BATCHED;
  p.flags |= WCC_FLAG_NO_GRAPH;
  p.flags &= ~WCC_FLAG_VALIDATE;
  TRY(check_params(p));
  TRY(check_csr(g));
  Workspace *wp;
  TRY(get_ws(&wp));
  Workspace &w = *wp;
  if (tried) *tried = 0;
  if (best_ms) *best_ms = 0;
  const char *cache = getenv("WCC_TUNE_CACHE");
  std::string key = tune_key(w, g, p);
  ExecCfg hit;
  if (cache && *cache && tune_cache_lookup(cache, key, &hit)) {
    w.cfg = hit;
    *best = hit;
    return WCC_OK;
  }
  int64_t N = g->num_vertices;
  int32_t *out = nullptr;
  if (N > 0 && hipMalloc((void **)&out, (size_t)N * 4) != hipSuccess) {
    (void)hipGetLastError();
    return WCC_ENOMEM;
  }
  ExecCfg keep = w.cfg, win = w.cfg;
  double win_ms = 1e300;
  int n = 0, rc = WCC_OK;
  for (const ExecCfg &c : tune_candidates()) {
    w.cfg = c;
    double t = 1e300;
    for (int r = 0; r < reps && rc == WCC_OK; r++) {
      wcc_stats st;
      rc = wcc_run_impl(w, g, mem_in, &p, out, &st, nullptr, 0, nullptr, s);
      if (rc == WCC_OK && st.ms_total < t) t = st.ms_total;
    }
    if (rc != WCC_OK) break;
    n++;
    if (t < win_ms) {
      win_ms = t;
      win = c;
    }
  }
  if (out) (void)hipFree(out);
  if (rc != WCC_OK) {
    w.cfg = keep;
    return rc;
  }
  w.cfg = win;
  *best = win;
  if (best_ms) *best_ms = win_ms;
  if (tried) *tried = n;
  if (cache && *cache) {
    FILE *f = fopen(cache, "a");
    if (f) {
      fprintf(f, "%s %d %d %d %d %d\n", key.c_str(), win.small_lds_kb, win.wg_per_cu, win.big_lds_kb, win.big_max_pct,
              win.chain_min_n);
      fclose(f);
    }
  }
  return WCC_OK;
}

// Workspace a job of N vertices and nnz entries grows to (the sizes run_front and the
// level driver ensure, with Buf's slack), for admission by HBM footprint.
int64_t est_workspace_bytes(int64_t N, int64_t nnz) {
  int64_t n1 = N + 1;
  int64_t b = 24 * 4 * N      // per-vertex int32 buffers of the front end and scratch
              + 3 * 8 * N     // rs0, rs1, cluster starts
              + 4 * N         // cluster ids
              + 3 * 32 * n1   // item lists and the sorted list
              + 4 * 4 * n1    // item sort keys / values
              + 3 * 4 * nnz   // two adjacency arenas and the crossing lists
              + nnz           // contraction marks
              + 2 * 8 * N     // radix / scan temporaries (upper bound)
              + (4 << 20);    // counters, large lists, bitmap regions (small)
  return b + b / 8 + 64 * 1024;
}

// CCR alone (Alg. 1): component labels of every cluster's induced subgraph.
int ccr_impl(const wcc_csr *g, const int32_t *mem, int32_t *out, hipStream_t s) {
  TRY(check_csr(g));
  int64_t N = g->num_vertices;
  if (N == 0) return WCC_OK;
  if (!mem || !out) return WCC_EINVAL;
  Workspace *wp;
  TRY(get_ws(&wp));
  Workspace &w = *wp;
  TRY(run_front(w, g, mem, false, false, s));
  TRY(items_ccr_init(mem, N, out, s));
  unsigned long long *cnt = w.b[B_DCNT].as<unsigned long long>() + 32;
  TRY(prim_fill32(cnt, 0u, 2 * CNT_NUM, s));
  FrontCounts fc;
  TRY(read_counts(w, &fc, s));
  wcc_params p;
  wcc_default_params(&p);
  ItemArgs A = base_args(w, p, (int32_t)(N + 1));
  A.ccr_out = out;
  int64_t lv = 0, launches = 0;
  double ms = 0;
  TRY(run_levels(w, A, fc.nitems, p.criterion, p, &lv, &ms, &launches, s));
  HIP_TRY(hipStreamSynchronize(s));
  return WCC_OK;
}

// ---------------------------------------------------------------- Connectivity Modifier
int bits_for(int64_t n) {
  int b = 1;
  while (b < 31 && (1LL << b) <= n) b++;
  return b;
}

// The label-propagation CDA on the parts given by part_of (labels: global vertex ids of
// the part's members): compaction of every part's induced subgraph, then `iters` rounds.
int lp_impl(Workspace &w, const wcc_csr *g, const int32_t *part_of, int32_t iters, int32_t *comm, hipStream_t s) {
  int64_t N = g->num_vertices;
  TRY(run_front(w, g, part_of, false, false, s));
  FrontCounts fc;
  TRY(read_counts(w, &fc, s));
  if (fc.na == 0) return WCC_OK;
  int64_t E = fc.E > 0 ? fc.E : 1, na = fc.na;
  for (int id : {B_LP_EROW, B_LP_ENB, B_LP_K1, B_LP_V1, B_LP_K2, B_LP_V2}) TRY(w.b[id].ensure((size_t)E * 4));
  TRY(w.b[B_LP_LAB].ensure((size_t)na * 4));
  TRY(w.b[B_LP_LAB2].ensure((size_t)na * 4));
  TRY(w.b[B_LP_TMP].ensure(prim_radix_tmp_bytes(E)));
  const FrontCounts *dfc = front_counts(w);
  const int64_t *na_p = &dfc->na;
  const int64_t *E_p = &dfc->E;
  int32_t *lab = w.b[B_LP_LAB].as<int32_t>(), *lab2 = w.b[B_LP_LAB2].as<int32_t>();
  TRY(lp_prepare(w.b[B_RS0].as<int64_t>(), w.b[B_RD0].as<int32_t>(), w.b[B_VTX0].as<int32_t>(),
                 w.b[B_CIDV].as<int32_t>(), w.b[B_CLSTART].as<int64_t>(), w.b[B_ADJ0].as<int32_t>(), na_p, na,
                 w.b[B_LP_EROW].as<int32_t>(), w.b[B_LP_ENB].as<int32_t>(), lab, s));
  int bits = bits_for(N);
  for (int t = 0; t < iters; t++) {
    TRY(lp_round(w.b[B_RS0].as<int64_t>(), w.b[B_RD0].as<int32_t>(), w.b[B_LP_EROW].as<int32_t>(),
                 w.b[B_LP_ENB].as<int32_t>(), na_p, na, E_p, fc.E, bits, lab, lab2, w.b[B_LP_K1].as<uint32_t>(),
                 w.b[B_LP_V1].as<uint32_t>(), w.b[B_LP_K2].as<uint32_t>(), w.b[B_LP_V2].as<uint32_t>(),
                 w.b[B_LP_TMP].p, w.b[B_LP_TMP].bytes, s));
    int32_t *t2 = lab;
    lab = lab2;
    lab2 = t2;
  }
  return lp_out(w.b[B_VTX0].as<int32_t>(), lab, na_p, na, comm, s);
}

// The CDA step of Alg. 5 on every part at once: comm[v] = community of v (-1 outside the
// parts).  *comm_bits receives the bit width of the labels.
int cda_impl(Workspace &w, const wcc_csr *g, const int32_t *part_of, const wcc_cm_params &cm, int32_t *comm,
             int *comm_bits, hipStream_t s) {
  int64_t N = g->num_vertices;
  TRY(prim_fill32(comm, 0xffffffffu, N, s));
  *comm_bits = bits_for(N);
  if (cm.cda == WCC_CDA_COMPONENTS) return ccr_impl(g, part_of, comm, s);
  if (cm.cda == WCC_CDA_LABELPROP) return lp_impl(w, g, part_of, cm.cda_iters, comm, s);
  // the caller's CDA: labels are any non-negative int32
  *comm_bits = 31;
  int rc = cm.fn(g, part_of, comm, cm.user, (void *)s);
  if (rc != WCC_OK) return rc < 0 ? rc : WCC_EINVAL;
  HIP_TRY(hipGetLastError());
  return WCC_OK;
}

int check_cm(const wcc_cm_params *cm) {
  if (!cm) return WCC_EINVAL;
  if (cm->cda == WCC_CDA_COMPONENTS) return WCC_OK;
  if (cm->cda == WCC_CDA_LABELPROP) return cm->cda_iters >= 0 && cm->cda_iters <= 1000 ? WCC_OK : WCC_EINVAL;
  if (cm->cda == WCC_CDA_CALLBACK) return cm->fn ? WCC_OK : WCC_EINVAL;
  return WCC_EINVAL;
}

// CM (Alg. 4) and its check CMC (Alg. 5), level by level: CCR, then per level one batched
// canonical cut of every current set, split records, saved sets, the two parts of every
// failing set, the CDA on all parts at once, and the next sets.
int cm_impl(const wcc_csr *g, const int32_t *mem_in, const wcc_params &p, const wcc_cm_params &cm, int32_t *out,
            wcc_stats *stats, wcc_record *rec, int64_t rec_cap, int64_t *nrec, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  TRY(check_params(p));
  TRY(check_csr(g));
  TRY(check_cm(&cm));
  if (rec_cap < 0 || (rec_cap > 0 && !rec)) return WCC_EINVAL;
  int64_t N = g->num_vertices;
  wcc_stats st;
  memset(&st, 0, sizeof(st));
  if (nrec) *nrec = 0;
  if (N == 0) {
    if (stats) *stats = st;
    return WCC_OK;
  }
  if (!mem_in || !out) return WCC_EINVAL;
  Workspace *wp;
  TRY(get_ws(&wp));
  Workspace &w = *wp;
  if (p.flags & WCC_FLAG_VALIDATE) TRY(run_validate(w, g, s));
  size_t n4 = (size_t)N * 4;
  for (int id : {B_CM_CUR, B_CM_PART, B_CM_COMM, B_CM_ACC, B_CM_SETOF, B_CM_VERTS, B_CM_SETIDX, B_CM_FLAG,
                 B_CM_FSCAN, B_CM_K1, B_CM_V1, B_CM_K2, B_CM_V2, B_CM_NCOMM, B_CM_CAPS, B_CM_HASE, B_CM_SSZ,
                 B_CM_LAM, B_CM_RUNF, B_CM_RUNS, B_CM_RUNSTART, B_CM_RUNSIZE})
    TRY(w.b[id].ensure(n4));
  TRY(w.b[B_CM_SO].ensure((size_t)(N + 1) * 8));
  TRY(w.b[B_CM_SHASH].ensure((size_t)N * 8));
  TRY(w.b[B_CM_PSZ].ensure(2 * n4));
  TRY(w.b[B_CM_PMIN].ensure(2 * n4));
  TRY(w.b[B_CM_SIDES].ensure((size_t)N + 64));
  TRY(w.b[B_CM_CTL].ensure(64 * 8 + CNT_NUM * 8));
  size_t tb = prim_radix_tmp_bytes(N), sb = prim_scan_tmp_bytes(N);
  TRY(w.b[B_CM_TMP].ensure(tb > sb ? tb : sb));
  int32_t *cur = w.b[B_CM_CUR].as<int32_t>(), *part = w.b[B_CM_PART].as<int32_t>();
  int32_t *comm = w.b[B_CM_COMM].as<int32_t>(), *acc = w.b[B_CM_ACC].as<int32_t>();
  int32_t *ctl = w.b[B_CM_CTL].as<int32_t>();  // [0] nv, [1] nsets, [2] nparts, [3] np, [4] nruns
  unsigned long long *cnt = (unsigned long long *)(w.b[B_CM_CTL].as<unsigned long long>() + 64);
  void *tmp = w.b[B_CM_TMP].p;
  size_t tmpb = w.b[B_CM_TMP].bytes;
  TRY(prim_fill32(cnt, 0u, 2 * CNT_NUM, s));
  TRY(prim_fill32(acc, 0xffffffffu, N, s));
  // Alg. 4: CCR, components larger than s_pre (a component is labelled by its smallest vertex)
  TRY(ccr_impl(g, mem_in, comm, s));
  TRY(cm_ccr_gate(comm, N, p.s_pre, w.b[B_CM_NCOMM].as<int32_t>(), cur, s));
  int nbits = bits_for(N);
  for (;;) {
    TRY(prim_fill32(ctl, 0u, 8, s));
    TRY(cm_set_keys(cur, N, w.b[B_CM_K1].as<uint32_t>(), w.b[B_CM_V1].as<uint32_t>(), ctl, s));
    int32_t hv[2];
    HIP_TRY(hipMemcpyAsync(hv, ctl, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t nv = hv[0];
    if (nv == 0) break;
    st.levels++;
    int alt = 0;
    TRY(prim_radix_sort_pairs(w.b[B_CM_K1].as<uint32_t>(), w.b[B_CM_V1].as<uint32_t>(), w.b[B_CM_K2].as<uint32_t>(),
                              w.b[B_CM_V2].as<uint32_t>(), N, nbits, tmp, tmpb, s, &alt));
    const uint32_t *sk = w.b[alt ? B_CM_K2 : B_CM_K1].as<uint32_t>();
    const uint32_t *sv = w.b[alt ? B_CM_V2 : B_CM_V1].as<uint32_t>();
    int32_t *verts = w.b[B_CM_VERTS].as<int32_t>(), *setidx = w.b[B_CM_SETIDX].as<int32_t>();
    int64_t *so = w.b[B_CM_SO].as<int64_t>();
    TRY(prim_fill32(w.b[B_CM_SETOF].p, 0xffffffffu, N, s));  // (vertices in no set: -1)
    TRY(cm_sets(sk, sv, nv, ctl, w.b[B_CM_FLAG].as<int32_t>(), w.b[B_CM_FSCAN].as<int32_t>(), ctl + 1, so, verts,
                setidx, w.b[B_CM_SETOF].as<int32_t>(), tmp, tmpb, s));
    HIP_TRY(hipMemcpyAsync(hv, ctl, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t nsets = hv[1];
    int32_t *caps = w.b[B_CM_CAPS].as<int32_t>(), *hase = w.b[B_CM_HASE].as<int32_t>();
    int32_t *ssz = w.b[B_CM_SSZ].as<int32_t>(), *lam = w.b[B_CM_LAM].as<int32_t>();
    int32_t *psz = w.b[B_CM_PSZ].as<int32_t>(), *pmin = w.b[B_CM_PMIN].as<int32_t>();
    unsigned long long *shash = w.b[B_CM_SHASH].as<unsigned long long>();
    uint8_t *sides = w.b[B_CM_SIDES].as<uint8_t>();
    TRY(cm_caps(so, ctl + 1, nsets, p, caps, hase, ssz, shash, psz, pmin, s));
    TRY(cm_edges(g, verts, setidx, w.b[B_CM_SETOF].as<int32_t>(), ctl, nv, hase, s));
    // GetMinCut + MinCutPartition of every set (capped at k(n), Alg. 5)
    TRY(split_batch_impl(g, verts, so, nsets, caps, lam, sides, nv, s));
    TRY(prim_fill32(part, 0xffffffffu, N, s));
    TRY(cm_outcome(so, verts, setidx, sides, ctl, ctl + 1, nv > nsets ? nv : nsets, hase, caps, lam, ssz, shash,
                   psz, pmin, p.s_post, acc, part, ctl + 2, rec, rec_cap, cnt, s));
    // the parts' communities (GetCommunities with the CDA), then the next sets
    int comm_bits = nbits;
    TRY(cda_impl(w, g, part, cm, comm, &comm_bits, s));
    TRY(cm_part_count(part, N, w.b[B_CM_FLAG].as<int32_t>(), w.b[B_CM_FSCAN].as<int32_t>(), ctl + 3, tmp, tmpb, s));
    int32_t hc[4];
    HIP_TRY(hipMemcpyAsync(hc, ctl, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t np = hc[3];
    TRY(prim_fill32(cur, 0xffffffffu, N, s));
    if (np == 0) continue;
    TRY(prim_fill32(w.b[B_CM_NCOMM].p, 0u, N, s));
    TRY(prim_fill32(w.b[B_CM_RUNSIZE].p, 0u, np, s));
    TRY(cm_next(part, comm, N, p.s_post, comm_bits, cur, w.b[B_CM_FSCAN].as<int32_t>(), ctl + 3, np,
                w.b[B_CM_K1].as<uint32_t>(), w.b[B_CM_V1].as<uint32_t>(), w.b[B_CM_K2].as<uint32_t>(),
                w.b[B_CM_V2].as<uint32_t>(), w.b[B_CM_NCOMM].as<int32_t>(), w.b[B_CM_RUNF].as<int32_t>(),
                w.b[B_CM_RUNS].as<int32_t>(), w.b[B_CM_RUNSTART].as<int32_t>(), w.b[B_CM_RUNSIZE].as<int32_t>(),
                ctl + 4, tmp, tmpb, s));
  }
  TRY(items_relabel(acc, N, w.b[B_MARK].as<int32_t>(), w.b[B_RANK].as<int32_t>(), out, w.b[B_TMP].p,
                    w.b[B_TMP].bytes, s));
  unsigned long long hcnt[CNT_NUM];
  HIP_TRY(hipMemcpyAsync(hcnt, cnt, sizeof(hcnt), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  st.mincuts = (int64_t)hcnt[CNT_MINCUTS];
  st.items = st.mincuts;
  st.accepted = (int64_t)hcnt[CNT_ACCEPTED];
  if (nrec) *nrec = (int64_t)hcnt[CNT_RECORDS];
  st.ms_total = ms_since(t0);
  if (stats) *stats = st;
  return WCC_OK;
}

}  // namespace

static thread_local char g_detail[512] = "";

// ---------------------------------------------------------------- allocation-free entry
// The workspace of wcc_run_noalloc lives in this array: one copy per GPU, held until the
// process ends.  Host code never uses the name as an address (on the host it is only a
// stand-in for the symbol): the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
constexpr int64_t NOALLOC_MAX_VERTICES = 1 << 16;
constexpr int64_t NOALLOC_MAX_ENTRIES = 1 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
struct NoallocDev {
  Workspace *w = nullptr;
  Carver carve;
};
std::vector<NoallocDev> g_noalloc;

// Set-up on the first call on a device: the scratch array's device address, and a
// workspace (streams, events) whose buffers are carved from it.
int noalloc_setup(NoallocDev **out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if ((int)g_noalloc.size() <= dev) g_noalloc.resize(dev + 1);
  NoallocDev &nd = g_noalloc[dev];
  if (!nd.w) {
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return WCC_EHIP;
    Workspace *w = new Workspace();
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    int rc = ws_init(*w, dev, prop);
    if (rc) {
      w->destroy();
      delete w;
      return rc;
    }
    nd.carve.base = (char *)ptr;
    nd.carve.size = NOALLOC_SCRATCH_BYTES;
    for (auto &b : w->b) b.carve = &nd.carve;
    nd.w = w;
  }
  *out = &nd;
  return WCC_OK;
}
}  // namespace

// ---------------------------------------------------------------- served form
struct wcc_server {
  struct Job {
    wcc_job j;
    int64_t id;
    double t_submit;
    int64_t est;
  };
  int dev = 0;
  int slots = 1;
  int64_t budget = 0;
  std::mutex mu;
  std::condition_variable cv;       // work arrived / budget freed / stop
  std::condition_variable cv_done;  // a job completed
  std::deque<Job> pending;
  std::vector<wcc_result> done;
  std::vector<Workspace *> ws;
  std::vector<hipStream_t> st;
  std::vector<int64_t> retained;    // workspace bytes a slot holds
  std::vector<char> busy;
  std::vector<std::thread> th;
  bool stop = false;
  int64_t next_id = 1;
  int64_t inflight = 0;             // submitted and not completed
  std::chrono::steady_clock::time_point t0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  int64_t total_retained() const {
    int64_t t = 0;
    for (int64_t r : retained) t += r;
    return t;
  }
  // Called with mu held: can slot i start the head job?  May release idle slots'
  // cached workspaces to make room.  Sets *fail when the job can never fit.
  bool admissible(int i, bool *fail) {
    *fail = false;
    const Job &jb = pending.front();
    int64_t need = jb.est > retained[i] ? jb.est - retained[i] : 0;
    if (total_retained() + need <= budget) return true;
    for (int k = 0; k < slots; k++)
      if (k != i && !busy[k] && retained[k] > 0) {
        ws[k]->release();
        retained[k] = 0;
        if (total_retained() + need <= budget) return true;
      }
    bool any_busy = false;
    for (int k = 0; k < slots; k++) any_busy = any_busy || busy[k];
    if (!any_busy) {
      // nothing else holds memory: release this slot's cache too, then it fits or never will
      ws[i]->release();
      retained[i] = 0;
      if (jb.est <= budget) return true;
      *fail = true;
    }
    return false;
  }
  void worker(int i) {
    (void)hipSetDevice(dev);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool fail = false;
      cv.wait(lk, [&] { return stop || (!pending.empty() && (admissible(i, &fail) || fail)); });
      if (stop) break;
      Job jb = pending.front();
      pending.pop_front();
      if (fail) {
        wcc_result r;
        memset(&r, 0, sizeof(r));
        r.job_id = jb.id;
        r.tag = jb.j.tag;
        r.status = WCC_ENOMEM;
        r.slot = -1;
        r.t_submit_ms = jb.t_submit;
        r.t_start_ms = r.t_end_ms = now_ms();
        r.footprint_bytes = jb.est;
        done.push_back(r);
        inflight--;
        cv_done.notify_all();
        cv.notify_all();
        continue;
      }
      busy[i] = 1;
      if (jb.est > retained[i]) retained[i] = jb.est;  // reserved while it runs
      cv.notify_all();  // the next job may fit on another slot
      lk.unlock();
      wcc_result r;
      memset(&r, 0, sizeof(r));
      r.job_id = jb.id;
      r.tag = jb.j.tag;
      r.slot = i;
      r.t_submit_ms = jb.t_submit;
      r.footprint_bytes = jb.est;
      r.t_start_ms = now_ms();
      wcc_params p = jb.j.params;
      p.flags |= WCC_FLAG_NO_GRAPH;
      int rc = wcc_run_impl(*ws[i], &jb.j.g, jb.j.membership_in, &p, jb.j.membership_out, &r.stats, nullptr, 0,
                            nullptr, st[i]);
      if (rc == WCC_OK && hipStreamSynchronize(st[i]) != hipSuccess) {
        (void)hipGetLastError();
        rc = WCC_EHIP;
      }
      r.status = rc;
      r.t_end_ms = now_ms();
      lk.lock();
      busy[i] = 0;
      retained[i] = ws[i]->bytes();
      done.push_back(r);
      inflight--;
      cv_done.notify_all();
      cv.notify_all();
    }
  }
};


void wcc_note_hip_error(hipError_t e, const char *expr, const char *file, int line) {
  const char *base = strrchr(file, '/');
  snprintf(g_detail, sizeof(g_detail), "%s (%d) at %s:%d: %s", hipGetErrorString(e), (int)e,
           base ? base + 1 : file, line, expr);
}

// ---------------------------------------------------------------- C ABI
extern "C" {

const char *wcc_last_error_detail(void) { return g_detail; }

void wcc_default_params(wcc_params *p) {
  if (!p) return;
  memset(p, 0, sizeof(*p));
  p->criterion = WCC_CRIT_LOG10;
  p->lin_num = 1;
  p->lin_den = 1;
  p->s_pre = 10;
  p->s_post = 10;
  p->prune_mode = WCC_PRUNE_KCORE;
  p->mincut_rule = 1;
  p->exec_mode = WCC_EXEC_PLAIN;
  p->flags = 0;
}

int wcc_run(const wcc_csr *g, const int32_t *membership_in, const wcc_params *p, int32_t *membership_out,
            wcc_stats *stats, wcc_record *records, int64_t records_cap, int64_t *num_records, void *stream) {
  std::lock_guard<std::mutex> lk(g_lock);
  try {
    Workspace *wp;
    TRY(get_ws(&wp));
    return wcc_run_impl(*wp, g, membership_in, p, membership_out, stats, records, records_cap, num_records,
                        (hipStream_t)stream);
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int wcc_mincut_split_batch(const wcc_csr *g, const int32_t *verts, const int64_t *set_offsets, int32_t num_sets,
                           const int32_t *caps, int32_t *lambdas, uint8_t *sides, void *stream) {
  std::lock_guard<std::mutex> lk(g_lock);
  try {
    if (num_sets < 0) return WCC_EINVAL;
    if (num_sets == 0) return WCC_OK;
    if (!set_offsets) return WCC_EINVAL;
    int64_t nv = 0;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipMemcpyAsync(&nv, set_offsets + num_sets, sizeof(nv), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (nv < 0) return WCC_EINVAL;
    return split_batch_impl(g, verts, set_offsets, num_sets, caps, lambdas, sides, nv, s);
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int wcc_ccr_components(const wcc_csr *g, const int32_t *membership_in, int32_t *comp_out, void *stream) {
  std::lock_guard<std::mutex> lk(g_lock);
  try {
    return ccr_impl(g, membership_in, comp_out, (hipStream_t)stream);
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int wcc_run_noalloc(const wcc_csr *g, const int32_t *membership_in, const wcc_params *p, int32_t *membership_out,
                    wcc_stats *stats, wcc_record *records, int64_t records_cap, int64_t *num_records,
                    void *stream) {
  std::lock_guard<std::mutex> lk(g_lock);
  try {
    int rc = check_csr(g);
    if (rc) return rc;
    if (g->num_vertices > NOALLOC_MAX_VERTICES || g->num_entries > NOALLOC_MAX_ENTRIES) {
      snprintf(g_detail, sizeof(g_detail),
               "wcc_run_noalloc: %lld vertices / %lld entries exceed its limits (%lld / %lld)",
               (long long)g->num_vertices, (long long)g->num_entries, (long long)NOALLOC_MAX_VERTICES,
               (long long)NOALLOC_MAX_ENTRIES);
      return WCC_EUNSUPPORTED;
    }
    NoallocDev *nd;
    TRY(noalloc_setup(&nd));
    // every call carves the workspace afresh from the start of the array
    nd->carve.used = 0;
    for (auto &b : nd->w->b) {
      b.p = nullptr;
      b.bytes = 0;
    }
    wcc_params pp;
    if (p) pp = *p;
    else wcc_default_params(&pp);
    pp.exec_mode = WCC_EXEC_PLAIN;  // (a recorded graph would be an allocation)
    return wcc_run_impl(*nd->w, g, membership_in, &pp, membership_out, stats, records, records_cap, num_records,
                        (hipStream_t)stream);
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int wcc_cm_run(const wcc_csr *g, const int32_t *membership_in, const wcc_params *p, const wcc_cm_params *cm,
               int32_t *membership_out, wcc_stats *stats, wcc_record *records, int64_t records_cap,
               int64_t *num_records, void *stream) {
  std::lock_guard<std::mutex> lk(g_lock);
  try {
    wcc_params pp;
    if (p) pp = *p;
    else wcc_default_params(&pp);
    if (!cm) return WCC_EINVAL;
    return cm_impl(g, membership_in, pp, *cm, membership_out, stats, records, records_cap, num_records,
                   (hipStream_t)stream);
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int wcc_cda(const wcc_csr *g, const int32_t *part_of, const wcc_cm_params *cm, int32_t *comm_out, void *stream) {
  std::lock_guard<std::mutex> lk(g_lock);
  try {
    TRY(check_csr(g));
    TRY(check_cm(cm));
    if (cm->cda == WCC_CDA_CALLBACK) return WCC_EINVAL;
    if (g->num_vertices == 0) return WCC_OK;
    if (!part_of || !comm_out) return WCC_EINVAL;
    Workspace *wp;
    TRY(get_ws(&wp));
    int bits = 0;
    hipStream_t s = (hipStream_t)stream;
    TRY(cda_impl(*wp, g, part_of, *cm, comm_out, &bits, s));
    HIP_TRY(hipStreamSynchronize(s));
    return WCC_OK;
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int wcc_mincut_split(const wcc_csr *g, const int32_t *verts, int32_t n, int32_t cap, int32_t *lambda,
                     uint8_t *side, void *stream) {
  if (!lambda || n < 0 || cap < 1) return WCC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  {
    std::lock_guard<std::mutex> lk(g_lock);
    try {
      Workspace *wp;
      rc = get_ws(&wp);
      if (rc) return rc;
      rc = wp->b[B_SMALL].ensure(64);
      if (rc) return rc;
      int64_t *so = wp->b[B_SMALL].as<int64_t>();
      int64_t hso[2] = {0, n};
      int32_t hcap = cap;
      HIP_TRY(hipMemcpyAsync(so, hso, sizeof(hso), hipMemcpyHostToDevice, s));
      HIP_TRY(hipMemcpyAsync(so + 2, &hcap, sizeof(hcap), hipMemcpyHostToDevice, s));
      int32_t *dl = (int32_t *)(so + 3);
      rc = split_batch_impl(g, verts, so, 1, (const int32_t *)(so + 2), dl, side, n, s);
      if (rc) return rc;
      HIP_TRY(hipMemcpyAsync(lambda, dl, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
    } catch (...) {
      return WCC_ENOMEM;
    }
  }
  return rc;
}

int wcc_cluster_csr(const wcc_csr *g, const int32_t *membership_in, int64_t *nclusters, int64_t *nassigned,
                    int64_t *nentries, int32_t *cl_ids, int64_t *cl_start, int32_t *vert, int64_t *row_off,
                    int32_t *adj, void *stream) {
  std::lock_guard<std::mutex> lk(g_lock);
  try {
    int rc = check_csr(g);
    if (rc) return rc;
    if (!nclusters || !nassigned || !nentries) return WCC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    *nclusters = *nassigned = *nentries = 0;
    if (g->num_vertices == 0) return WCC_OK;
    if (!membership_in) return WCC_EINVAL;
    Workspace *wp;
    TRY(get_ws(&wp));
    Workspace &w = *wp;
    TRY(run_front(w, g, membership_in, true, false, s));
    FrontCounts fo;
    TRY(read_counts(w, &fo, s));
    *nclusters = fo.K;
    *nassigned = fo.na;
    *nentries = fo.E;
    if (cl_ids && fo.K > 0) HIP_TRY(hipMemcpyAsync(cl_ids, w.b[B_CLIDS].p, fo.K * 4, hipMemcpyDeviceToDevice, s));
    if (cl_start) HIP_TRY(hipMemcpyAsync(cl_start, w.b[B_CLSTART].p, (fo.K + 1) * 8, hipMemcpyDeviceToDevice, s));
    if (vert && fo.na > 0) HIP_TRY(hipMemcpyAsync(vert, w.b[B_VTX0].p, fo.na * 4, hipMemcpyDeviceToDevice, s));
    if (row_off) {
      if (fo.na > 0) HIP_TRY(hipMemcpyAsync(row_off, w.b[B_RS0].p, fo.na * 8, hipMemcpyDeviceToDevice, s));
      int64_t E = fo.E;
      HIP_TRY(hipMemcpyAsync(row_off + fo.na, &E, 8, hipMemcpyHostToDevice, s));
    }
    if (adj && fo.E > 0) HIP_TRY(hipMemcpyAsync(adj, w.b[B_ADJ0].p, fo.E * 4, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return WCC_OK;
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int64_t wcc_threshold(int32_t criterion, int64_t n, int32_t lin_num, int32_t lin_den) {
  if (criterion < WCC_CRIT_LOG10 || criterion > WCC_CRIT_LINEAR) return -1;
  if (criterion == WCC_CRIT_LINEAR && (lin_den < 1 || lin_num < 0)) return -1;
  return wcc_k_of(criterion, n, lin_num, lin_den);
}

const char *wcc_strerror(int code) {
  switch (code) {
    case WCC_OK: return "ok";
    case WCC_EINVAL: return "invalid argument";
    case WCC_EGRAPH: return "malformed graph (CSR not symmetric simple)";
    case WCC_ENOMEM: return "out of device memory";
    case WCC_EHIP: return "HIP runtime error";
    case WCC_ENOTCONNECTED: return "set not connected";
    case WCC_ECANCELLED: return "cancelled";
    case WCC_ETIMEOUT: return "timed out";
    case WCC_ENODEV: return "no HIP device";
    case WCC_EUNSUPPORTED: return "size or parameter beyond the library's limits";
  }
  return "unknown error";
}

int wcc_autotune(const wcc_csr *g, const int32_t *membership_in, const wcc_params *pp, int32_t reps,
                 wcc_exec_config *best, double *best_ms, int32_t *tried, void *stream) {
  if (!best || reps < 1 || reps > 16) return WCC_EINVAL;
  std::lock_guard<std::mutex> lk(g_lock);
  try {
    return autotune_impl(g, membership_in, pp, reps, best, best_ms, tried, (hipStream_t)stream);
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int wcc_server_create(const wcc_server_cfg *cfg, wcc_server **out) {
  if (!cfg || !out || cfg->slots < 1 || cfg->slots > 16 || cfg->pool_bytes < 0) return WCC_EINVAL;
  *out = nullptr;
  try {
    wcc_server *sv = new wcc_server();
    int rc = WCC_OK;
    HIP_TRY(hipGetDevice(&sv->dev));
    size_t fr = 0, tot = 0;
    HIP_TRY(hipMemGetInfo(&fr, &tot));
    sv->budget = cfg->pool_bytes > 0 ? cfg->pool_bytes : (int64_t)(fr / 10 * 8);
    sv->slots = cfg->slots;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, sv->dev));
    for (int i = 0; i < sv->slots && rc == WCC_OK; i++) {
      Workspace *w = new Workspace();
      rc = ws_init(*w, sv->dev, prop);
      hipStream_t s1 = nullptr;
      if (rc == WCC_OK && hipStreamCreateWithFlags(&s1, hipStreamNonBlocking) != hipSuccess) rc = WCC_EHIP;
      sv->ws.push_back(w);
      sv->st.push_back(s1);
      sv->retained.push_back(0);
      sv->busy.push_back(0);
    }
    if (rc != WCC_OK) {
      for (size_t i = 0; i < sv->ws.size(); i++) {
        sv->ws[i]->destroy();
        delete sv->ws[i];
        if (sv->st[i]) (void)hipStreamDestroy(sv->st[i]);
      }
      delete sv;
      return rc;
    }
    sv->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < sv->slots; i++) sv->th.emplace_back([sv, i] { sv->worker(i); });
    *out = sv;
    return WCC_OK;
  } catch (...) {
    return WCC_ENOMEM;
  }
}

int wcc_server_submit(wcc_server *sv, const wcc_job *job, int64_t *job_id) {
  if (!sv || !job) return WCC_EINVAL;
  int rc = check_params(job->params);
  if (rc == WCC_OK) rc = check_csr(&job->g);
  if (rc != WCC_OK) return rc;
  if (job->g.num_vertices > 0 && (!job->membership_in || !job->membership_out)) return WCC_EINVAL;
  try {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) return WCC_ECANCELLED;
    wcc_server::Job jb;
    jb.j = *job;
    jb.id = sv->next_id++;
    jb.t_submit = sv->now_ms();
    jb.est = est_workspace_bytes(job->g.num_vertices, job->g.num_entries);
    sv->pending.push_back(jb);
    sv->inflight++;
    if (job_id) *job_id = jb.id;
  } catch (...) {
    return WCC_ENOMEM;
  }
  sv->cv.notify_all();
  return WCC_OK;
}

int wcc_server_poll(wcc_server *sv, wcc_result *out, int32_t max, int32_t *n) {
  if (!sv || !n || max < 0 || (max > 0 && !out)) return WCC_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  int32_t k = 0;
  while (k < max && !sv->done.empty()) {
    out[k++] = sv->done.front();
    sv->done.erase(sv->done.begin());
  }
  *n = k;
  return WCC_OK;
}

int wcc_server_wait(wcc_server *sv, int64_t timeout_ms) {
  if (!sv) return WCC_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto idle = [&] { return sv->inflight == 0; };
  if (timeout_ms < 0) {
    sv->cv_done.wait(lk, idle);
    return WCC_OK;
  }
  return sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), idle) ? WCC_OK : WCC_ETIMEOUT;
}

int wcc_server_destroy(wcc_server *sv) {
  if (!sv) return WCC_EINVAL;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->inflight -= (int64_t)sv->pending.size();
    sv->pending.clear();
  }
  sv->cv.notify_all();
  for (auto &t : sv->th) t.join();
  for (size_t i = 0; i < sv->ws.size(); i++) {
    sv->ws[i]->destroy();
    delete sv->ws[i];
    if (sv->st[i]) (void)hipStreamDestroy(sv->st[i]);
  }
  delete sv;
  return WCC_OK;
}

int wcc_get_exec_config(wcc_exec_config *cfg) {
  if (!cfg) return WCC_EINVAL;
  std::lock_guard<std::mutex> lk(g_lock);
  Workspace *wp;
  TRY(get_ws(&wp));
  *cfg = wp->cfg;
  return WCC_OK;
}

int wcc_set_exec_config(const wcc_exec_config *cfg) {
  std::lock_guard<std::mutex> lk(g_lock);
  Workspace *wp;
  TRY(get_ws(&wp));
  ExecCfg c;
  if (cfg) {
    if (!cfg_valid(*cfg)) return WCC_EINVAL;
    static_cast<wcc_exec_config &>(c) = *cfg;
  }
  wp->cfg = c;
  return WCC_OK;
}

int wcc_release(void) {
  std::lock_guard<std::mutex> lk(g_lock);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WCC_EHIP;
  if (dev < (int)g_ws.size() && g_ws[dev]) g_ws[dev]->release();
  return WCC_OK;
}

int wcc_abi_version(void) { return 1; }

}  // extern "C"
