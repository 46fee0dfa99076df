/*
 * wcc.h -- C ABI of the MI355X (gfx950) Well-Connected Clusters hot path.
 *
 * Method: Dindoost et al., "On the Optimization of Methods for Establishing
 * Well-Connected Communities", arXiv 2509.02590.
 *   - CCR, Alg. 1: each input cluster's induced subgraph; when it has edges, its
 *     connected components larger than s_pre are queued.
 *   - WCC, Alg. 2, and isWCC, Alg. 3: a queued set whose exact global minimum cut exceeds
 *     the criterion f(n) of its size (Sec. 2: log10 n, log2 n, sqrt n, or linear k*n) is
 *     saved; otherwise it is split along the cut and every part larger than s_post is
 *     processed again.
 *   - GetMinCut / MinCutPartition, Alg. 3 and Sec. 2.1: the cut and its two sides.
 *
 * Conventions shared by every entry point:
 *   - Graphs are undirected, simple and unweighted, in symmetric CSR form: each edge
 *     {u,v} is stored once in u's row and once in v's row, no self-loops, no
 *     duplicates.  The order of entries inside a row does not matter.
 *   - Every pointer documented "device" is a device allocation owned by the caller.
 *     The library never frees caller memory; it owns its own workspace, which it
 *     allocates lazily per device and keeps until wcc_release() or process exit.
 *   - stream is a hipStream_t passed as void*; NULL means the null stream.  Each call
 *     enqueues its work on that stream and returns once the documented outputs are
 *     complete (the calls are blocking).
 *   - Return value: WCC_OK (0) or one of the negative WCC_E* codes.  No C++ exception
 *     crosses this boundary.  On error the outputs are unspecified.
 *   - Calls on the same device are serialised by an internal lock.
 *
 * Canonical results (needed for bit-exact comparison, not fixed by the paper):
 *   - the threshold test "cut > f(n)" is evaluated as cut >= k(n), k(n) the least
 *     integer above f(n): LOG10 -> decimal digits of n, LOG2 -> bit length of n,
 *     SQRT -> isqrt(n)+1, LINEAR -> floor(num*n/den)+1;
 *   - among equal minimum cuts the library returns the one produced by the canonical
 *     scan-and-contract rule: degree pre-pass, then rounds of maximum-adjacency scans
 *     from the smallest vertex id with keys capped at the current bound, ties to the
 *     smallest id, contraction of every edge whose key reaches the bound, and a
 *     strict-improvement degree check in ascending id order;
 *   - local ids are ranks of global vertex ids, so "smallest id" means smallest global id;
 *   - output labels number the saved sets 0..K-1 by ascending smallest global vertex id;
 *     every other vertex gets -1.
 */
#ifndef WCC_H
#define WCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ error codes */
#define WCC_OK 0
#define WCC_EINVAL -1        /* bad argument or parameter */
#define WCC_EGRAPH -2        /* CSR is not symmetric simple (checked with WCC_FLAG_VALIDATE) */
#define WCC_ENOMEM -3        /* device workspace could not be allocated */
#define WCC_EHIP -4          /* a HIP runtime call failed */
#define WCC_ENOTCONNECTED -5 /* reserved */
#define WCC_ECANCELLED -6    /* a served job was cancelled */
#define WCC_ETIMEOUT -7      /* a served job did not finish in time */
#define WCC_ENODEV -8        /* no HIP device */
#define WCC_EUNSUPPORTED -9  /* a size or parameter beyond the library's limits */

/* ------------------------------------------------------------------ inputs */
typedef struct {
  int64_t num_vertices;    /* N */
  int64_t num_entries;     /* directed CSR entries, 2m */
  const void *row_offsets; /* device, N+1 offsets of width offset_bits (32 or 64) */
  int32_t offset_bits;     /* 32 -> int32_t offsets, 64 -> int64_t offsets */
  int32_t reserved;
  const int32_t *col_indices; /* device, num_entries neighbour ids in [0, N) */
} wcc_csr;

/* Criterion f(n) of Sec. 2. */
#define WCC_CRIT_LOG10 0
#define WCC_CRIT_LOG2 1
#define WCC_CRIT_SQRT 2
#define WCC_CRIT_LINEAR 3 /* f(n) = lin_num * n / lin_den */

/* Pruning at entry of a queued set. */
#define WCC_PRUNE_PAPER 0 /* Alg. 1-3 as printed: no pruning */
#define WCC_PRUNE_KCORE 1 /* a set of size n is replaced by the connected components of its
                             k(n)-core (larger than s_post) whenever that core is not the
                             whole set; only whole-core sets are cut */

#define WCC_EXEC_PLAIN 0   /* level-synchronous: per recursion depth, one launch for each
                              size bin, the host reading the child count in between */
#define WCC_EXEC_BATCHED 1 /* device-driven: per recursion depth one launch for each size
                              bin whose item count is read on the device; children go
                              straight into the next depth's size-bin lists, the host does
                              not synchronise inside a run, and the whole call is recorded
                              as a HIP graph and replayed when called again with the same
                              buffers and parameters */

#define WCC_FLAG_VALIDATE 1u /* check the CSR first: offsets non-decreasing from 0 to
                                num_entries, ids in [0, N), no self-loop, no entry repeated
                                in its row, every entry matched by its reverse; WCC_EGRAPH
                                if any check fails */
#define WCC_FLAG_NO_GRAPH 2u /* BATCHED: neither record nor replay a HIP graph */

typedef struct {
  int32_t criterion;   /* WCC_CRIT_* (default LOG10) */
  int32_t lin_num;     /* LINEAR only; lin_num >= 0, lin_den >= 1 */
  int32_t lin_den;
  int32_t s_pre;       /* CCR keeps components with size > s_pre (Alg. 1); >= 0 */
  int32_t s_post;      /* parts with size > s_post are processed again (Alg. 3); >= 0 */
  int32_t prune_mode;  /* WCC_PRUNE_* */
  int32_t mincut_rule; /* 1 = the canonical rule above (the only one) */
  int32_t exec_mode;   /* WCC_EXEC_* */
  uint32_t flags;      /* WCC_FLAG_* */
  int32_t reserved;
} wcc_params;

/* Fills *p with the defaults: LOG10, s_pre = s_post = 10, KCORE, rule 1, PLAIN. */
void wcc_default_params(wcc_params *p);

/* Per-call counters (host struct, filled on success when non-NULL). */
typedef struct {
  int64_t clusters;      /* distinct input cluster ids */
  int64_t intra_entries; /* directed entries of all induced cluster subgraphs */
  int64_t items;         /* queued sets processed, clusters included */
  int64_t mincuts;       /* minimum-cut evaluations */
  int64_t accepted;      /* saved sets */
  int64_t levels;        /* recursion depths (launch rounds) */
  int64_t scan_steps;    /* maximum-adjacency scan steps over all cuts (a cut whose
                            lambda >= bound is certified by edge-disjoint spanning
                            forests adds none; work counters only, the results do not
                            depend on which way a cut was found) */
  int64_t scan_rounds;   /* scan-and-contract rounds over all cuts */
  double ms_front;       /* device time: validation, grouping and compaction */
  double ms_items;       /* device time: all item launches */
  double ms_item_kernel; /* summed durations of the item-kernel launches */
  int64_t item_launches; /* number of item-kernel launches */
  double ms_total;       /* host wall time of the call */
  int64_t item_alg_bytes; /* algorithmic bytes of the item launches: each processed set's
                             rows read once (16 B per vertex + 4 B per entry), each child's
                             rows written once, 4 B per saved vertex */
  int64_t graph_replays;  /* 1 when the call replayed a recorded HIP graph */
  int64_t reserved[3];
} wcc_stats;

/* One record per minimum-cut evaluation (order of records is unspecified). */
typedef struct {
  int32_t minv;   /* smallest global vertex id of the set */
  int32_t n;      /* set size */
  int32_t k;      /* k(n), used as the cut cap */
  int32_t lambda; /* returned cut value: exact if below k, else k */
  int32_t ssize;  /* size of the recorded side S (0 if none) */
  int32_t reserved;
  uint64_t shash; /* sum over v in S of splitmix64-finaliser(v + 0x9E3779B97F4A7C15) */
} wcc_record;

/* ------------------------------------------------------------------ entry points */

/*
 * wcc_run -- WCC over a whole graph and input clustering (Alg. 1-3).
 *   g              device CSR of G (N vertices).
 *   membership_in  device, N int32: input cluster id of each vertex (any non-negative
 *                  value; clusters are the classes of equal ids) or < 0 for unassigned.
 *   p              host parameters (NULL = defaults).
 *   membership_out device, N int32, caller-allocated: canonical label or -1.
 *   stats          host, nullable.
 *   records        device, nullable: up to records_cap wcc_record entries; the total
 *                  number produced is written to *num_records (host, nullable) even
 *                  when it exceeds records_cap (then only the first records_cap are kept).
 * Errors: WCC_EINVAL (NULL required pointers, s_pre/s_post < 0, bad criterion, N < 0 or
 * num_entries inconsistent with offsets), WCC_EGRAPH (with WCC_FLAG_VALIDATE),
 * WCC_ENOMEM, WCC_EHIP, WCC_EUNSUPPORTED (a cluster with more than 2^24 - 1 vertices).
 */
int wcc_run(const wcc_csr *g, const int32_t *membership_in, const wcc_params *p,
            int32_t *membership_out, wcc_stats *stats, wcc_record *records, int64_t records_cap,
            int64_t *num_records, void *stream);

/*
 * wcc_mincut_split -- GetMinCut + MinCutPartition (Alg. 3; the CM step of Alg. 5) on the
 * subgraph of G induced by one vertex set.
 *   verts   device, n int32 global ids, sorted ascending, unique.
 *   cap     >= 1: the cut is exact when its value is below cap; otherwise cap is
 *           returned (pass INT32_MAX for an uncapped exact cut, of any value; WCC uses
 *           k(n)).
 *   lambda  host, out: the cut value (0 if the induced subgraph is disconnected or n < 2).
 *   side    device, n bytes, out: 1 for vertices in S.  A disconnected set returns S =
 *           the component of verts[0]; n < 2 returns S empty.
 * Errors: WCC_EINVAL (unsorted/duplicate/out-of-range verts are checked on the device),
 * WCC_ENOMEM, WCC_EHIP, WCC_EUNSUPPORTED (a set with more than 2^24 - 1 vertices).
 */
int wcc_mincut_split(const wcc_csr *g, const int32_t *verts, int32_t n, int32_t cap,
                     int32_t *lambda, uint8_t *side, void *stream);

/*
 * wcc_mincut_split_batch -- the same for num_sets pairwise disjoint vertex sets at once.
 *   verts        device, concatenated sorted unique ids of all sets.
 *   set_offsets  device, num_sets+1 int64: set i is verts[set_offsets[i] .. set_offsets[i+1]).
 *   caps         device, num_sets int32 (each >= 1).
 *   lambdas      device, num_sets int32, out.
 *   sides        device, set_offsets[num_sets] bytes, out (aligned with verts).
 * Errors as wcc_mincut_split; overlapping sets give WCC_EINVAL.
 */
int wcc_mincut_split_batch(const wcc_csr *g, const int32_t *verts, const int64_t *set_offsets,
                           int32_t num_sets, const int32_t *caps, int32_t *lambdas,
                           uint8_t *sides, void *stream);

/*
 * wcc_cluster_csr -- the membership-filtered compaction alone (the first step of Alg. 1:
 * E_c = edges with both endpoints in c), exposed for inspection and tests.
 * Outputs are cluster-major: clusters in ascending cluster id, vertices in ascending id
 * inside a cluster, each row holding local ids (ranks inside the cluster) in
 * unspecified order.  Call once with NULL outputs to get the sizes.
 *   nclusters, nassigned, nentries   host, out.
 *   cl_ids     device, nclusters int32          cl_start  device, nclusters+1 int64
 *   vert       device, nassigned int32 global ids
 *   row_off    device, nassigned+1 int64        adj       device, nentries int32
 */
int wcc_cluster_csr(const wcc_csr *g, const int32_t *membership_in, int64_t *nclusters,
                    int64_t *nassigned, int64_t *nentries, int32_t *cl_ids, int64_t *cl_start,
                    int32_t *vert, int64_t *row_off, int32_t *adj, void *stream);

/*
 * wcc_ccr_components -- connected component refinement alone (Alg. 1, the first step of
 * both WCC and CM): for every assigned vertex v, comp_out[v] = the smallest global id in
 * v's connected component of the subgraph induced by v's cluster; -1 when v is
 * unassigned.  No size gate is applied (a caller keeps components larger than s_pre).
 *   g              device CSR (as for wcc_run)
 *   membership_in  device, N int32 (negative = unassigned)
 *   comp_out       device, N int32, caller-allocated
 * Blocks until comp_out is complete.  Errors: WCC_EINVAL, WCC_ENOMEM, WCC_EHIP.
 */
int wcc_ccr_components(const wcc_csr *g, const int32_t *membership_in, int32_t *comp_out, void *stream);

/* ------------------------------------------------------------------ Connectivity Modifier */
/* The community detection step of CM (GetCommunities with a CDA, Alg. 5).  Built in:
 *   WCC_CDA_COMPONENTS  the connected components of each part;
 *   WCC_CDA_LABELPROP   label propagation with ties broken deterministically: every vertex
 *                       starts with its own id as label; in each of cda_iters synchronous
 *                       rounds every vertex with a neighbour in its part takes the label that
 *                       occurs most often among those neighbours' labels of the previous
 *                       round, the smallest such label on ties; communities are the classes
 *                       of equal final labels;
 *   WCC_CDA_CALLBACK    the caller's function (e.g. a Leiden implementation). */
#define WCC_CDA_COMPONENTS 0
#define WCC_CDA_LABELPROP 1
#define WCC_CDA_CALLBACK 2

/* A caller-supplied CDA.  part_of: device, N int32: the part of every vertex (a label
 * >= 0; vertices with equal labels form one part) or -1.  comm_out: device, N int32,
 * prefilled with -1: the callback writes a community label (any int32 >= 0) for every
 * vertex of a part; vertices of one part with equal labels form one community, and
 * communities are formed inside each part only.  The callback enqueues its work on
 * `stream` (a hipStream_t as void*) or completes it before returning, and returns
 * WCC_OK or a negative WCC_E* code, which wcc_cm_run then returns.  It must not call
 * back into this library (the calling thread holds the library's device lock). */
typedef int (*wcc_cda_fn)(const wcc_csr *g, const int32_t *part_of, int32_t *comm_out, void *user, void *stream);

typedef struct {
  int32_t cda;       /* WCC_CDA_* */
  int32_t cda_iters; /* LABELPROP: synchronous rounds, 0..1000 */
  wcc_cda_fn fn;     /* CALLBACK: the function */
  void *user;        /* CALLBACK: passed through unchanged */
} wcc_cm_params;

/*
 * wcc_cm_run -- the Connectivity Modifier (CM, Alg. 4, with its check CMC, Alg. 5) over a
 * whole graph and input clustering.  CCR (Alg. 1) first; then every queued set with at
 * least one edge gets the canonical minimum cut capped at k(n) (as in wcc_run) and is
 * saved when the cut reaches k(n).  Otherwise each side of the cut with more than s_post
 * vertices is split into communities by the CDA: when there are several, every community
 * with more than s_post vertices is checked again; when there is one, the whole side is
 * checked again ("processed as a single unit").  A disconnected set (a CDA community can
 * be one) has cut 0 and S = the component of its smallest vertex.  CM prunes nothing:
 * p->prune_mode and p->exec_mode are ignored.
 *   g, membership_in, membership_out, stats, records, records_cap, num_records: as for
 *   wcc_run (labels: saved sets by ascending smallest vertex, others -1; one record per
 *   minimum-cut evaluation).  stats carries clusters = 0, items = mincuts, accepted,
 *   levels and ms_total.
 *   cm   host: the CDA (see above).
 * Errors: WCC_EINVAL (bad arguments or CDA parameters), WCC_EGRAPH (WCC_FLAG_VALIDATE),
 * WCC_ENOMEM, WCC_EHIP, a callback's own error code.
 */
int wcc_cm_run(const wcc_csr *g, const int32_t *membership_in, const wcc_params *p, const wcc_cm_params *cm,
               int32_t *membership_out, wcc_stats *stats, wcc_record *records, int64_t records_cap,
               int64_t *num_records, void *stream);

/*
 * wcc_cda -- one built-in CDA step alone on parts of G (the GetCommunities call of Alg. 5):
 * comm_out[v] = the community label of v (a global vertex id of v's part: the smallest
 * vertex of v's component, or v's final label-propagation label), -1 for v in no part.
 *   part_of   device, N int32 (labels >= 0 or -1)
 *   cm        host: WCC_CDA_COMPONENTS or WCC_CDA_LABELPROP
 *   comm_out  device, N int32, caller-allocated
 * Blocks until comm_out is complete.  Errors: WCC_EINVAL (also for WCC_CDA_CALLBACK),
 * WCC_ENOMEM, WCC_EHIP.
 */
int wcc_cda(const wcc_csr *g, const int32_t *part_of, const wcc_cm_params *cm, int32_t *comm_out, void *stream);

/*
 * wcc_run_noalloc -- wcc_run for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, outputs and results as wcc_run in the plain execution form (p->exec_mode is
 * ignored).  The caller still passes every input and output; the library's workspace
 * is a fixed 64 MiB device array per GPU (allocated when the library is loaded and held
 * until the process ends), so the input is limited to 65,536 vertices and 1,048,576 CSR
 * entries.  The first call on a device sets up its streams and events; no call allocates
 * or frees device memory.  Every call on a GPU shares that GPU's array, so calls that
 * overlap on one GPU race; calls are serialised by the library's lock, and the array's
 * contents after a call are unspecified (each call starts from its own inputs).
 * Errors: as wcc_run; WCC_EUNSUPPORTED for inputs beyond the limits (nothing is launched).
 */
int wcc_run_noalloc(const wcc_csr *g, const int32_t *membership_in, const wcc_params *p, int32_t *membership_out,
                    wcc_stats *stats, wcc_record *records, int64_t records_cap, int64_t *num_records,
                    void *stream);

/* Threshold k(n) used by the library for the given criterion (host function). */
int64_t wcc_threshold(int32_t criterion, int64_t n, int32_t lin_num, int32_t lin_den);

/* Human-readable text of an error code (static storage). */
const char *wcc_strerror(int code);

/* ------------------------------------------------------------------ launch shape */
/* Launch shape of the item kernels on the current device.  It changes speed only: every
 * shape gives the same results.  An item goes to the large bin when its scan state does
 * not fit small_lds_kb, so small_lds_kb is the size-bin boundary. */
typedef struct {
  int32_t small_lds_kb; /* dynamic LDS of a small-bin workgroup, 4..64 KB (default 32) */
  int32_t wg_per_cu;    /* small-bin workgroups per CU; 0 = as many as the LDS allows, <= 8 */
  int32_t big_lds_kb;   /* dynamic LDS of a large-bin workgroup (one per CU), <= 159 KB */
  int32_t big_max_pct;  /* BATCHED: at most this share of the CUs (percent) runs
                           large-bin workgroups; 0 = no large-bin launch (default 100) */
  int32_t chain_min_n;  /* BATCHED: a workgroup that splits an item goes on with its largest
                           child itself (without waiting for the level to end) when that child
                           has at least this many vertices and belongs to the workgroup's size
                           bin; INT32_MAX = never; -1 (default) = automatic: every child when
                           the large items are at most four times the large-bin workgroups
                           (few long chains), never otherwise (the children of many large
                           items are better spread over the next level) */
} wcc_exec_config;

/* Current shape (host out).  Environment variables WCC_LDS_KB, WCC_WG_PER_CU,
 * WCC_BIG_LDS_KB and WCC_BIG_PCT set the initial values. */
int wcc_get_exec_config(wcc_exec_config *cfg);

/* Sets the shape used by later calls on the current device; NULL restores the
 * defaults.  WCC_EINVAL when a field is outside its range. */
int wcc_set_exec_config(const wcc_exec_config *cfg);

/* Autotuner of the launch shape.  Times wcc_run (BATCHED, no graph) on the caller's
 * input for every candidate shape -- small-bin LDS 8..64 KB (the size-bin boundary),
 * small-bin workgroups per CU, the share of CUs for the large bin -- `reps` times each
 * (best of reps, 1 <= reps <= 16), installs the fastest with wcc_set_exec_config and
 * returns it.  Every shape gives the same result, so tuning never changes output.
 *   g, membership_in, p   as for wcc_run (p may be NULL for the defaults; its
 *                         exec_mode is ignored)
 *   best                  host out: the chosen shape
 *   best_ms               host out (nullable): its best wall time per run, ms
 *   tried                 host out (nullable): number of shapes timed
 * With the environment variable WCC_TUNE_CACHE naming a file, a shape tuned earlier
 * for the same device, graph size and parameters is read from it instead of timed
 * again (then *tried = 0), and a newly tuned shape is appended to it.
 * Errors: as wcc_run; WCC_EINVAL for reps out of range or best == NULL.  The call
 * allocates the workspace wcc_run needs and an output buffer of N int32. */
int wcc_autotune(const wcc_csr *g, const int32_t *membership_in, const wcc_params *p, int32_t reps,
                 wcc_exec_config *best, double *best_ms, int32_t *tried, void *stream);

/* ------------------------------------------------------------------ served form */
/* A request loop for whole WCC jobs on the current device.  `slots` worker threads each
 * own a workspace and streams, so admitted jobs run concurrently and their kernels
 * overlap on the device.  Jobs are admitted first-in first-out when a slot is free and
 * the job's estimated workspace fits the HBM budget (idle slots give back their cached
 * workspace when that makes room); a slot takes the next job as soon as its job ends. */
typedef struct {
  int32_t slots;      /* concurrent jobs, 1..16 */
  int32_t reserved;
  int64_t pool_bytes; /* HBM budget for the slots' workspaces; 0 = 80% of free memory */
} wcc_server_cfg;

typedef struct wcc_server wcc_server;

typedef struct {
  wcc_csr g;                     /* device CSR; caller-owned, valid until the job's result is polled */
  const int32_t *membership_in;  /* device, N */
  int32_t *membership_out;       /* device, N, caller-allocated */
  wcc_params params;             /* as for wcc_run (no graph recording in the served form) */
  int64_t tag;                   /* caller's value, echoed in the result */
} wcc_job;

typedef struct {
  int64_t job_id;                /* from wcc_server_submit */
  int64_t tag;
  int32_t status;                /* WCC_OK or a negative error code (WCC_ENOMEM: larger than the budget) */
  int32_t slot;                  /* worker that ran it, -1 if never started */
  double t_submit_ms;            /* server clock: milliseconds since wcc_server_create */
  double t_start_ms;             /* admitted on a slot */
  double t_end_ms;               /* membership_out complete on the device */
  int64_t footprint_bytes;       /* workspace estimate used for admission */
  wcc_stats stats;
} wcc_result;

/* Starts the worker threads (host out *out).  WCC_EINVAL for slots outside 1..16. */
int wcc_server_create(const wcc_server_cfg *cfg, wcc_server **out);

/* Queues a job (non-blocking; the job struct is copied).  *job_id (host out) numbers jobs
 * from 1.  WCC_EINVAL for malformed arguments, WCC_ECANCELLED after destroy began. */
int wcc_server_submit(wcc_server *srv, const wcc_job *job, int64_t *job_id);

/* Moves up to max completed results into out (host array); *n (host out) = how many. */
int wcc_server_poll(wcc_server *srv, wcc_result *out, int32_t max, int32_t *n);

/* Blocks until every submitted job has completed (WCC_ETIMEOUT after timeout_ms if
 * timeout_ms >= 0). */
int wcc_server_wait(wcc_server *srv, int64_t timeout_ms);

/* Lets running jobs finish, drops queued ones, joins the workers and frees every slot's
 * workspace.  Results not yet polled are discarded. */
int wcc_server_destroy(wcc_server *srv);

/* Text describing the last failing HIP call of this thread (empty if none). */
const char *wcc_last_error_detail(void);

/* Frees the library's workspace on the current device. */
int wcc_release(void);

/* ABI version of this header: 1. */
int wcc_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* WCC_H */
