// wcc_internal.h -- declarations shared between the translation units of the library.
#pragma once

#include "wcc_common.h"

// Inputs and scratch of the front end (grouping and compaction).
struct FrontBufs {
  const void *off;
  int obits;
  const int32_t *idx;
  const int32_t *mem;
  int64_t N, nnz;
  uint32_t *keys, *vals, *keys2, *vals2;   // N each
  int32_t *flag, *flag_scan;               // N each
  int32_t *cidv, *posv, *deg_in;          // N each (posv: cluster-major position)
  int32_t *stage;                          // nnz words: intra entries by original row
  void *tmp;
  size_t tmp_bytes;
  int32_t *vtab_a, *vtab_b;                // validation: nnz words each (duplicate tables)
  unsigned long long *dcnt;                // >= 8 device counters
  int32_t *dmax;
};

// Device-resident sizes produced by the front end.
struct FrontCounts {
  int64_t na;      // vertices with a cluster
  int64_t K;       // clusters
  int64_t E;       // directed entries of all induced cluster subgraphs
  int32_t K32;     // cluster count as written by the scan
  int32_t maxid;   // largest cluster id, -1 if none
  int32_t nitems;  // initial items
  int32_t pad[3];
};

// wcc_front.hip
int front_validate(const FrontBufs &f, hipStream_t s, int *ok);
int front_build(const FrontBufs &f, FrontCounts *fc, int32_t *vtx0, int64_t *cl_start, int32_t *cl_ids,
                int32_t *rd0, int64_t *rs0, int32_t *adj0, ItemDesc *items, int32_t *item_set, bool all_items,
                hipStream_t s);
int front_split_membership(const int32_t *verts, const int64_t *set_offsets, int32_t num_sets, int64_t nv,
                           int64_t N, int32_t *mem, unsigned long long *bad, hipStream_t s);

// What decides an item's size bin: its scan-state size with the cut cap of its criterion
// (WCC) or of its caller's set (caps indexed by set[i]), against the small-bin LDS words.
struct SortNeed {
  int32_t crit, lin_num, lin_den;
  const int32_t *caps;  // mincut_split: caps per set (nullptr: k(n) of the criterion)
  const int32_t *set;   // set of each item (filled in by items_sort_desc)
  int64_t small_words;
};

// wcc_items.hip
int items_block();
int items_launch(const ItemArgs &A, int grid, size_t lds_bytes, hipStream_t s);
int items_level_words();
int items_ccr_init(const int32_t *mem, int64_t N, int32_t *out, hipStream_t s);
int items_level_prep(int32_t *ctl, int nx, hipStream_t s);
int items_route0(const ItemDesc *sorted, int32_t nitems, const int32_t *nbig, const FrontCounts *fc,
                 int32_t g_nitems, int32_t g_nbig, int32_t g_top, ItemDesc *lstS, ItemDesc *lstB, int32_t *ctl,
                 unsigned long long *cnt, hipStream_t s);
int items_sort_desc(const ItemDesc *in, int32_t n, ItemDesc *out, const int32_t *set_in, int32_t *set_out,
                    uint32_t *k1, uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes,
                    hipStream_t s, const SortNeed &nd, int32_t *sz);
int items_sort_desc_dev(const ItemDesc *in, int32_t cap, const int32_t *count, ItemDesc *out, uint32_t *k1,
                        uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes, hipStream_t s);
int items_relabel(const int32_t *acc, int64_t N, int32_t *mark, int32_t *rank, int32_t *out, void *tmp,
                  size_t tmp_bytes, hipStream_t s);

// wcc_cm.hip (Connectivity Modifier levels and the label-propagation CDA)
int cm_set_keys(const int32_t *cur, int64_t N, uint32_t *keys, uint32_t *vals, int32_t *nv, hipStream_t s);
int cm_sets(const uint32_t *skeys, const uint32_t *svals, int64_t cap, const int32_t *nv, int32_t *flag,
            int32_t *fscan, int32_t *nsets, int64_t *set_off, int32_t *verts, int32_t *setidx, int32_t *setof,
            void *tmp, size_t tmp_bytes, hipStream_t s);
int cm_caps(const int64_t *set_off, const int32_t *nsets, int64_t cap, const wcc_params &p, int32_t *caps,
            int32_t *has_edge, int32_t *ssize, unsigned long long *shash, int32_t *psize, int32_t *pmin,
            hipStream_t s);
int cm_edges(const wcc_csr *g, const int32_t *verts, const int32_t *setidx, const int32_t *setof,
             const int32_t *nv, int64_t cap, int32_t *has_edge, hipStream_t s);
int cm_outcome(const int64_t *set_off, const int32_t *verts, const int32_t *setidx, const uint8_t *sides,
               const int32_t *nv, const int32_t *nsets, int64_t cap, const int32_t *has_edge, const int32_t *caps,
               const int32_t *lam, int32_t *ssize, unsigned long long *shash, int32_t *psize, int32_t *pmin,
               int32_t s_post, int32_t *acc, int32_t *part_of, int32_t *nparts, wcc_record *rec, int64_t rec_cap,
               unsigned long long *cnt, hipStream_t s);
int cm_part_count(const int32_t *part_of, int64_t N, int32_t *flag, int32_t *fscan, int32_t *np, void *tmp,
                  size_t tmp_bytes, hipStream_t s);
int cm_next(const int32_t *part_of, const int32_t *comm, int64_t N, int32_t s_post, int comm_bits, int32_t *cur,
            const int32_t *fscan, const int32_t *np, int np_host, uint32_t *k1, uint32_t *v1, uint32_t *k2,
            uint32_t *v2, int32_t *ncomm, int32_t *run_flag, int32_t *run_scan, int32_t *run_start,
            int32_t *run_size, int32_t *nruns, void *tmp, size_t tmp_bytes, hipStream_t s);
int cm_ccr_gate(const int32_t *comp, int64_t N, int32_t gate, int32_t *cnt, int32_t *cur, hipStream_t s);
int lp_prepare(const int64_t *rs0, const int32_t *rd0, const int32_t *vtx0, const int32_t *cidv,
               const int64_t *cl_start, const int32_t *adj0, const int64_t *na_p, int64_t na_cap, int32_t *erow,
               int32_t *enb, int32_t *lab, hipStream_t s);
int lp_round(const int64_t *rs0, const int32_t *rd0, const int32_t *erow, const int32_t *enb, const int64_t *na_p,
             int64_t na_cap, const int64_t *E_p, int64_t E_host, int bits, int32_t *lab, int32_t *lab_new,
             uint32_t *k1, uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes, hipStream_t s);
int lp_out(const int32_t *vtx0, const int32_t *lab, const int64_t *na_p, int64_t na_cap, int32_t *comm,
           hipStream_t s);
