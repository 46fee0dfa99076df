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
  int32_t *cidv, *posv, *deg_in, *cursor;  // N each (posv: cluster-major position)
  void *tmp;
  size_t tmp_bytes;
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

// wcc_items.hip
int items_block();
int64_t items_lds_words(int64_t n, int cap);
int items_max_level();
int64_t items_bitmap_words(int64_t n, int cap);
int items_launch(const ItemArgs &A, int grid, size_t lds_bytes, hipStream_t s);
int items_level_words();
int items_ccr_init(const int32_t *mem, int64_t N, int32_t *out, hipStream_t s);
int items_level_prep(int32_t *ctl, int nx, hipStream_t s);
int items_route0(const ItemDesc *sorted, int32_t nitems, const int32_t *nbig, const FrontCounts *fc,
                 int32_t g_nitems, int32_t g_nbig, int32_t g_top, ItemDesc *lstS, ItemDesc *lstB, int32_t *ctl,
                 unsigned long long *cnt, hipStream_t s);
int items_sort_desc(const ItemDesc *in, int32_t n, ItemDesc *out, const int32_t *set_in, int32_t *set_out,
                    uint32_t *k1, uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes,
                    hipStream_t s, int small_max, int32_t *nbig);
int items_sort_desc_dev(const ItemDesc *in, int32_t cap, const int32_t *count, ItemDesc *out, uint32_t *k1,
                        uint32_t *v1, uint32_t *k2, uint32_t *v2, void *tmp, size_t tmp_bytes, hipStream_t s);
int items_relabel(const int32_t *acc, int64_t N, int32_t *mark, int32_t *rank, int32_t *out, void *tmp,
                  size_t tmp_bytes, hipStream_t s);
