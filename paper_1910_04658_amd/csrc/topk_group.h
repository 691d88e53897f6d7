// Internal (C++) interface of the top-k pipeline for grouped execution: many
// independent query-vs-corpus problems of different sizes and widths run as
// one kernel launch per pipeline stage and kernel variant. Used by bs_topk (a
// group of one) and by the batched entry points.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "binsketch.h"

namespace bs {

// Tile-shape choices of the scan (0 or negative = the built-in heuristic).
struct TopkTune {
  int32_t qpl = 0;    // 64-query groups per wave of the query-lane scan (1, 2 or 4; 2 for N <= 1024, 4 for N <= 512)
  int32_t waves = 0;  // approximate waves of the scan grid (sets the corpus slab length)
  int32_t rows = -1;  // 0: never use the row-lane scan; otherwise it is used for batches of <= 64 queries
  int32_t mma = -1;   // 0: never use the matrix-core scan; otherwise it is used for N a multiple of 256
};

struct TopkItem {
  const uint64_t* Q;  // [nQ][N/64]
  const int32_t* popQ;
  int64_t nQ;
  const uint64_t* C;  // [nC][N/64]
  const int32_t* popC;
  int64_t nC;
  int32_t N, k;
  int32_t* out_idx;   // [nQ][k]
  float* out_score;   // [nQ][k] or null
  const float* t32;   // T(0..N), FP32 (shared by items of one width)
};

// Validates an item (the bs_topk argument rules, popcounts required).
bs_status topk_item_check(const TopkItem& it, int32_t measure);
// Device scratch of one item (256-byte aligned base).
size_t topk_item_workspace(int64_t nQ, int64_t nC, int32_t N, int32_t k, const TopkTune& tune);

struct TopkGroup;  // host-side plan of a group
// Device bytes for the group's argument blocks and block tables.
size_t topk_group_meta_bytes(int32_t n_items);
// Plans the group, uploads its argument blocks into `meta` (a synchronous
// copy) and returns a host object to launch from. item_ws[i] is item i's
// scratch (topk_item_workspace bytes).
bs_status topk_group_create(const TopkItem* items, const TopkTune* tunes, int32_t n_items, int32_t measure,
                            void* const* item_ws, void* meta, size_t meta_bytes, bool persistent,
                            TopkGroup** out);
// Enqueues every stage for every item (stage-major: all sample passes, then
// all scans, ...). `cls` < 0 runs every variant class, else only that class.
bs_status topk_group_launch(const TopkGroup* g, hipStream_t s, int32_t cls = -1);
int32_t topk_group_classes(const TopkGroup* g);
// Item indices of class `cls` (returns the count; fills up to `cap` entries).
int32_t topk_group_class_items(const TopkGroup* g, int32_t cls, int32_t* items, int32_t cap);
void topk_group_destroy(TopkGroup* g);

}  // namespace bs
