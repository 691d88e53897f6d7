// Internal (C++) interface for sketching many independent CSR matrices (each
// with its own map, width and size) in one kernel launch.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

#include "binsketch.h"

namespace bs {

struct SketchItem {
  const int32_t* indptr;   // [n_rows + 1]
  const int32_t* indices;  // [nnz]
  int64_t n_rows, nnz;
  const int32_t* pi;       // [d]
  int64_t d;
  int32_t N;
  uint64_t* sketches;      // [n_rows][N/64]
  int32_t* popcounts;      // [n_rows] or null
  int32_t* err;            // error flag word or null
  uint16_t* pi16;          // scratch for the map as 16-bit targets ([d], packed by the launch), or null
};

// Validates an item (the bs_sketch argument rules).
bs_status sketch_item_check(const SketchItem& it);
struct SketchGroup;
// Device bytes for the argument blocks and the window table.
size_t sketch_group_meta_bytes(int32_t n_items);
// Plans the launch and uploads its tables into `meta` (a synchronous copy).
bs_status sketch_group_create(const SketchItem* items, int32_t n_items, void* meta, size_t meta_bytes,
                              bool persistent, SketchGroup** out);
bs_status sketch_group_launch(const SketchGroup* g, hipStream_t s);
void sketch_group_destroy(SketchGroup* g);

}  // namespace bs
