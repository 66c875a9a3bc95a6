// Persistent batched launch of small triad jobs (see batch.hip).
#pragma once

#include <vector>

#include "common.h"
#include "pages.h"
#include "prof.h"

namespace schedk {

struct BatchDesc {
  uint64_t oa, ob, oc;         // logical offsets (multiples of 4096) of output and inputs
  int64_t n;                   // elements
  uint64_t seed;               // input contents: SplitMix64 state seed << 32
  int32_t iters;               // triad sweeps
  int32_t pad;
  unsigned long long *digest;  // += position-keyed digest of a[] (pages.h)
};

// Header followed by max_desc descriptors and max_desc + 1 item offsets; the
// pointers inside are valid in the address space of whoever reads the table.
// The jobs of a batch share one placement, mapped by `map`.
struct BatchTable {
  int32_t n_desc;
  int32_t pad;
  int64_t n_items;
  int64_t chunk;               // elements per work item (a divisor of 16384)
  unsigned long long work;     // next work item
  BatchDesc *desc;
  int64_t *item_off;           // first work item of each job; [n_desc] = total
  PageMap map;
  int64_t need;                // pages the batch's jobs touch
  static size_t desc_offset() { return 128; }
  static size_t off_offset(int max_desc) { return 128 + sizeof(BatchDesc) * size_t(max_desc); }
  static size_t bytes_for(int max_desc) { return off_offset(max_desc) + 8 * size_t(max_desc + 1); }
  static void layout_at(BatchTable *t, char *base, int max_desc) {
    t->desc = (BatchDesc *)(base + desc_offset());
    t->item_off = (int64_t *)(base + off_offset(max_desc));
  }
  static void layout(BatchTable *t, int max_desc) { layout_at(t, (char *)t, max_desc); }
};
static_assert(sizeof(BatchTable) <= 128, "the descriptors start at byte 128");

struct BatchGraph {
  int block = 0, grid = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct BatchEngine {
  int device = 0;
  int max_desc = 0;
  BatchTable *h_table = nullptr;      // pinned, host view
  BatchTable *h_table_dev = nullptr;  // same memory, device view
  BatchTable *d_table = nullptr;      // device copy
  int cus = 0;
  int block = 256, per_cu = 4;
  int64_t chunk = 1 << 14;
  int best_block = 256, best_per_cu = 4;
  bool tuned = false;
  bool from_cache = false;     // the shape was read from the tuner's cache file
  double tune_ms = 0.0;
  std::vector<BatchGraph> graphs;
};

int batch_init(BatchEngine &b, int device, int max_desc);
void batch_free(BatchEngine &b);
int batch_fill(BatchEngine &b, const std::vector<BatchDesc> &descs, int64_t chunk, const PageMap &map,
               int64_t need);
int batch_launch(BatchEngine &b, hipStream_t s, bool use_graph);
int batch_autotune(BatchEngine &b, const char *cache_path, hipStream_t s);

}  // namespace schedk
