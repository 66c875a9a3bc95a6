// Persistent batched launch of small jobs of every kind (see batch.hip).
#pragma once

#include <vector>

#include "common.h"
#include "pages.h"
#include "prof.h"

namespace schedk {

// Work of a batch runs in up to three phases, each one persistent launch
// pulling work items from its own counter; a phase starts when the previous
// launch has ended, so an item may read whatever the previous phase wrote.
//   phase 0: triads (fill, sweeps and digest, per chunk); histogram bins
//            zeroed; GEMM operands filled (one page per item)
//   phase 1: histogram key chunks (fill and count); GEMM output tiles
//   phase 2: histogram and GEMM digests (and the GEMM samples)
constexpr int BATCH_PHASES = 3;

struct BatchDesc {
  uint64_t o0, o1, o2;         // logical offsets (multiples of 4096) of the job's arrays:
                               // triad a, b, c; histogram keys, bins; GEMM A, B^T, C
                               // (GEMM arrays at page boundaries)
  int64_t n;                   // triad / histogram elements; GEMM: N
  uint64_t seed;               // input contents (SplitMix64 state seed << 32)
  int32_t iters;               // triad sweeps
  int32_t kind;                // SCHED_JOB_*
  unsigned long long *digest;  // += position-keyed digest of the output (pages.h)
  float *samples;              // GEMM: GEMM_SAMPLES sampled entries of C
  int32_t items[BATCH_PHASES]; // work items of each phase (batch_fill)
  int32_t pad;
};

// Header followed by max_desc descriptors and, per phase, max_desc + 1 item
// offsets; the pointers inside are valid in the address space of whoever
// reads the table.  The jobs of a batch share one placement, mapped by `map`.
struct BatchTable {
  int32_t n_desc;
  int32_t stride;              // max_desc + 1: distance between the phases' offset lists
  int64_t chunk;               // elements per streaming work item (a divisor of 16384)
  int64_t n_items[BATCH_PHASES];
  unsigned long long work[BATCH_PHASES];  // next work item of each phase
  BatchDesc *desc;
  int64_t *item_off;           // phase p, job j: first item at item_off[p * stride + j]
  PageMap map;
  int64_t need;                // pages the batch's jobs touch
  int32_t tile;                // GEMM output tile edge (64 or 128)
  int32_t pad;
  static size_t desc_offset() { return 256; }
  static size_t off_offset(int max_desc) { return 256 + sizeof(BatchDesc) * size_t(max_desc); }
  static size_t bytes_for(int max_desc) {
    return off_offset(max_desc) + 8 * size_t(BATCH_PHASES) * size_t(max_desc + 1);
  }
  static void layout_at(BatchTable *t, char *base, int max_desc) {
    t->desc = (BatchDesc *)(base + desc_offset());
    t->item_off = (int64_t *)(base + off_offset(max_desc));
    t->stride = max_desc + 1;
  }
  static void layout(BatchTable *t, int max_desc) { layout_at(t, (char *)t, max_desc); }
};
static_assert(sizeof(BatchTable) <= 256, "the descriptors start at byte 256");

struct BatchGraph {
  int block = 0, grid = 0, tile = 0, grid1 = 0, phases = 0;
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
  // phase 0 (streaming items): block, workgroups per CU, elements per item
  int block = 256, per_cu = 4;
  int64_t chunk = 1 << 14;
  int best_block = 256, best_per_cu = 4;
  // phase 1 (GEMM tiles, histogram chunks): tile edge, workgroups per CU
  int tile = 128, per_cu1 = 2;
  int phases = 1;                     // launches the filled batch needs (1 or 3)
  bool tuned = false;
  bool from_cache = false;     // the shapes were read from the tuner's cache file
  double tune_ms = 0.0, tune_gemm_ms = 0.0;
  std::vector<BatchGraph> graphs;
};

int batch_init(BatchEngine &b, int device, int max_desc);
void batch_free(BatchEngine &b);
// Fills the pinned table; descriptors' items[] are computed here.
int batch_fill(BatchEngine &b, const std::vector<BatchDesc> &descs, int64_t chunk, const PageMap &map,
               int64_t need);
int batch_launch(BatchEngine &b, hipStream_t s, bool use_graph);
int batch_autotune(BatchEngine &b, const char *cache_path, hipStream_t s);

}  // namespace schedk
