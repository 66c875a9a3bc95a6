// Host side of a context's state in one position-independent block (sizes
// and offsets only, no pointers).  It lives in private memory, or, once the
// context is shared, in a POSIX shared-memory object that every attached
// process maps (Sec. III-B: clients in separate processes share one
// structure; here the structure is this block plus the device arrays,
// opened by the other processes through HIP IPC handles).  A process-shared
// robust mutex plays the paper's file lock and a process-shared condition
// variable its user signals.
#pragma once

#include <hip/hip_runtime.h>
#include <pthread.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/cosched.h"

// Device arrays a shared context exports, in this order.
enum IpcArr : int {
  IPC_DEMAND = 0,
  IPC_JOB,
  IPC_PRIO,
  IPC_SEQ,
  IPC_DECISION,
  IPC_ADM_JOB,
  IPC_ADM_SEQ,
  IPC_RES,
  IPC_STATE,
  IPC_PRIO_OF_JOB,
  IPC_RUN_LIST,
  IPC_CTL,
  IPC_FLAGS,
  IPC_N
};

// A waiting request made with sched_admit.  key = seq + 1 (0: empty slot,
// -1: deleted), so zero-filled memory is an empty table.
struct SeqEntry {
  int64_t key;
  int32_t job;
  int32_t pad;
};

struct SharedHost {
  uint64_t magic;
  uint32_t version;
  int32_t shared;            // 1 once exported to other processes
  uint64_t bytes;            // size of the whole block
  pthread_mutex_t mu;
  pthread_cond_t cv;
  // configuration (what an attaching process needs)
  int32_t device, policy, window_limit, max_jobs;
  int64_t capacity, q_capacity, max_tiles;
  int32_t owner_pid, attached;  // process that created the context; live attachments
  char pci_bus_id[64];
  hipIpcMemHandle_t ipc[IPC_N];
  // scheduler state mirrored on the host
  int64_t head_h, tail_h, used_h, seq_next, last_A, rel_jobs_seen, rel_bytes_seen, last_adm_off;
  int32_t n_jobs, closing;
  sched_stats_t stats;
  int32_t prio_lo, prio_hi;
  int64_t prio_sorted_tail;
  uint64_t eng_launch;       // the admission engine's launch counter and look-back epoch
  uint32_t eng_epoch, pad1;
  int32_t n_owned, pad2;     // jobs whose owner process was set (owned[])
  int64_t req_cap, req_live, req_used;  // table slots (a power of two), live, live + deleted
  uint64_t off_prio, off_timeout, off_pending, off_owner, off_owned, off_req;

  int32_t *prio() { return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(this) + off_prio); }
  int32_t *timeout_ms() {
    return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(this) + off_timeout);
  }
  int32_t *pending() {
    return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(this) + off_pending);
  }
  int32_t *owner() { return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(this) + off_owner); }
  int32_t *owned() { return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(this) + off_owned); }
  SeqEntry *req() { return reinterpret_cast<SeqEntry *>(reinterpret_cast<char *>(this) + off_req); }

  // bytes a block for max_jobs jobs and a queue of q_cap entries takes
  static size_t size_for(int32_t max_jobs, int64_t q_cap);
  // lays a block out in zero-filled memory and initialises its mutex and
  // condition variable (process-shared when pshared)
  static SharedHost *init_at(void *zeroed, size_t bytes, int32_t max_jobs, int64_t q_cap,
                             bool pshared);
  // (re)initialises the mutex and condition variable in place
  static void init_sync(SharedHost *h, bool pshared);

  // waiting-request table
  bool req_contains(int64_t seq);
  bool req_put(int64_t seq, int32_t job);  // false when the table is full
  bool req_take(int64_t seq, int32_t *job);
  void req_erase_job(int32_t job);
  void req_clear();
  template <typename F>
  void req_for_each(F f) {
    SeqEntry *t = req();
    for (int64_t i = 0; i < req_cap; ++i)
      if (t[i].key > 0) f(t[i].key - 1, t[i].job);
  }
  bool req_empty() const { return req_live == 0; }

 private:
  void req_rebuild();
};

constexpr uint64_t SHARED_MAGIC = 0x53434845445348ULL;  // "SCHEDSH"
constexpr uint32_t SHARED_VERSION = 2;
