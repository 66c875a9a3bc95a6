/*
 * cosched.h -- C ABI of the memory-safe GPU co-scheduler for one MI355X (gfx950).
 *
 * The scheduler decides which queued jobs may share the GPU so that the sum
 * of their declared memory demands never exceeds the device memory it
 * manages, then serves the admitted jobs (Reano, Silla, Nikolopoulos,
 * Varghese, "Intra-node Memory Safe GPU Co-Scheduling", IEEE TPDS 2017).
 * The life-cycle calls follow Sec. II and Sec. IV of the paper:
 *   initialisation -> sched_create + sched_register
 *   pre-allocation -> sched_admit (+ sched_wait when it has to wait)
 *   post-free      -> sched_release
 *   shutdown       -> sched_release(job, -1, 0) / sched_destroy
 * The waiting queue is served by one of the notification policies of Sec. V.
 *
 * Conventions for every call below:
 *   - the return value is a status code (SCHED_OK or one of the codes below);
 *     no C++ exception crosses this boundary;
 *   - out-parameters are written only when SCHED_OK is returned (unless a
 *     call states otherwise);
 *   - "device pointer" means memory on the context's GPU (hipMalloc or a
 *     torch CUDA tensor); "host pointer" means ordinary process memory;
 *   - a sched_stream_t is a hipStream_t of the context's device; NULL means
 *     the context's own stream.  Stream-ordered calls enqueue work and return
 *     before it finishes unless they say they synchronise;
 *   - every call taking a sched_ctx_t* is thread-safe per context (one mutex);
 *     calls on one context are serialised in the order they take the mutex.
 *   - all byte counts are int64, all demands are positive multiples of 1 B;
 *     the largest capacity a context accepts is 2^46 - 2 bytes.
 */
#ifndef COSCHED_H
#define COSCHED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define SCHED_OK 0
#define SCHED_NOT_READY 1   /* request queued, not admitted yet (Sec. IV: the
                               non-blocking pre-allocation result)           */
#define SCHED_TIMEOUT 2     /* blocking wait exceeded the job's timeout; the
                               request was withdrawn and is never admitted   */
#define SCHED_E_INVALID (-1) /* bad handle, device, size, or a release/free of
                                memory the job does not hold (Sec. IV checks) */
#define SCHED_E_TOOBIG (-2)  /* demand larger than the whole capacity        */
#define SCHED_E_QUOTA (-3)   /* allocation beyond the job's reservation      */
#define SCHED_E_NOMEM (-4)   /* sub-allocator pool or class exhausted        */
#define SCHED_E_INTERNAL (-5) /* HIP runtime failure (the paper's "unknown") */

/* ---- notification policies (Sec. V) ------------------------------------ */
#define SCHED_POLICY_FIFO 0       /* Policy 1: serve in queue order, stop at the first
                              waiting request that does not fit              */
#define SCHED_POLICY_MMU 1        /* Policy 2: serve, in queue order, every request
                              that fits the memory still free (first-fit)    */
#define SCHED_POLICY_PRIO_FIFO 2  /* Policy 3: FIFO over (priority, arrival) order  */
#define SCHED_POLICY_PRIO_MMU 3   /* Policy 4: MMU over (priority, arrival) order   */

/* sched_admit flags */
#define SCHED_NONBLOCK 1u  /* return SCHED_NOT_READY instead of waiting      */

typedef struct sched_ctx sched_ctx_t;
typedef int32_t sched_job_t;
typedef void *sched_stream_t;

typedef struct {
  int32_t device;          /* HIP device ordinal                               */
  int32_t policy;          /* SCHED_POLICY_FIFO .. SCHED_POLICY_PRIO_MMU                     */
  int64_t capacity_bytes;  /* managed memory; 0 = free device memory minus
                              headroom_bytes at creation                       */
  int64_t headroom_bytes;  /* kept back when capacity_bytes == 0               */
  int64_t slab_pool_bytes; /* slab sub-allocator pool; 0 = no pool            */
  int32_t max_jobs;        /* job handles [0, max_jobs)                        */
  int32_t max_tenants;     /* slab tenants with their own quota; 0 = max_jobs */
  int64_t queue_capacity;  /* pending requests the device queue holds         */
  int32_t window_limit;    /* windows of 256 entries the single-wave
                              admission kernel scans before the grid-wide
                              round kernel takes over; 0 = 64                  */
  int32_t flags;           /* reserved, 0                                      */
} sched_config_t;

typedef struct {
  int64_t capacity;        /* bytes managed                                    */
  int64_t used;            /* sum of reservations of running jobs (Sec. III-B) */
  int64_t pending;         /* entries in the queue: waiting requests, plus
                              withdrawn ones (timeouts, sanity checks) until
                              a pass that admits past them compacts them away */
  int64_t running;         /* jobs holding a reservation                       */
  int64_t passes;          /* admission passes run                             */
  int64_t rounds;          /* first-fit rounds run (all passes)                */
  int64_t admitted;        /* requests admitted (all passes)                   */
  int64_t released_bytes;  /* bytes released (all calls)                       */
  int64_t withdrawn;       /* requests withdrawn after a timeout               */
  int64_t violations;      /* allocation failures inside a job's reservation   */
  int64_t slab_pool_used;  /* bytes charged to the slab pool                   */
  int64_t last_pass_us_x1000; /* last pass, host-measured, in ns               */
} sched_stats_t;

/* Result of one admission pass. */
typedef struct {
  int64_t admitted;        /* requests admitted by this pass                   */
  int64_t admitted_bytes;  /* their total demand                               */
  int64_t free_before;     /* R at the start of the pass                       */
  int64_t free_after;      /* R at the end: free_before - admitted_bytes       */
  int64_t rounds;          /* first-fit rounds (1 for FIFO)                    */
  int64_t scanned;         /* queue entries the pass decided                   */
  int64_t pending_after;   /* requests still waiting                           */
  int64_t compacted;       /* queue entries the compaction step rewrote        */
  int64_t released;        /* jobs whose reservation reached 0 through
                              post-frees since the previous pass result (a
                              chain round's release step, or calls made
                              between two passes)                             */
  int64_t released_bytes;  /* bytes post-freed over the same span              */
} sched_pass_result_t;

/* ======================================================================== */
/* Life cycle (Sec. II, Sec. IV)                                             */
/* ======================================================================== */

/* Initialisation of the shared state (Sec. IV "Initialisation"): the context
 * owns the device-resident state -- capacity, used bytes, per-job
 * reservations and the waiting queue (Sec. III-B) -- and, if requested, the
 * slab pool.  cfg is read, not kept.  On success *out owns every resource
 * until sched_destroy.  Errors: SCHED_E_INVALID for a bad cfg,
 * SCHED_E_INTERNAL if a HIP allocation fails. */
int sched_create(const sched_config_t *cfg, sched_ctx_t **out);

/* Shutdown (Sec. IV "Shutdown"): waits for the context's stream, releases
 * every reservation and frees all device memory.  ctx is invalid afterwards.
 * Pointers returned by sched_alloc become invalid. */
int sched_destroy(sched_ctx_t *ctx);

/* schedGPUInit(timeout, priority) of Sec. IV: a new job handle with its
 * priority (lower value = higher priority; default 0) and the timeout in ms
 * a blocking pre-allocation waits (default 60000).  Errors: SCHED_E_INVALID
 * when max_jobs handles exist. */
int sched_register(sched_ctx_t *ctx, int32_t priority, int32_t timeout_ms, sched_job_t *out_job);

/* Registers n jobs with consecutive handles *out_first .. *out_first + n - 1. */
int sched_register_batch(sched_ctx_t *ctx, int32_t n, int32_t priority, int32_t timeout_ms,
                         sched_job_t *out_first);

/* Sharing a context between processes (Sec. III-B: clients in separate
 * processes share one structure; the paper's shared-memory approach).
 * sched_share publishes ctx under `name` (a POSIX shared-memory name such as
 * "/sched-demo"): the host side of the state moves into that shared-memory
 * object, guarded by a process-shared robust mutex and condition variable,
 * and the device arrays (queue, reservations, job states, control block,
 * look-back flags) are exported as HIP IPC handles (each allocation must be
 * under 2 GiB: queue_capacity <= 2^27).  Only a context without a slab pool
 * and with no request waiting can be shared; SCHED_E_INVALID otherwise, or
 * if the name exists.  The process that shared it destroys it last
 * (sched_destroy also removes the name).
 * sched_attach opens the context shared under `name` in another process (on
 * the device with the same PCI bus id) and returns a handle to it.  On a
 * shared or attached context the life-cycle calls (register, admit, wait,
 * release, set_owner, sanity_check, stats, reservation) and the pass entry
 * points (sched_pass, sched_enqueue_batch, sched_last_admitted) work across
 * processes: job handles are common to all, a request made in one process
 * can be admitted by a pass another runs, and a blocked waiter in any
 * process wakes up.  sched_serve, sched_pass_chain, sched_reset,
 * sched_checkpoint and sched_restore return SCHED_E_INVALID there.
 * sched_destroy on an attached handle detaches it. */
int sched_share(sched_ctx_t *ctx, const char *name);
int sched_attach(const char *name, sched_ctx_t **out);

/* Pre-allocation (Sec. IV): checks the device and the size, queues the
 * request behind the waiting ones, runs one admission pass of the context's
 * policy over the whole queue (Sec. V) and reports whether THIS request was
 * admitted.  A request larger than the capacity is refused with
 * SCHED_E_TOOBIG and never queued.  With SCHED_NONBLOCK a request that has
 * to wait returns SCHED_NOT_READY and stays queued (sched_wait can wait for
 * it later); without the flag the call waits up to the job's timeout like
 * sched_wait.  Errors: SCHED_E_INVALID (unknown job, device != the
 * context's device, bytes <= 0), SCHED_E_INTERNAL. */
int sched_admit(sched_ctx_t *ctx, sched_job_t job, int32_t device, int64_t bytes, uint32_t flags);

/* Blocks until every queued request of job is admitted (SCHED_OK) or
 * timeout_ms passes (SCHED_TIMEOUT; timeout_ms < 0 uses the job's own
 * timeout).  On timeout the job's waiting requests are withdrawn under the
 * context mutex, so a request is either admitted or withdrawn, never both.
 * SCHED_OK is returned at once when nothing of the job is waiting. */
int sched_wait(sched_ctx_t *ctx, sched_job_t job, int32_t timeout_ms);

/* Post-free (Sec. IV; postCudaFree(device, bytes)): returns bytes of the
 * job's reservation; bytes == 0 returns all of it; device < 0 means every
 * device.  Does not free GPU memory -- accounting only -- then runs one
 * admission pass to serve waiting requests.  Errors: SCHED_E_INVALID when
 * bytes exceeds the job's reservation, bytes < 0 or the device is not the
 * context's; nothing changes on error. */
int sched_release(sched_ctx_t *ctx, sched_job_t job, int32_t device, int64_t bytes);

/* Names the process that holds the job's memory (Sec. III-B keeps the
 * clients' processes in the shared state): pid > 0 makes the job subject to
 * the sanity check, pid = 0 exempts it (the default).  SCHED_E_INVALID for
 * an unknown job or pid < 0.  Host-side only. */
int sched_set_owner(sched_ctx_t *ctx, sched_job_t job, int32_t pid);

/* Sanity check (Sec. III-B, third robustness feature; Sec. IV): every job
 * whose owner process no longer exists (kill(pid, 0) fails with ESRCH) has
 * its waiting requests withdrawn and its whole reservation released, after
 * which one pass serves the waiting requests.  The library also runs it when
 * an admission does not fit, when a job releases everything (its shutdown)
 * and every 50 ms while a caller waits for memory.  *reclaimed_jobs and
 * *reclaimed_bytes (either may be NULL) receive what was reclaimed.
 * Synchronises. */
int sched_sanity_check(sched_ctx_t *ctx, int64_t *reclaimed_jobs, int64_t *reclaimed_bytes);

/* Returns the context to its state right after sched_create with every job
 * still registered: empty queue, no reservations, used = 0.  Slab blocks are
 * not touched (sched_slab_reset does that).  Does not wait for the device:
 * the reset kernels are ordered on the context's own stream.  Every later
 * call sees the reset state: calls that work on that stream (the batched
 * intake, passes and chains without a stream argument) follow it in stream
 * order, and every other call -- or one given another stream -- first waits
 * for the reset to finish. */
int sched_reset(sched_ctx_t *ctx);

/* Checkpoint (Sec. III-B, first robustness feature: a backup of the shared
 * state).  Writes into the caller's host buffer buf[0, cap) a self-contained
 * little-endian record of the admission state:
 *   header (64 B): magic "SCHEDCK1", version 1 (u32), policy (i32),
 *     capacity, used (i64), n_jobs (i32), 0 (i32), n_pending (i64),
 *     checksum (u64, FNV-1a 64 over the whole record with this field 0), 0;
 *   per registered job (24 B): priority, timeout_ms, owner pid, 0 (i32),
 *     reservation in bytes (i64);
 *   per waiting request (16 B): demand (i64), job, priority (i32), in the
 *     order the policy serves them: arrival order, or (priority, arrival)
 *     under the priority policies.  Withdrawn requests are left out.
 * *out_bytes receives the record's size.  buf = NULL asks for an upper bound
 * of that size (cap is ignored).  SCHED_E_INVALID if cap is too small;
 * SCHED_E_INTERNAL if the live state fails the integrity check of
 * sched_restore (then no record is handed out).  Slab blocks, counters and
 * the device's decision bytes are not part of it.  Work the caller queued on
 * its own streams (sched_enqueue_batch, sched_pass_chain) must be complete.
 * Synchronises. */
int sched_checkpoint(sched_ctx_t *ctx, void *buf, size_t cap, size_t *out_bytes);

/* Integrity check and recovery (Sec. III-B, second robustness feature;
 * Sec. IV, initialisation).  Loads a record written by sched_checkpoint into
 * ctx, which must be fresh: no job registered, an empty queue, the record's
 * policy and capacity, and room for its waiting requests in the queue.  The
 * record is checked first -- magic, version, size, checksum, every
 * reservation in [0, capacity] with their sum equal to the used total, every
 * request naming a job of the record with that job's priority and a demand
 * in [1, capacity] -- and a record that fails, or a context that is not
 * fresh, gives SCHED_E_INVALID with ctx untouched (the caller then keeps the
 * freshly initialised state).  On success the jobs get ids 0..n_jobs-1 with
 * their priority, timeout, owner and reservation, and the requests wait in
 * the record's order as if made by sched_admit: sched_wait works on them and
 * the next pass serves them.  Buffer owned by the caller.  Synchronises. */
int sched_restore(sched_ctx_t *ctx, const void *buf, size_t bytes);

/* Counters; see sched_stats_t. */
int sched_stats(sched_ctx_t *ctx, sched_stats_t *out);

/* The job's current reservation in bytes (host pointer out). */
int sched_reservation(sched_ctx_t *ctx, sched_job_t job, int64_t *out_bytes);

/* ======================================================================== */
/* Device-batched admission (the same state, driven with device arrays)     */
/* ======================================================================== */

/* Request intake: appends n requests (device arrays d_job[n], d_demand[n],
 * arrival order) at the queue tail, stream-ordered.  Every job must be
 * registered and every demand in [1, capacity]; the queue must have room.
 * Synchronises the stream to validate the batch; SCHED_E_INVALID on a bad
 * batch (nothing is appended). */
int sched_enqueue_batch(sched_ctx_t *ctx, int64_t n, const int32_t *d_job, const int64_t *d_demand,
                        sched_stream_t stream);

/* Runs one admission pass (Sec. V policy of the context) over the waiting
 * queue and writes the result to *out (host pointer).  The admitted requests
 * leave the queue (stable order kept for the rest), their demands are added
 * to their jobs' reservations and to the used total.  Synchronises the
 * stream.  The admitted jobs, in queue order, can be read with
 * sched_last_admitted. */
int sched_pass(sched_ctx_t *ctx, sched_stream_t stream, sched_pass_result_t *out);

/* Copies the job ids admitted by the last pass (queue order) into the
 * device array d_out[cap]; *out_n receives the count (which may exceed cap:
 * then only cap ids are copied).  Stream-ordered copy. */
int sched_last_admitted(sched_ctx_t *ctx, int32_t *d_out, int64_t cap, int64_t *out_n,
                        sched_stream_t stream);

/* `rounds` (1..256) release+admit rounds chained on the device with a single
 * host synchronisation at the end: round 0 is one pass; round r > 0 first
 * releases every running job j < n_mask whose byte d_masks[(r-1)*n_mask + j]
 * is non-zero (Sec. IV post-free with bytes == 0) and then runs one pass.
 * Every pass runs to completion in the single-wave window kernel.  out (host
 * array of `rounds`, may be NULL) receives each pass's result; the admitted
 * job ids of all rounds, concatenated in round and queue order, are copied to
 * the device array d_admitted[cap] (up to cap of them).  Not allowed while
 * requests made with sched_admit wait (SCHED_E_INVALID).  Synchronises. */
int sched_pass_chain(sched_ctx_t *ctx, int32_t rounds, const uint8_t *d_masks, int64_t n_mask,
                     sched_stream_t stream, sched_pass_result_t *out, int32_t *d_admitted,
                     int64_t cap);

/* sched_enqueue_batch of n requests (d_job[n], d_demand[n], device arrays)
 * followed by sched_pass_chain, with one synchronisation instead of two:
 * the chain is queued right behind the intake on the same stream and commits
 * the intake on the device.  An invalid batch (as sched_enqueue_batch
 * defines it) is refused whole: SCHED_E_INVALID, nothing is appended and no
 * round runs, so the context is as before the call.  Other arguments and
 * errors as for the two calls. */
int sched_enqueue_chain(sched_ctx_t *ctx, int64_t n, const int32_t *d_job, const int64_t *d_demand,
                        int32_t rounds, const uint8_t *d_masks, int64_t n_mask,
                        sched_stream_t stream, sched_pass_result_t *out, int32_t *d_admitted,
                        int64_t cap);

/* Post-free for many jobs at once: every running job j < n whose byte
 * d_mask[j] (device array of n bytes) is non-zero returns its whole
 * reservation (Sec. IV, bytes == 0).  n must not exceed the number of
 * registered jobs.  No pass runs; call sched_pass afterwards.
 * Stream-ordered. */
int sched_release_masked(sched_ctx_t *ctx, const uint8_t *d_mask, int64_t n, sched_stream_t stream);

/* ======================================================================== */
/* Stateless admission scan over a caller's array                           */
/* ======================================================================== */

typedef struct {
  int64_t admitted;        /* entries admitted                                 */
  int64_t admitted_bytes;  /* their sum                                        */
  int64_t free_after;      /* R minus admitted_bytes                           */
  int64_t rounds;          /* rounds run                                       */
  int64_t last_admitted;   /* index of the last admitted entry, -1 if none     */
} sched_scan_result_t;

/* Bytes of device workspace sched_scan needs for n entries: a control block,
 * a pass summary and one look-back flag per 4096-entry tile (+1). */
size_t sched_scan_workspace_size(int64_t n);

/* One pass of policy SCHED_POLICY_FIFO or SCHED_POLICY_MMU (Sec. V) over d_demand[n]
 * (device, int64, queue order; an entry < 0 is a withdrawn request that is
 * skipped) with free memory R (0 <= R <= 2^46 - 2).  Sets d_decision[i] = 1
 * for every admitted entry and writes 0 to entries it rejects; entries after
 * the point where the pass stopped are written only when write_all != 0, so
 * callers that read the whole vector either zero it first or pass
 * write_all = 1.  d_ws is device workspace of at least
 * sched_scan_workspace_size(n) bytes, 256-byte aligned (the call then
 * allocates nothing; it clears the part it uses on the stream first, so the
 * memory may hold anything; calls sharing one workspace must not overlap), or
 * NULL to use a workspace the library allocates and keeps for the device.
 * The pass runs in grid-wide rounds: a decoupled look-back scan, or, for a
 * FIFO scan in the library's own workspace (d_ws NULL), one round in three
 * launches (tile sums and candidate bits, the break found by one workgroup,
 * the decisions written from the bits); results are the same either way.
 * Single-workgroup windows are used first when window_limit > 0 (at most 2
 * under FIFO, whose first break ends the pass, so that a long admitted
 * prefix goes to the grid at streaming rate).
 * Synchronises the stream; *out is a host pointer.
 * Errors: SCHED_E_INVALID for bad sizes, policy or R. */
int sched_scan(int32_t policy, int64_t n, const int64_t *d_demand, int64_t R, uint8_t *d_decision,
               int32_t write_all, int32_t window_limit, void *d_ws, size_t ws_bytes,
               sched_stream_t stream, sched_scan_result_t *out);

/* sched_scan for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same pass with the same arguments and results, its
 * workspace a fixed device array the library holds on each GPU for the life
 * of the process, sized for n <= 2^28 entries (about 512 KiB); larger n is
 * SCHED_E_INVALID.  It calls no hipMalloc, hipFree or other allocating
 * routine.  Calls on one GPU share that array: the library runs them one at
 * a time (each returns after its kernels have finished), and the part of
 * the array a call uses is cleared on the stream first, so what an earlier
 * call left behind does not matter.  Synchronises the stream. */
int sched_scan_noalloc(int32_t policy, int64_t n, const int64_t *d_demand, int64_t R,
                       uint8_t *d_decision, int32_t write_all, int32_t window_limit,
                       sched_stream_t stream, sched_scan_result_t *out);

/* Look-back bound of the grid rounds (the HBM-bound part of a pass: a
 * single-pass prefix scan across workgroups, Sec. V policies).  A tile waits
 * for a predecessor's published sum at most `polls` polls (default 256),
 * then sums that predecessor's demands itself; results do not depend on it.
 * 0 makes every look-back compute missing sums at once (used by tests to
 * exercise that path).  Process-wide; applies to rounds launched afterwards.
 * SCHED_E_INVALID for polls < 0. */
int sched_set_lookback_polls(int32_t polls);

/* ======================================================================== */
/* Quota-checked slab sub-allocator                                          */
/* ======================================================================== */
/* Itemised use per client (Sec. III-B) carried down to blocks: every block a
 * tenant allocates is charged to it (and to the pool), and a free is accepted
 * only for a live block the tenant holds (the post-free check of Sec. IV).
 * Classes are powers of two from 256 B to 1 MiB; the pool (cfg
 * slab_pool_bytes) is split into 13 equal regions of whole MiB, one per class,
 * so class c holds region_bytes / (256 << c) blocks (class_blocks[c]).
 * Tenants are jobs unless sched_slab_set_quotas installs explicit quotas; a
 * job's quota is then its admitted reservation. */
typedef struct {
  uint64_t pool_base;       /* device address of region 0                      */
  int64_t pool_bytes;       /* accounting limit of the pool counter            */
  int64_t region_bytes;     /* bytes of each class region                      */
  int64_t class_blocks[13]; /* blocks each class can hold                      */
  int32_t n_classes;        /* 13                                              */
  int32_t n_tenants;        /* tenant ids [0, n_tenants)                       */
} sched_slab_info_t;

/* Allocates bytes for job: <= 1 MiB from the slab (charged the class size),
 * larger sizes from a separate device allocation charged in 4 KiB pages.  The
 * charge must fit the job's quota (its reservation): SCHED_E_QUOTA otherwise.
 * SCHED_E_NOMEM when the pool or the class is exhausted; for a job inside its
 * quota that is a memory-safety violation and is counted in sched_stats.
 * *dev_ptr (host pointer to a device address) is written only on SCHED_OK;
 * the block stays valid until sched_free or sched_destroy.  Synchronises. */
int sched_alloc(sched_ctx_t *ctx, sched_job_t job, size_t bytes, void **dev_ptr);

/* Returns a block job holds.  A pointer the job does not hold, or a second
 * free of one block, is SCHED_E_INVALID and changes nothing.  Synchronises. */
int sched_free(sched_ctx_t *ctx, sched_job_t job, void *dev_ptr);

/* Installs explicit quotas (host array h_quotas[n], bytes >= 0) for tenants
 * [0, n); tenants >= n get quota 0. */
int sched_slab_set_quotas(sched_ctx_t *ctx, int32_t n, const int64_t *h_quotas);

/* One phase of concurrent allocator ops [begin, end) on device arrays indexed
 * by global op index (each holds at least `end` entries): d_kind[i] 0 = alloc
 * of d_size[i] bytes, 1 = free of the block returned by alloc op d_ref[i]
 * (which must belong to an earlier phase, i.e. d_ref[i] < begin); d_tenant[i]
 * the tenant.  Writes d_ptr[i] (the block of a successful alloc, else 0) and
 * d_status[i]: 0 ok, 1 over quota, 2 pool exhausted, 3 class exhausted,
 * 4 invalid.  Ops of one call run concurrently in any order.  Stream-ordered. */
int sched_slab_ops(sched_ctx_t *ctx, int64_t begin, int64_t end, const uint8_t *d_kind,
                   const int32_t *d_tenant, const int64_t *d_size, const int64_t *d_ref,
                   uint64_t *d_ptr, int8_t *d_status, sched_stream_t stream);

/* Layout of the pool; *out is a host pointer. */
int sched_slab_info(sched_ctx_t *ctx, sched_slab_info_t *out);

/* Copies the first n tenants' charged bytes and the pool counter to host
 * memory (synchronises the context stream first). */
int sched_slab_counters(sched_ctx_t *ctx, int32_t n, int64_t *h_charged, int64_t *h_pool_used);

/* Frees every block and clears all charges. */
int sched_slab_reset(sched_ctx_t *ctx);

/* ======================================================================== */
/* Synthetic tenant jobs                                                     */
/* ======================================================================== */
/* The paper co-schedules third-party applications (Sec. VI); the jobs here
 * are three synthetic kinds with plain definitions.  Contents come from
 * SplitMix64 (Steele, Lea, Flood 2014) with state seed << 32: output i is
 * h_i.  All pointers are device pointers; every call is stream-ordered on
 * `stream` (NULL = the null stream) and returns SCHED_E_INVALID for bad
 * sizes, NULL or misaligned pointers. */
#define SCHED_HIST_BINS 4096

/* b[i] = 1 + (h_i & 0xFFFF) / 2^16, c[i] = 1 + ((h_i >> 16) & 0xFFFF) / 2^16. */
int sched_triad_fill(float *b, float *c, int64_t n, uint64_t seed, sched_stream_t stream);

/* iters sweeps of the STREAM triad a[i] = b[i] + s * c[i] over n fp32
 * elements, one kernel launch per sweep.  a, b, c 16-byte aligned. */
int sched_triad(float *a, const float *b, const float *c, float s, int64_t n, int32_t iters,
                sched_stream_t stream);

/* keys[i] = low 32 bits of h_i. */
int sched_hist_fill(uint32_t *keys, int64_t n, uint64_t seed, sched_stream_t stream);

/* bins[b] = #{i : (keys[i] & mask) == b} for SCHED_HIST_BINS bins; bins is
 * zeroed by the call; mask < SCHED_HIST_BINS (4095: all bins; 63: the skewed
 * case); keys 16-byte aligned. */
int sched_hist(const uint32_t *keys, int64_t n, uint32_t mask, uint32_t *bins,
               sched_stream_t stream);

/* x[r * K + k] = bf16 bits of ((h_{r*K+k} & 255) - 128) / 64 (exact). */
int sched_gemm_fill(uint16_t *x, int64_t rows, int64_t K, uint64_t seed, sched_stream_t stream);

/* C[m * N + n] = sum_k A[m * K + k] * Bt[n * K + k]: bf16 inputs (raw bits),
 * fp32 accumulation on MFMA, fp32 output.  M and N multiples of 128, K a
 * multiple of 64; A and Bt 16-byte aligned. */
int sched_gemm_bf16(const uint16_t *A, const uint16_t *Bt, float *C, int64_t M, int64_t N,
                    int64_t K, sched_stream_t stream);

/* ======================================================================== */
/* Serving loop: admission + concurrent execution of a job mix               */
/* ======================================================================== */
/* The life cycle of Sec. II for every job of a mix: a job arrives, declares
 * its demand (pre-allocation, Sec. IV), waits in the queue until the policy
 * of the context (any of the four of Sec. V) admits it,
 * runs concurrently with the other admitted jobs, and returns its
 * reservation when it ends (post-free).  Jobs run on a pool of streams; with
 * batch_small, admitted jobs of every kind under small_bytes are packed into
 * one persistent batched launch (a HIP graph replay when use_graph): a
 * streaming phase, then, when the batch holds histograms or GEMMs, a phase of
 * key chunks and GEMM output tiles and a phase of digests.  Its block, chunk,
 * workgroups per CU and GEMM tile edge come from an autotuner (cached in
 * tune_cache when non-NULL).
 *
 * Memory: right after the pass that admits it, a job (or a batch of small
 * ones) is placed in a device page pool of 64 KiB pages: its buffers (each
 * rounded up to 4 KiB, at most its declared demand) are charged to the job
 * against its reservation -- the slab's per-tenant counters, tenants = jobs
 * -- and mapped page by page, so no contiguous range is needed.  The pool
 * holds the capacity plus one page per placement slot (max_placed, default
 * min(n, 16384)); an admitted job waits for a slot only when all are taken
 * (slot_waits).  A placement that fails for an admitted job is a
 * memory-safety violation (counted; the job's status is SCHED_E_NOMEM and
 * its work does nothing).  The context's slab, if it has one, must have
 * tenants = jobs with reservations as quotas; a context without one gets a
 * small one.  A GEMM job's N must be a power of two in [256, 16384]. */
#define SCHED_JOB_TRIAD 0  /* size = fp32 elements per array (3 arrays)       */
#define SCHED_JOB_GEMM 1   /* size = N of an N x N x N bf16 GEMM               */
#define SCHED_JOB_HIST 2   /* size = uint32 keys                              */

#define SCHED_SERVE_REALTIME 0 /* arrivals at their timestamps, real durations */
#define SCHED_SERVE_VIRTUAL 1  /* event order (time, releases first, job index),
                                  one pass per event, end = admit + vdur_s;
                                  no job work runs                             */

typedef struct {
  double arrival_s;   /* arrival, seconds from the start; non-decreasing      */
  double vdur_s;      /* duration in the virtual-clock mode                   */
  int64_t demand;     /* declared bytes (>= what the kind allocates)          */
  int64_t size;       /* kind's size parameter                                */
  int32_t kind;       /* SCHED_JOB_*                                          */
  int32_t priority;   /* lower value = higher priority                        */
  uint64_t seed;      /* input contents                                       */
} sched_job_desc_t;

#define SCHED_GEMM_SAMPLES 8

typedef struct {
  double t_arrive;    /* seconds from the start                               */
  double t_admit;     /* when the pass that admitted it returned              */
  double t_place;     /* when its placement was issued (>= t_admit)           */
  double t_start;     /* device time its work could start                     */
  double t_end;       /* device time its work ended                           */
  /* with digest: sum over the output's 32-bit words w_i of (s_i | 1) * w_i
   * mod 2^64, s_i = SplitMix64 output i for state 0x6A09E667F3BCC908 (the
   * triad's a, the GEMM's C in row-major order, the 4096 histogram bins)    */
  uint64_t digest;
  int32_t status;     /* SCHED_OK, SCHED_E_TOOBIG, SCHED_E_NOMEM, ...         */
  int32_t batched;    /* 1 if it ran inside a batched launch                  */
  /* with digest, GEMM jobs: C's element p_k (row-major) for k < 8, p_k =
   * (SplitMix64 output k for state (seed << 32) ^ 0xBB67AE8584CAA73B) mod N^2 */
  float sample[SCHED_GEMM_SAMPLES];
} sched_job_result_t;

typedef struct {
  int32_t mode;        /* SCHED_SERVE_REALTIME / SCHED_SERVE_VIRTUAL           */
  int32_t n_streams;   /* stream pool for single-job launches; without
                          batching capped at the hardware queues
                          (GPU_MAX_HW_QUEUES, default 4) left after the
                          control stream and one queue for the runtime's own
                          work; each job goes to the stream with the least
                          nominal work still in flight                        */
  int32_t serial;      /* 1: every demand := capacity (exclusive execution)   */
  int32_t batch_small; /* 1: persistent batched launch for small jobs          */
  int64_t small_bytes; /* demand threshold for batching                       */
  int32_t iters;       /* triad sweeps per job                                 */
  int32_t digest;      /* 1: compute each job's output digest                  */
  double time_scale;   /* arrival times are multiplied by this (0 = 1)         */
  int32_t use_graph;   /* 1: replay the batched launch as a HIP graph          */
  int32_t max_placed;  /* placement slots (0: min(n, 16384))                   */
  const char *tune_cache; /* JSON file for the autotuner result, or NULL       */
} sched_serve_opts_t;

typedef struct {
  double wall_s;       /* host time of the whole run                           */
  double makespan_s;   /* last job end                                         */
  double jobs_per_s;   /* completed / makespan                                 */
  /* nearest rank; wait = placement - arrival, turnaround = end - arrival    */
  double p50_wait_s, p99_wait_s, p50_turn_s, p99_turn_s;
  int64_t completed, rejected, violations, passes, batches, batched_jobs;
  int64_t peak_used, max_running;
  int64_t tuned_block, tuned_chunk, tuned_per_cu;
  /* where the controller's host time went (real-time mode), in seconds:
   * admission passes, launches of admitted work, completion polling and
   * releases, and idle waits; dev_busy_s is the time at least one job was
   * running on the device (union of the jobs' [start, end] intervals) */
  double host_pass_s, host_launch_s, host_poll_s, host_idle_s, dev_busy_s;
  int64_t tuned_from_cache; /* batching: 1 = shape read from tune_cache, 0 = the
                               tuner timed its candidates in this run; -1 = no
                               batching                                         */
  /* page pool (real-time mode) */
  int64_t slot_waits;      /* admitted jobs that waited for a placement slot  */
  int64_t placements;      /* placements made (a batch is one)                */
  int64_t placement_slots, pool_pages, peak_pages;
  int64_t pages_left, charged_left; /* at the end: both 0                     */
  int64_t page_check;      /* free-list entries duplicated or out of range at
                              the end (0), -1 if placements were left          */
  /* batching: the autotuned GEMM output tile edge (64 or 128) and workgroups
   * per CU of the batch's tile phase */
  int64_t tuned_gemm_tile, tuned_gemm_per_cu;
} sched_serve_summary_t;

/* Runs n jobs (jobs[i] is job handle i; the context needs max_jobs >= n and
 * is reset first) and fills results[n] and *summary (host pointers).
 * Synchronises; the context mutex is held for the whole run.  Errors:
 * SCHED_E_INVALID for bad descriptors. */
int sched_serve(sched_ctx_t *ctx, int64_t n, const sched_job_desc_t *jobs,
                const sched_serve_opts_t *opts, sched_job_result_t *results,
                sched_serve_summary_t *summary);

/* ======================================================================== */
/* Kernel timing                                                             */
/* ======================================================================== */
/* enable == 1 clears the totals and starts bracketing every library kernel
 * launch with a pair of HIP events on the launch's stream; 2 resumes
 * bracketing without clearing (to sample some calls of a timed loop); 0
 * stops it and keeps the totals for sched_profile_read. */
int sched_profile(int32_t enable);

/* Total device time in ms and launch count of the kernel named `kernel`
 * (k_window, k_round, k_compact, k_release_masked, k_triad, k_hist,
 * k_gemm_bf16, k_slab_phase, ...) since sched_profile(1), over the bracketed
 * launches only.  Waits for the
 * recorded events. */
int sched_profile_read(const char *kernel, double *total_ms, int64_t *launches);

/* Library version string. */
const char *sched_version(void);

/* sizeof of the ABI's structures, for bindings to check their layouts: 0
 * sched_config_t, 1 sched_stats_t, 2 sched_pass_result_t, 3
 * sched_job_desc_t, 4 sched_job_result_t, 5 sched_serve_opts_t, 6
 * sched_serve_summary_t, 7 sched_slab_info_t, 8 sched_scan_result_t; -1 for
 * any other value.  Touches no device. */
int64_t sched_abi_sizeof(int32_t which);

#ifdef __cplusplus
}
#endif

#endif /* COSCHED_H */
