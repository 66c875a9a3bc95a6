"""Python binding of the co-scheduler C ABI (include/cosched.h).

Argument marshalling only: every function has the name of the C entry point
it calls, returns the C status code (plus out-values as a tuple), and passes
device memory as raw pointers taken from torch tensors.  All scheduling work
runs in the HIP library ``libsched.so``; there is no Python fallback, and the
first call raises if the library has not been built.

torch is imported before the library is loaded so that the process holds one
HIP runtime (torch's) and torch tensors/streams are valid in the library.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (must precede the library load)

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsched.so")

SCHED_OK = 0
SCHED_NOT_READY = 1
SCHED_TIMEOUT = 2
SCHED_E_INVALID = -1
SCHED_E_TOOBIG = -2
SCHED_E_QUOTA = -3
SCHED_E_NOMEM = -4
SCHED_E_INTERNAL = -5

SCHED_POLICY_FIFO = 0
SCHED_POLICY_MMU = 1
SCHED_POLICY_PRIO_FIFO = 2
SCHED_POLICY_PRIO_MMU = 3

SCHED_NONBLOCK = 1

i32, i64, u32, u64, vp = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64, C.c_void_p


class sched_config_t(C.Structure):
    _fields_ = [("device", i32), ("policy", i32), ("capacity_bytes", i64),
                ("headroom_bytes", i64), ("slab_pool_bytes", i64), ("max_jobs", i32),
                ("max_tenants", i32), ("queue_capacity", i64), ("window_limit", i32),
                ("flags", i32)]


class sched_stats_t(C.Structure):
    _fields_ = [(n, i64) for n in ("capacity", "used", "pending", "running", "passes", "rounds",
                                   "admitted", "released_bytes", "withdrawn", "violations",
                                   "slab_pool_used", "last_pass_ns")]


class sched_pass_result_t(C.Structure):
    _fields_ = [(n, i64) for n in ("admitted", "admitted_bytes", "free_before", "free_after",
                                   "rounds", "scanned", "pending_after", "compacted",
                                   "released", "released_bytes")]


class sched_scan_result_t(C.Structure):
    _fields_ = [(n, i64) for n in ("admitted", "admitted_bytes", "free_after", "rounds",
                                   "last_admitted")]


class sched_slab_info_t(C.Structure):
    _fields_ = [("pool_base", u64), ("pool_bytes", i64), ("region_bytes", i64),
                ("class_blocks", i64 * 13), ("n_classes", i32), ("n_tenants", i32)]


class sched_serve_opts_t(C.Structure):
    _fields_ = [("mode", i32), ("n_streams", i32), ("serial", i32), ("batch_small", i32),
                ("small_bytes", i64), ("iters", i32), ("digest", i32), ("time_scale", C.c_double),
                ("use_graph", i32), ("max_placed", i32), ("tune_cache", C.c_char_p)]


class sched_serve_summary_t(C.Structure):
    _fields_ = ([(n, C.c_double) for n in ("wall_s", "makespan_s", "jobs_per_s", "p50_wait_s",
                                             "p99_wait_s", "p50_turn_s", "p99_turn_s")]
                + [(n, i64) for n in ("completed", "rejected", "violations", "passes", "batches",
                                      "batched_jobs", "peak_used", "max_running", "tuned_block",
                                      "tuned_chunk", "tuned_per_cu")]
                + [(n, C.c_double) for n in ("host_pass_s", "host_launch_s", "host_poll_s",
                                             "host_idle_s", "dev_busy_s")]
                + [(n, i64) for n in ("tuned_from_cache", "slot_waits", "placements",
                                      "placement_slots", "pool_pages", "peak_pages", "pages_left",
                                      "charged_left", "page_check", "tuned_gemm_tile",
                                      "tuned_gemm_per_cu")])


SCHED_JOB_TRIAD = 0
SCHED_JOB_GEMM = 1
SCHED_JOB_HIST = 2
SCHED_SERVE_REALTIME = 0
SCHED_SERVE_VIRTUAL = 1

# numpy layout of sched_job_result_t
import numpy as _np  # noqa: E402

SCHED_GEMM_SAMPLES = 8
# numpy layout of sched_job_desc_t
JOB_DTYPE = _np.dtype([("arrival_s", "<f8"), ("vdur_s", "<f8"), ("demand", "<i8"), ("size", "<i8"),
                       ("kind", "<i4"), ("priority", "<i4"), ("seed", "<u8")])
RESULT_DTYPE = _np.dtype([("t_arrive", "<f8"), ("t_admit", "<f8"), ("t_place", "<f8"),
                          ("t_start", "<f8"), ("t_end", "<f8"), ("digest", "<u8"),
                          ("status", "<i4"), ("batched", "<i4"),
                          ("sample", "<f4", (SCHED_GEMM_SAMPLES,))])

# name -> (restype, argtypes); mirrors include/cosched.h
_SIGS = {
    "sched_create": (i32, [C.POINTER(sched_config_t), C.POINTER(vp)]),
    "sched_destroy": (i32, [vp]),
    "sched_register": (i32, [vp, i32, i32, C.POINTER(i32)]),
    "sched_register_batch": (i32, [vp, i32, i32, i32, C.POINTER(i32)]),
    "sched_admit": (i32, [vp, i32, i32, i64, u32]),
    "sched_wait": (i32, [vp, i32, i32]),
    "sched_release": (i32, [vp, i32, i32, i64]),
    "sched_stats": (i32, [vp, C.POINTER(sched_stats_t)]),
    "sched_reservation": (i32, [vp, i32, C.POINTER(i64)]),
    "sched_enqueue_batch": (i32, [vp, i64, vp, vp, vp]),
    "sched_pass": (i32, [vp, vp, C.POINTER(sched_pass_result_t)]),
    "sched_last_admitted": (i32, [vp, vp, i64, C.POINTER(i64), vp]),
    "sched_release_masked": (i32, [vp, vp, i64, vp]),
    "sched_pass_chain": (i32, [vp, i32, vp, i64, vp, vp, vp, i64]),
    "sched_enqueue_chain": (i32, [vp, i64, vp, vp, i32, vp, i64, vp, vp, vp, i64]),
    "sched_set_owner": (i32, [vp, i32, i32]),
    "sched_sanity_check": (i32, [vp, vp, vp]),
    "sched_checkpoint": (i32, [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]),
    "sched_restore": (i32, [vp, vp, C.c_size_t]),
    "sched_scan_workspace_size": (C.c_size_t, [i64]),
    "sched_set_lookback_polls": (i32, [i32]),
    "sched_scan_noalloc": (i32, [i32, i64, vp, i64, vp, i32, i32, vp, C.POINTER(sched_scan_result_t)]),
    "sched_scan": (i32, [i32, i64, vp, i64, vp, i32, i32, vp, C.c_size_t, vp,
                         C.POINTER(sched_scan_result_t)]),
    "sched_alloc": (i32, [vp, i32, C.c_size_t, C.POINTER(vp)]),
    "sched_free": (i32, [vp, i32, vp]),
    "sched_slab_set_quotas": (i32, [vp, i32, C.POINTER(i64)]),
    "sched_slab_ops": (i32, [vp, i64, i64, vp, vp, vp, vp, vp, vp, vp]),
    "sched_slab_info": (i32, [vp, C.POINTER(sched_slab_info_t)]),
    "sched_slab_counters": (i32, [vp, i32, C.POINTER(i64), C.POINTER(i64)]),
    "sched_slab_reset": (i32, [vp]),
    "sched_triad_fill": (i32, [vp, vp, i64, u64, vp]),
    "sched_triad": (i32, [vp, vp, vp, C.c_float, i64, i32, vp]),
    "sched_hist_fill": (i32, [vp, i64, u64, vp]),
    "sched_hist": (i32, [vp, i64, u32, vp, vp]),
    "sched_gemm_fill": (i32, [vp, i64, i64, u64, vp]),
    "sched_gemm_bf16": (i32, [vp, vp, vp, i64, i64, i64, vp]),
    "sched_reset": (i32, [vp]),
    "sched_profile": (i32, [i32]),
    "sched_profile_read": (i32, [C.c_char_p, C.POINTER(C.c_double), C.POINTER(i64)]),
    "sched_serve": (i32, [vp, i64, vp, C.POINTER(sched_serve_opts_t), vp,
                          C.POINTER(sched_serve_summary_t)]),
    "sched_version": (C.c_char_p, []),
    "sched_abi_sizeof": (i64, [i32]),
    "sched_share": (i32, [vp, C.c_char_p]),
    "sched_attach": (i32, [C.c_char_p, C.POINTER(vp)]),
}


def abi_layouts():
    """(library sizeof, binding sizeof) of every structure the ABI passes."""
    mine = [C.sizeof(sched_config_t), C.sizeof(sched_stats_t), C.sizeof(sched_pass_result_t),
            JOB_DTYPE.itemsize, RESULT_DTYPE.itemsize, C.sizeof(sched_serve_opts_t),
            C.sizeof(sched_serve_summary_t), C.sizeof(sched_slab_info_t),
            C.sizeof(sched_scan_result_t)]
    return [(int(lib().sched_abi_sizeof(k)), m) for k, m in enumerate(mine)]

_lib = None


def lib() -> C.CDLL:
    """Loads libsched.so once; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH}; run __graft_entry__.build()")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(s) -> int | None:
    if s is None:
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ---------------------------------------------------------------- life cycle
def sched_create(device=0, policy=SCHED_POLICY_MMU, capacity_bytes=0, headroom_bytes=0,
                 slab_pool_bytes=0, max_jobs=1024, max_tenants=0, queue_capacity=1 << 16,
                 window_limit=0):
    cfg = sched_config_t(device, policy, capacity_bytes, headroom_bytes, slab_pool_bytes,
                         max_jobs, max_tenants, queue_capacity, window_limit, 0)
    out = vp()
    rc = lib().sched_create(C.byref(cfg), C.byref(out))
    return rc, out.value


def sched_share(ctx, name):
    return lib().sched_share(ctx, name.encode())


def sched_attach(name):
    h = vp()
    rc = lib().sched_attach(name.encode(), C.byref(h))
    return rc, h.value


def sched_destroy(ctx):
    return lib().sched_destroy(ctx)


def sched_register(ctx, priority=0, timeout_ms=60000):
    j = i32()
    rc = lib().sched_register(ctx, priority, timeout_ms, C.byref(j))
    return rc, j.value


def sched_register_batch(ctx, n, priority=0, timeout_ms=60000):
    j = i32()
    rc = lib().sched_register_batch(ctx, n, priority, timeout_ms, C.byref(j))
    return rc, j.value


def sched_admit(ctx, job, device, nbytes, flags=0):
    return lib().sched_admit(ctx, job, device, nbytes, flags)


def sched_wait(ctx, job, timeout_ms=-1):
    return lib().sched_wait(ctx, job, timeout_ms)


def sched_release(ctx, job, device=-1, nbytes=0):
    return lib().sched_release(ctx, job, device, nbytes)


def sched_stats(ctx):
    s = sched_stats_t()
    rc = lib().sched_stats(ctx, C.byref(s))
    return rc, {k: getattr(s, k) for k, _ in sched_stats_t._fields_}


def sched_set_owner(ctx, job, pid):
    return lib().sched_set_owner(ctx, job, pid)


def sched_sanity_check(ctx):
    """Returns (rc, reclaimed_jobs, reclaimed_bytes)."""
    nj, nb = i64(), i64()
    rc = lib().sched_sanity_check(ctx, C.byref(nj), C.byref(nb))
    return rc, nj.value, nb.value


def sched_set_lookback_polls(polls):
    return lib().sched_set_lookback_polls(polls)


def sched_checkpoint(ctx):
    """Returns (rc, record bytes); the buffer is sized by the library's own
    size query first."""
    n = C.c_size_t()
    rc = lib().sched_checkpoint(ctx, None, 0, C.byref(n))
    if rc:
        return rc, b""
    buf = C.create_string_buffer(max(n.value, 1))
    rc = lib().sched_checkpoint(ctx, buf, n.value, C.byref(n))
    return rc, (buf.raw[: n.value] if rc == 0 else b"")


def sched_checkpoint_size(ctx):
    """Returns (rc, upper bound of the record's size)."""
    n = C.c_size_t()
    rc = lib().sched_checkpoint(ctx, None, 0, C.byref(n))
    return rc, n.value


def sched_restore(ctx, record: bytes):
    buf = C.create_string_buffer(bytes(record), len(record))
    return lib().sched_restore(ctx, buf, len(record))


def sched_reservation(ctx, job):
    v = i64()
    rc = lib().sched_reservation(ctx, job, C.byref(v))
    return rc, v.value


# ---------------------------------------------------------- device batched
def sched_enqueue_batch(ctx, d_job, d_demand, stream=None):
    n = 0 if d_job is None else int(d_job.numel())
    return lib().sched_enqueue_batch(ctx, n, _ptr(d_job), _ptr(d_demand), _stream(stream))


def sched_pass(ctx, stream=None):
    r = sched_pass_result_t()
    rc = lib().sched_pass(ctx, _stream(stream), C.byref(r))
    return rc, {k: getattr(r, k) for k, _ in sched_pass_result_t._fields_}


def sched_last_admitted(ctx, d_out, stream=None):
    n = i64()
    cap = 0 if d_out is None else int(d_out.numel())
    rc = lib().sched_last_admitted(ctx, _ptr(d_out), cap, C.byref(n), _stream(stream))
    return rc, n.value


def sched_release_masked(ctx, d_mask, stream=None):
    n = 0 if d_mask is None else int(d_mask.numel())
    return lib().sched_release_masked(ctx, _ptr(d_mask), n, _stream(stream))


def sched_pass_chain(ctx, rounds, d_masks=None, d_admitted=None, stream=None):
    """d_masks: uint8 device tensor [rounds - 1, n_mask] (or None)."""
    rc, arr = sched_pass_chain_array(ctx, rounds, d_masks, d_admitted, stream)
    return rc, [dict(zip(PASS_FIELDS, (int(v) for v in row))) for row in arr]


# column order of sched_pass_chain_array's rows
PASS_FIELDS = tuple(k for k, _ in sched_pass_result_t._fields_)


def sched_pass_chain_array(ctx, rounds, d_masks=None, d_admitted=None, stream=None):
    """As sched_pass_chain, with the results as one int64 array of shape
    [rounds, len(PASS_FIELDS)] (columns in PASS_FIELDS order)."""
    import numpy as np
    n_mask = 0 if d_masks is None else int(d_masks.shape[-1])
    res = np.zeros((rounds, len(PASS_FIELDS)), dtype=np.int64)
    cap = 0 if d_admitted is None else int(d_admitted.numel())
    rc = lib().sched_pass_chain(ctx, rounds, _ptr(d_masks), n_mask, _stream(stream),
                                res.ctypes.data,
                                _ptr(d_admitted), cap)
    return rc, res


def sched_enqueue_chain_array(ctx, d_job, d_demand, rounds, d_masks=None, d_admitted=None,
                              stream=None):
    """sched_enqueue_batch + sched_pass_chain in one call (one synchronisation);
    results as sched_pass_chain_array."""
    import numpy as np
    n = int(d_job.numel())
    assert int(d_demand.numel()) == n
    n_mask = 0 if d_masks is None else int(d_masks.shape[-1])
    res = np.zeros((rounds, len(PASS_FIELDS)), dtype=np.int64)
    cap = 0 if d_admitted is None else int(d_admitted.numel())
    rc = lib().sched_enqueue_chain(ctx, n, _ptr(d_job), _ptr(d_demand), rounds, _ptr(d_masks), n_mask,
                                   _stream(stream), res.ctypes.data, _ptr(d_admitted), cap)
    return rc, res


def sched_enqueue_chain(ctx, d_job, d_demand, rounds, d_masks=None, d_admitted=None, stream=None):
    rc, arr = sched_enqueue_chain_array(ctx, d_job, d_demand, rounds, d_masks, d_admitted, stream)
    return rc, [dict(zip(PASS_FIELDS, (int(v) for v in row))) for row in arr]


# ---------------------------------------------------------- stateless scan
def sched_scan_workspace_size(n):
    return int(lib().sched_scan_workspace_size(n))


def sched_scan(policy, d_demand, R, d_decision, write_all=0, window_limit=0, d_ws=None,
               ws_bytes=0, stream=None):
    r = sched_scan_result_t()
    n = int(d_demand.numel())
    rc = lib().sched_scan(policy, n, _ptr(d_demand), int(R), _ptr(d_decision), write_all,
                          window_limit, _ptr(d_ws), ws_bytes, _stream(stream), C.byref(r))
    return rc, {k: getattr(r, k) for k, _ in sched_scan_result_t._fields_}


def sched_scan_noalloc(policy, d_demand, R, d_decision, write_all=0, window_limit=0, stream=None):
    r = sched_scan_result_t()
    n = int(d_demand.numel())
    rc = lib().sched_scan_noalloc(policy, n, _ptr(d_demand), int(R), _ptr(d_decision), write_all,
                                  window_limit, _stream(stream), C.byref(r))
    return rc, {k: getattr(r, k) for k, _ in sched_scan_result_t._fields_}


# ---------------------------------------------------------- slab allocator
def sched_alloc(ctx, job, nbytes):
    p = vp()
    rc = lib().sched_alloc(ctx, job, nbytes, C.byref(p))
    return rc, p.value


def sched_free(ctx, job, ptr):
    return lib().sched_free(ctx, job, ptr)


def sched_slab_set_quotas(ctx, quotas):
    arr = (i64 * len(quotas))(*[int(q) for q in quotas])
    return lib().sched_slab_set_quotas(ctx, len(quotas), arr)


def sched_slab_ops(ctx, begin, end, d_kind, d_tenant, d_size, d_ref, d_ptr, d_status, stream=None):
    for t in (d_kind, d_tenant, d_size, d_ref, d_ptr, d_status):
        if t.numel() < end:
            raise ValueError("op arrays must hold at least `end` entries")
    return lib().sched_slab_ops(ctx, begin, end, _ptr(d_kind), _ptr(d_tenant), _ptr(d_size),
                                _ptr(d_ref), _ptr(d_ptr), _ptr(d_status), _stream(stream))


def sched_slab_info(ctx):
    r = sched_slab_info_t()
    rc = lib().sched_slab_info(ctx, C.byref(r))
    return rc, {"pool_base": r.pool_base, "pool_bytes": r.pool_bytes,
                "region_bytes": r.region_bytes, "class_blocks": list(r.class_blocks),
                "n_classes": r.n_classes, "n_tenants": r.n_tenants}


def sched_slab_counters(ctx, n):
    arr = (i64 * max(n, 1))()
    pool = i64()
    rc = lib().sched_slab_counters(ctx, n, arr, C.byref(pool))
    return rc, [arr[i] for i in range(n)], pool.value


def sched_slab_reset(ctx):
    return lib().sched_slab_reset(ctx)


# ---------------------------------------------------------- tenant jobs
SCHED_HIST_BINS = 4096


def sched_triad_fill(b, c, seed, stream=None):
    return lib().sched_triad_fill(_ptr(b), _ptr(c), int(b.numel()), seed, _stream(stream))


def sched_triad(a, b, c, s, iters=10, stream=None):
    return lib().sched_triad(_ptr(a), _ptr(b), _ptr(c), float(s), int(a.numel()), iters,
                             _stream(stream))


def sched_hist_fill(keys, seed, stream=None):
    return lib().sched_hist_fill(_ptr(keys), int(keys.numel()), seed, _stream(stream))


def sched_hist(keys, bins, mask=4095, stream=None):
    return lib().sched_hist(_ptr(keys), int(keys.numel()), mask, _ptr(bins), _stream(stream))


def sched_gemm_fill(x, rows, K, seed, stream=None):
    return lib().sched_gemm_fill(_ptr(x), rows, K, seed, _stream(stream))


def sched_gemm_bf16(A, Bt, Cout, M, N, K, stream=None):
    return lib().sched_gemm_bf16(_ptr(A), _ptr(Bt), _ptr(Cout), M, N, K, _stream(stream))


def sched_reset(ctx):
    return lib().sched_reset(ctx)


def sched_profile(enable):
    """True/1: clear the totals and start; 2: resume without clearing;
    False/0: stop (totals kept for sched_profile_read)."""
    return lib().sched_profile(int(enable) if enable in (0, 1, 2) else 1)


def sched_profile_read(kernel):
    ms = C.c_double()
    n = i64()
    rc = lib().sched_profile_read(kernel.encode(), C.byref(ms), C.byref(n))
    return rc, ms.value, n.value


# ---------------------------------------------------------- serving loop
def sched_serve(ctx, jobs, mode=SCHED_SERVE_REALTIME, n_streams=8, serial=0, batch_small=0,
                small_bytes=16 << 20, iters=10, digest=0, time_scale=1.0, use_graph=1,
                tune_cache=None, max_placed=0):
    """jobs: numpy structured array in the layout of sched_job_desc_t
    (workloads.job_table).  Returns (rc, results structured array, summary dict)."""
    jobs = _np.ascontiguousarray(jobs)
    assert jobs.dtype == JOB_DTYPE, jobs.dtype
    res = _np.zeros(jobs.shape[0], dtype=RESULT_DTYPE)
    o = sched_serve_opts_t(mode, n_streams, serial, batch_small, small_bytes, iters, digest,
                           time_scale, use_graph, max_placed,
                           tune_cache.encode() if tune_cache else None)
    sm = sched_serve_summary_t()
    rc = lib().sched_serve(ctx, jobs.shape[0], jobs.ctypes.data, C.byref(o), res.ctypes.data,
                           C.byref(sm))
    return rc, res, {k: getattr(sm, k) for k, _ in sched_serve_summary_t._fields_}


def sched_version():
    return lib().sched_version().decode()
