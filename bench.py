#!/usr/bin/env python3
"""Benchmark of the co-scheduler hot path on one MI355X.

Default workload (the admission microbenchmark): a queue of 2^20 pending
requests whose demands are log-uniform in [4 KiB, 4 GiB) (4 KiB aligned),
capacity 280e9 B, first-fit admission (FIFO prefix + backfill, the paper's
MMU policy), 8 rounds of "release a coin-chosen half of the running jobs,
then one admission pass".  One step = reset + intake of the 2^20 requests +
the 8 release/admit rounds; inputs are resident in HBM before timing.

Prints one JSON line.  `value` is admissions per second over the timed
steps.  `roofline` reports the dominant kernel of the step with its
algorithmic bytes per launch over its event-timed average duration;
`cpu_baseline` is the CPU oracle timed on the host on the same workload;
`dense_scan` reports the HBM-bound variant (one first-fit pass that reads a
2^26-entry queue) against the HBM peak.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "jobs/s + p99 turnaround, co-scheduled vs serial; admissions/s (GB/s of HBM)"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--queue-log2", type=int, default=20)
    ap.add_argument("--dense-log2", type=int, default=26)
    ap.add_argument("--dense-reps", type=int, default=10)
    ap.add_argument("--dense-sweep", default="24,26,28",
                    help="log2 sizes of the C2-D sweep (FIFO pass deciding every entry, and "
                         "first fit over 64 MiB-4 GiB demands); empty = none")
    ap.add_argument("--dense-window", type=int, default=64,
                    help="single-wave windows before the grid rounds take over")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="bound on the oracle's CPU time for cpu_baseline (0 = skip)")
    ap.add_argument("--no-profile", action="store_true",
                    help="time the steps without kernel events (no roofline)")
    ap.add_argument("--profile-every", type=int, default=5,
                    help="bracket the kernels of every n-th timed step with HIP events "
                         "(events cost time of their own; 1 = every step)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run a plain device-to-device copy of this many MiB first (the "
                         "known-size reference for hardware byte counters)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="no GPU run: turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, then "
                         "WRITE_SIZE) of a run with --copy-calib-mib into the traffic record "
                         "of --traffic-kernel under profiles/")
    ap.add_argument("--traffic-kernel", default="k_chain")
    ap.add_argument("--extras", default="dense,tenants,slab",
                    help="measurements to add after the admission steps (dense, tenants, "
                         "slab; empty = none)")
    ap.add_argument("--cosched", default="c1,c4,c5,hol",
                    help="co-scheduled vs serial runs to add (c1, c4, c5; hol = the "
                         "head-of-line study, FIFO vs MMU; empty = none)")
    ap.add_argument("--cosched-streams", type=int, default=3,
                    help="HIP streams for single-job launches in the co-scheduled runs (with "
                         "more streams than the process's hardware queues, the scheduler's "
                         "own stream shares a queue with job kernels and its passes wait "
                         "behind them)")
    ap.add_argument("--c5-jobs", type=int, default=50_000)
    ap.add_argument("--c4-jobs", type=int, default=10_000)
    ap.add_argument("--tune-cache", default="",
                    help="file for the batch autotuner's result (default: one per GPU "
                         "architecture and batch-kernel source hash in the temp directory)")
    return ap.parse_args()


def tune_cache_path(torch):
    """The autotuner's cache file, keyed by GPU architecture and by the hash of
    the batch kernel's source, so a changed kernel or another GPU tunes again."""
    import tempfile
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    sha = _sha256("paper_1712_04495_amd/csrc/batch.hip")[:16]
    return os.path.join(tempfile.gettempdir(), f"cosched_batch_tune_{arch}_{sha}.json")


def cosched_run(cs, name, n_jobs, dev_free, n_streams=3, tune_cache=""):
    """One job mix co-scheduled (MMU, batching of small triads) and exclusive
    serial (every demand := capacity).  Returns a dict of results."""
    import numpy as np
    from workloads import c1_jobs, c4_jobs, c5_jobs, job_table
    if name == "c1":
        mix = c1_jobs(1)
        policy, batch = cs.SCHED_POLICY_FIFO, 0
    elif name == "c4":
        cap = min(280 * 10**9, dev_free - (8 << 30))
        mix = c4_jobs(4, n=n_jobs, capacity=cap)
        policy, batch = cs.SCHED_POLICY_MMU, 0
    else:
        cap = min(280 * 10**9, dev_free - (8 << 30))
        mix = c5_jobs(5, n=n_jobs, capacity=cap)
        policy, batch = cs.SCHED_POLICY_MMU, 1
    jt = job_table(mix)
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=mix.capacity, max_jobs=mix.n,
                              queue_capacity=max(mix.n, 4096), window_limit=16)
    assert rc == 0, rc
    out = {"jobs": mix.n, "capacity_bytes": int(mix.capacity),
           "policy": "fifo" if policy == 0 else "mmu"}
    try:
        for label, kw in (("coscheduled", dict(n_streams=n_streams, batch_small=batch, use_graph=1,
                                               tune_cache=tune_cache)),
                          ("serial", dict(n_streams=1, serial=1))):
            print(f"[bench] {name} {label}: {mix.n} jobs", file=sys.stderr, flush=True)
            rc, res, sm = cs.sched_serve(ctx, jt, **kw)
            assert rc == 0, rc
            ok = res["status"] == 0
            out[label] = {"jobs_per_s": sm["jobs_per_s"], "makespan_s": sm["makespan_s"],
                          "p50_turnaround_s": sm["p50_turn_s"], "p99_turnaround_s": sm["p99_turn_s"],
                          "p50_wait_s": sm["p50_wait_s"], "p99_wait_s": sm["p99_wait_s"],
                          "completed": sm["completed"], "rejected": sm["rejected"],
                          "violations": sm["violations"], "passes": sm["passes"],
                          "max_running": sm["max_running"], "batches": sm["batches"],
                          "batched_jobs": sm["batched_jobs"], "wall_s": sm["wall_s"],
                          "host_s": {k: sm["host_" + k + "_s"] for k in ("pass", "launch", "poll",
                                                                          "idle")},
                          "dev_busy_s": sm["dev_busy_s"],
                          "memory": {k: sm[k] for k in ("placements", "slot_waits",
                                                        "placement_slots", "pool_pages",
                                                        "peak_pages", "pages_left",
                                                        "charged_left", "page_check")}}
            # wait = placement - arrival (the summary's); the admission part alone
            w_adm = np.sort((res["t_admit"] - res["t_arrive"])[ok])
            if w_adm.size:
                out[label]["p50_admit_wait_s"] = float(w_adm[int(np.ceil(0.5 * w_adm.size)) - 1])
                out[label]["p99_admit_wait_s"] = float(w_adm[int(np.ceil(0.99 * w_adm.size)) - 1])
            if label == "coscheduled" and batch:
                out[label]["autotuned"] = {"block": sm["tuned_block"], "chunk": sm["tuned_chunk"],
                                           "per_cu": sm["tuned_per_cu"],
                                           "tuner_ran": sm["tuned_from_cache"] == 0,
                                           "cache": tune_cache}
            out[label]["completed_ok"] = int(ok.sum())
    finally:
        cs.sched_destroy(ctx)
    out["speedup_vs_serial"] = (out["coscheduled"]["jobs_per_s"] /
                                max(out["serial"]["jobs_per_s"], 1e-12))
    # what removing the serial run's idle time alone could give: its makespan
    # over the time the device had a job kernel running; beyond it, the gain
    # comes from jobs that leave the device partly idle running side by side
    out["serial_idle_ceiling"] = (out["serial"]["makespan_s"] /
                                  max(out["serial"]["dev_busy_s"], 1e-12))
    # roofline-bound ceiling of the co-scheduled/serial ratio: no schedule can
    # finish before the mix's HBM bytes at peak bandwidth, its GEMM flops at
    # peak bf16 MFMA rate, or the last arrival
    kind, size = np.asarray(jt["kind"]), np.asarray(jt["size"], dtype=np.float64)
    tri, gem, his = kind == 0, kind == 1, kind == 2
    hbm_bytes = (float(((8 + 12 * 10) * size[tri]).sum()) + float((8 * size[his]).sum())
                 + float((8 * size[gem] ** 2).sum()) + float((4 * size[gem] ** 2).sum()))
    flops = float((2 * size[gem] ** 3).sum())
    t_floor = max(hbm_bytes / (HBM_PEAK_GBS * 1e9), flops / 2.5e15, float(jt["arrival_s"][-1]))
    out["roofline_ceiling"] = {"hbm_bytes": hbm_bytes, "gemm_flops": flops,
                               "t_floor_s": t_floor,
                               "ratio_ceiling": out["serial"]["makespan_s"] / t_floor,
                               "note": "serial makespan over max(bytes / 8 TB/s, flops / "
                                       "2.5 PFLOP/s, last arrival)"}
    return out


def nearest_rank(x, p):
    """p-th percentile by nearest rank: sorted[ceil(p n / 100) - 1]."""
    import numpy as np
    x = np.sort(np.asarray(x, dtype=np.float64))
    if x.size == 0:
        return float("nan")
    return float(x[max(int(np.ceil(p * x.size / 100.0)) - 1, 0)])


def hol_run(cs, n_streams=3):
    """Head-of-line study: the HOL mix served in real time under FIFO and MMU
    (co-scheduled), with the small jobs' and the blocker's waits."""
    import numpy as np
    from workloads import HOL_BLOCKER, HOL_SMALL, hol_jobs, job_table
    mix = hol_jobs()
    jt = job_table(mix)
    cls = mix.extra["cls"]
    out = {"jobs": mix.n, "capacity_bytes": int(mix.capacity),
           "shape": "20 GiB triad at 0, 16 GiB blocker at 1 ms, 200 triads of 64-256 MiB "
                    "from 2 ms at 1000/s"}
    for label, policy in (("fifo", cs.SCHED_POLICY_FIFO), ("mmu", cs.SCHED_POLICY_MMU)):
        print(f"[bench] hol {label}: {mix.n} jobs", file=sys.stderr, flush=True)
        rc, ctx = cs.sched_create(policy=policy, capacity_bytes=mix.capacity, max_jobs=mix.n,
                                  queue_capacity=4096, window_limit=16)
        assert rc == 0, rc
        try:
            rc, res, sm = cs.sched_serve(ctx, jt, n_streams=n_streams, use_graph=1)
            assert rc == 0, rc
        finally:
            cs.sched_destroy(ctx)
        wait = res["t_admit"] - res["t_arrive"]
        small = cls == HOL_SMALL
        blk = int(np.flatnonzero(cls == HOL_BLOCKER)[0])
        out[label] = {"jobs_per_s": sm["jobs_per_s"], "makespan_s": sm["makespan_s"],
                      "small_p50_wait_s": nearest_rank(wait[small], 50),
                      "small_p99_wait_s": nearest_rank(wait[small], 99),
                      "blocker_wait_s": float(wait[blk]),
                      "small_admitted_before_blocker":
                          int((res["t_admit"][small] < res["t_admit"][blk]).sum()),
                      "completed": sm["completed"], "violations": sm["violations"]}
    out["small_p99_wait_fifo_over_mmu"] = (out["fifo"]["small_p99_wait_s"] /
                                           max(out["mmu"]["small_p99_wait_s"], 1e-9))
    return out


def c2_step(cs, ctx, d_job, d_dem, coins):
    """reset + intake of the whole queue + the release/admit rounds chained
    on the device.  Intake and chain are one call (sched_enqueue_chain): the
    chain runs right behind the intake and checks its validity verdict on the
    device, so the step has one host synchronisation, the chain's."""
    assert cs.sched_reset(ctx) == 0
    rc, res = cs.sched_enqueue_chain_array(ctx, d_job, d_dem, coins.shape[0] + 1, coins)
    assert rc == 0
    return res


def c2_step_totals(cs, res):
    """Per-step totals of a c2_step result array (outside the timed region)."""
    col = {k: i for i, k in enumerate(cs.PASS_FIELDS)}
    tot = {k: int(res[:, col[k]].sum()) for k in ("admitted", "scanned", "compacted", "released")}
    # running jobs each round's release step looks at
    running, considered = 0, 0
    for i in range(res.shape[0]):
        if i > 0:
            considered += running
        running += int(res[i, col["admitted"]] - res[i, col["released"]])
    tot["considered"] = considered
    per_pass = [(int(res[i, col["admitted"]]), int(res[i, col["free_after"]]))
                for i in range(res.shape[0])]
    return tot, per_pass


def c2_step_synchronous(cs, ctx, d_job, d_dem, coins):
    """The same rounds through the per-pass host API (sched_pass after each
    sched_release_masked): every pass returns to the host."""
    assert cs.sched_reset(ctx) == 0
    assert cs.sched_enqueue_batch(ctx, d_job, d_dem) == 0
    admitted = 0
    for r in range(coins.shape[0] + 1):
        if r > 0:
            assert cs.sched_release_masked(ctx, coins[r - 1]) == 0
        rc, res = cs.sched_pass(ctx)
        assert rc == 0
        admitted += res["admitted"]
    return admitted


def tenant_measure(cs, torch, dev):
    """Event-timed tenant kernels against their roofline: triad and histogram
    against HBM, GEMM against dense bf16 MFMA."""
    out = {}
    n = 1 << 29                                    # 2 GiB per fp32 array, 6 GiB in all
    b = torch.empty(n, dtype=torch.float32, device=dev)
    c = torch.empty_like(b)
    a = torch.empty_like(b)
    assert cs.sched_triad_fill(b, c, 1) == 0
    assert cs.sched_triad(a, b, c, 3.0, 2) == 0
    cs.sched_profile(True)
    assert cs.sched_triad(a, b, c, 3.0, 10) == 0
    torch.cuda.synchronize()
    rc, ms, launches = cs.sched_profile_read("k_triad")
    cs.sched_profile(False)
    gbs = 12.0 * n * launches / (ms * 1e-3) / 1e9
    out["triad"] = {"elements": n, "sweeps": launches, "avg_sweep_us": 1e3 * ms / launches,
                    "GBps": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS,
                    "bytes_per_sweep": 12 * n}
    del a, b, c
    keys = torch.empty(n, dtype=torch.int32, device=dev)
    bins = torch.empty(4096, dtype=torch.int32, device=dev)
    assert cs.sched_hist_fill(keys, 1) == 0
    assert cs.sched_hist(keys, bins) == 0
    cs.sched_profile(True)
    for _ in range(5):
        assert cs.sched_hist(keys, bins) == 0
    torch.cuda.synchronize()
    rc, ms, launches = cs.sched_profile_read("k_hist")
    cs.sched_profile(False)
    gbs = 4.0 * n * launches / (ms * 1e-3) / 1e9
    out["hist"] = {"keys": n, "avg_us": 1e3 * ms / launches, "GBps": gbs,
                   "frac_of_peak": gbs / HBM_PEAK_GBS}
    del keys, bins
    N = 8192
    A = torch.empty(N * N, dtype=torch.int16, device=dev)
    B = torch.empty(N * N, dtype=torch.int16, device=dev)
    C = torch.empty(N * N, dtype=torch.float32, device=dev)
    assert cs.sched_gemm_fill(A, N, N, 1) == 0
    assert cs.sched_gemm_fill(B, N, N, 2) == 0
    for _ in range(3):
        assert cs.sched_gemm_bf16(A, B, C, N, N, N) == 0
    cs.sched_profile(True)
    for _ in range(10):
        assert cs.sched_gemm_bf16(A, B, C, N, N, N) == 0
    torch.cuda.synchronize()
    rc, ms, launches = cs.sched_profile_read("k_gemm_bf16")
    cs.sched_profile(False)
    tf = 2.0 * N ** 3 * launches / (ms * 1e-3) / 1e12
    out["gemm_bf16"] = {"N": N, "avg_ms": ms / launches, "TFLOPs": tf,
                        "frac_of_peak": tf / 2500.0, "peak_TFLOPs": 2500.0}
    del A, B, C
    torch.cuda.empty_cache()
    return out


def first_fit_holds(demand, R, admit):
    """Checks a first-fit (Sec. V, MMU) result by the property that fixes it:
    entry i is admitted exactly when it is present and fits the memory left
    after the admitted entries before it (one exclusive prefix sum).  A check
    of the bench's own output, independent of how the device computed it."""
    import numpy as np
    d = np.asarray(demand, dtype=np.int64)
    a = np.asarray(admit, dtype=bool)
    if np.any(a & (d < 0)):
        return False
    taken = np.where(a, d, 0)
    before = np.cumsum(taken) - taken
    return bool(np.array_equal((d >= 0) & (d <= int(R) - before), a))


def dense_sweep(cs, torch, dev, sizes, seed, window, reps=5):
    """C2-D at each size: (a) FIFO over a queue whose whole length is the
    admitted prefix, (b) first fit over 64 MiB-4 GiB demands (every entry is
    inspected).  Whole calls by the host clock, kernels by HIP events; each
    result checked (first fit: the property that fixes it; FIFO: everything
    admitted, no memory left)."""
    from workloads import c2d_fifo_queue, c2d_queue
    out = []
    for lg in sizes:
        n = 1 << lg
        for name, pol, q in (("fifo_all", cs.SCHED_POLICY_FIFO, c2d_fifo_queue(seed=seed, n=n)),
                             ("first_fit", cs.SCHED_POLICY_MMU, c2d_queue(seed=seed, n=n))):
            dd = torch.from_numpy(q.demand).to(dev)
            dec = torch.zeros(n, dtype=torch.uint8, device=dev)
            rc, r = cs.sched_scan(pol, dd, q.capacity, dec, window_limit=window)
            assert rc == 0
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                rc, r = cs.sched_scan(pol, dd, q.capacity, dec, window_limit=window)
                assert rc == 0
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / reps
            cs.sched_profile(True)
            for _ in range(reps):
                assert cs.sched_scan(pol, dd, q.capacity, dec, window_limit=window)[0] == 0
            torch.cuda.synchronize()
            ms = sum(cs.sched_profile_read(k)[1] for k in ("k_round", "k_window", "k_split_reduce",
                                                           "k_split_scan", "k_split_write"))
            cs.sched_profile(False)
            a = dec.cpu().numpy().astype(bool)
            ok = (bool(a.all()) and r["free_after"] == 0) if pol == cs.SCHED_POLICY_FIFO else \
                first_fit_holds(q.demand, q.capacity, a)
            kern = ms * 1e-3 / reps
            bytes_pass = 9 * n
            out.append({"log2_n": lg, "pass": name, "pass_us": dt * 1e6, "kernels_us": kern * 1e6,
                        "rounds": r["rounds"], "GBps_pass": bytes_pass / dt / 1e9,
                        "GBps_kernels": bytes_pass / kern / 1e9,
                        "frac_of_peak_kernels": bytes_pass / kern / 1e9 / HBM_PEAK_GBS,
                        "frac_of_peak_pass": bytes_pass / dt / 1e9 / HBM_PEAK_GBS, "ok": bool(ok)})
            print(f"[bench] dense sweep: {json.dumps(out[-1])}", file=sys.stderr, flush=True)
            del dd, dec, q, a
            torch.cuda.empty_cache()
    return out


def slab_measure(cs, torch, dev):
    """C3: 2^22 allocator ops in 64 concurrent phases; ops/s over the phases."""
    from workloads import c3_ops
    ops = c3_ops(seed=3)
    rc, ctx = cs.sched_create(capacity_bytes=1 << 40, max_jobs=16, max_tenants=ops.quotas.size,
                              slab_pool_bytes=ops.pool, queue_capacity=4096)
    assert rc == 0
    try:
        assert cs.sched_slab_set_quotas(ctx, ops.quotas) == 0
        kind = torch.from_numpy(ops.kind).to(dev)
        ten = torch.from_numpy(ops.tenant).to(dev)
        size = torch.from_numpy(ops.size).to(dev)
        ref = torch.from_numpy(ops.ref).to(dev)
        ptr = torch.zeros(ops.n, dtype=torch.int64, device=dev)
        st = torch.zeros(ops.n, dtype=torch.int8, device=dev)
        torch.cuda.synchronize()
        cs.sched_profile(True)
        t0 = time.perf_counter()
        for p0 in range(0, ops.n, ops.phase_len):
            assert cs.sched_slab_ops(ctx, p0, min(p0 + ops.phase_len, ops.n), kind, ten, size,
                                     ref, ptr, st) == 0
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rc, ms, launches = cs.sched_profile_read("k_slab_phase")
        cs.sched_profile(False)
        ok = int((st == 0).sum().item())
    finally:
        cs.sched_destroy(ctx)
    return {"ops": ops.n, "phases": launches, "ops_per_s": ops.n / dt,
            "ops_per_s_kernels": ops.n / (ms * 1e-3), "avg_phase_us": 1e3 * ms / launches,
            "ok": ok, "bound": "device atomics (no HBM or MFMA roofline applies)"}


def cpu_baseline_c2(q, seconds):
    """The oracle as it stands, on one host core, on whole C2 steps: the plain
    sequential C loop (gcc -O2) and the numpy/Python statement, each for about
    half of `seconds`.  `value` is the compiled oracle's rate."""
    from oracle import c2seq
    from oracle import sched as S
    c2seq.lib()

    def timed(fn, budget):
        t0 = time.perf_counter()
        steps, admitted, last = 0, 0, None
        while True:
            admitted, last = fn(admitted)
            steps += 1
            if time.perf_counter() - t0 >= budget:
                break
        return steps, admitted, time.perf_counter() - t0, last

    def run_c(acc):
        res = c2seq.release_rounds(q.demand, q.capacity, q.coins, q.rounds, S.MMU)
        return acc + sum(int(r[0].size) for r in res), [(int(r[0].size), int(r[1])) for r in res]

    def run_py(acc):
        res = S.release_rounds(q.demand, q.capacity, q.coins, q.rounds, S.MMU)
        return (acc + sum(int(r.admitted.size) for r in res),
                [(int(r.admitted.size), int(r.R_after)) for r in res])

    c_steps, c_adm, c_dt, c_last = timed(run_c, seconds / 2)
    p_steps, p_adm, p_dt, p_last = timed(run_py, seconds / 2)
    assert c_last == p_last, "the C and numpy oracles disagree"
    host = host_info()
    return {"value": c_adm / c_dt, "unit": "admissions/s", "cores": 1, "kind": "oracle",
            "cpu": host["model"], "nproc": host["nproc"], "cpu_count": host["cpu_count"],
            "sample": f"{c_steps} full steps (intake of 2^{q.n.bit_length() - 1} requests + "
                      f"{q.rounds} release/admit passes) in {c_dt:.1f} s, plain sequential C "
                      f"(oracle/c2seq.c, gcc -O2), one thread",
            "us_per_step": 1e6 * c_dt / c_steps,
            "python": {"value": p_adm / p_dt, "unit": "admissions/s", "cores": 1,
                       "us_per_step": 1e6 * p_dt / p_steps,
                       "sample": f"{p_steps} full steps in {p_dt:.1f} s, numpy/Python "
                                 f"(oracle/sched.py release_rounds), one thread"}}, c_last


def host_info():
    """The host CPU: model name (lscpu, else /proc/cpuinfo), the cores this
    process may run on (nproc) and the cores the machine has."""
    import subprocess
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model == "unknown":
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        model = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    return {"model": model, "nproc": nproc, "cpu_count": os.cpu_count()}


ROOT = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = {"k_chain": "paper_1712_04495_amd/csrc/admission.hip",
                 "k_window": "paper_1712_04495_amd/csrc/admission.hip",
                 "k_round": "paper_1712_04495_amd/csrc/admission.hip"}


def _sha256(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def _counter_rows(path, counter):
    """(kernel name, value) per dispatch from a rocprofv3 counter CSV."""
    import csv
    out = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name", "").strip() != counter:
                continue
            out.append((r.get("Kernel_Name", ""), float(r["Counter_Value"])))
    return out


def traffic_record(fetch_csv, write_csv, copy_mib, kernel):
    """HBM bytes per launch of `kernel`: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch) scaled by what the same counters read for a device-to-device
    copy of copy_mib MiB (which reads and writes exactly that many bytes)."""
    copy_bytes = float(copy_mib) * (1 << 20)
    rec = {"kernel": kernel, "source": KERNEL_SOURCE[kernel],
           "source_sha256": _sha256(KERNEL_SOURCE[kernel]), "copy_bytes": copy_bytes}
    for name, path, key in (("FETCH_SIZE", fetch_csv, "fetch"), ("WRITE_SIZE", write_csv, "write")):
        rows = _counter_rows(path, name)
        mine = [v for k, v in rows if k.split("(")[0].strip().endswith(kernel)]
        copies = [v for k, v in rows if "copy" in k.lower() and kernel not in k]
        assert mine and copies, f"no {kernel} or copy dispatches with {name} in {path}"
        copy_kib = max(copies)       # the calibration copy is the largest copy
        factor = copy_bytes / (copy_kib * 1024.0)
        per = sum(mine) / len(mine) * 1024.0 * factor
        rec[key] = {"counter_kib_per_dispatch": sum(mine) / len(mine), "dispatches": len(mine),
                    "copy_counter_kib": copy_kib, "scale": factor, "bytes_per_launch": per}
    rec["bytes_per_launch"] = rec["fetch"]["bytes_per_launch"] + rec["write"]["bytes_per_launch"]
    return rec


def traffic_for(kernel):
    """The committed traffic record of `kernel`, or None if there is none or
    its source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_c2_traffic.json")
    if kernel not in KERNEL_SOURCE or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != _sha256(KERNEL_SOURCE[kernel]):
        return None
    return rec["bytes_per_launch"]


def main():
    args = parse()
    if args.traffic_from:
        rec = traffic_record(args.traffic_from[0], args.traffic_from[1], args.copy_calib_mib,
                             args.traffic_kernel)
        path = os.path.join(ROOT, "profiles", f"{args.traffic_kernel}_c2_traffic.json")
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
        print(json.dumps(rec))
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: the admission state is "
                                   "per device, and sharding across GPUs is not implemented", "n_gpus": args.gpus}))
        return 2

    import numpy as np
    import torch

    from paper_1712_04495_amd import cosched as cs
    from workloads import c2_queue, c2d_queue

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = "cuda:0"
    cs.lib()
    n = 1 << args.queue_log2
    q = c2_queue(seed=args.seed, n=n)
    rc, ctx = cs.sched_create(policy=cs.SCHED_POLICY_MMU, capacity_bytes=q.capacity, max_jobs=n,
                              queue_capacity=n, window_limit=16)
    assert rc == 0, rc
    rc, j0 = cs.sched_register_batch(ctx, n)
    assert rc == 0 and j0 == 0
    d_job = torch.arange(n, dtype=torch.int32, device=dev)
    d_dem = torch.from_numpy(q.demand).to(dev)
    coins = torch.from_numpy(q.coins).to(dev)
    torch.cuda.synchronize()

    if args.copy_calib_mib > 0:
        src = torch.ones(args.copy_calib_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        c2_step(cs, ctx, d_job, d_dem, coins)
    profile = not args.no_profile
    every = max(1, args.profile_every)
    cs.sched_profile(1)
    cs.sched_profile(0)
    print(f"[bench] c2: {args.steps} timed steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, sampled_steps = [], []
    for i in range(args.steps):
        sampled = profile and i % every == every - 1
        if sampled:
            cs.sched_profile(2)
        results.append(c2_step(cs, ctx, d_job, d_dem, coins))
        if sampled:
            cs.sched_profile(0)
            sampled_steps.append(i)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # per-step totals, outside the timed region
    tot_adm = 0
    prof = {"scanned": 0, "compacted": 0, "released": 0, "considered": 0}
    last = None
    for i, res in enumerate(results):
        tot, last = c2_step_totals(cs, res)
        tot_adm += tot["admitted"]
        if i in sampled_steps:
            for k in prof:
                prof[k] += tot[k]
    prof_steps = len(sampled_steps)
    profile = profile and prof_steps > 0
    kern = {}
    if profile:
        for k in ("k_chain", "k_run_list", "k_window", "k_round", "k_compact", "k_release_masked"):
            rc, ms, launches = cs.sched_profile_read(k)
            if launches:
                kern[k] = (ms, launches)
    # the per-pass host API on the same rounds, for comparison
    t1 = time.perf_counter()
    sync_adm = 0
    for _ in range(args.steps):
        sync_adm += c2_step_synchronous(cs, ctx, d_job, d_dem, coins)
    torch.cuda.synchronize()
    sync_dt = time.perf_counter() - t1
    assert sync_adm == tot_adm
    cs.sched_destroy(ctx)

    out = {
        "metric": METRIC,
        "value": tot_adm / dt,
        "unit": "admissions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": f"admission microbench: 2^{args.queue_log2} requests, demands "
                               "log-uniform 4 KiB-4 GiB (4 KiB aligned), capacity 280e9 B, "
                               "MMU (FIFO prefix + first-fit backfill), 8 release/admit rounds",
                   "queue": n, "rounds": q.rounds, "capacity_bytes": q.capacity,
                   "policy": "mmu", "seed": args.seed,
                   "admissions_per_step": tot_adm // args.steps,
                   "us_per_pass": 1e6 * dt / args.steps / q.rounds,
                   "step": "reset + intake of 2^20 requests + 8 rounds chained on the device (intake and chain in one call, one host synchronisation)",
                   "per_pass_host_api": {"admissions_per_s": sync_adm / sync_dt,
                                         "us_per_pass": 1e6 * sync_dt / args.steps / q.rounds}},
    }
    if profile:
        # Algorithmic bytes of the dominant kernel: 8 B demand read + 1 B
        # decision written per queue entry a pass inspects (the admission
        # decision itself).  What the chain also moves for the release step
        # (4 B id + 4 B state + 1 B mask per running job it looks at, 8 B
        # reservation read + 12 B written per released job) and the compaction
        # (25 B read + 24 B written per entry of [head, last admitted]) is
        # reported beside it, not counted in `achieved`.
        per_step_decide = 9 * prof["scanned"]
        # (the running-list scan, 4 B of state per job, runs only when jobs
        # may be running; after the step's reset the list starts empty)
        side = {"release_bytes": 9 * prof["considered"] + 20 * prof["released"],
                "compaction_bytes": 49 * prof["compacted"],
                "run_list_bytes": 4 * n * kern["k_run_list"][1] if "k_run_list" in kern else 0}
        alg = {"k_chain": per_step_decide, "k_run_list": side["run_list_bytes"]}
        dom = max(kern, key=lambda k: kern[k][0])
        ms, launches = kern[dom]
        avg_s = ms * 1e-3 / max(launches, 1)
        bytes_per_launch = alg.get(dom, 0) / max(launches, 1)
        ach = bytes_per_launch / avg_s / 1e9 if avg_s > 0 else 0.0
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": traffic_for(dom), "kernel": dom,
                           "avg_launch_us": avg_s * 1e6, "bytes_per_launch": bytes_per_launch,
                           "inspected_entries_per_launch": prof["scanned"] / max(launches, 1),
                           "bytes_per_unit": "9 B per inspected queue entry (8 B demand + 1 B "
                                             "decision)",
                           "side_bytes_per_launch": {k: v / max(launches, 1) for k, v in side.items()},
                           "profiled_steps": prof_steps,
                           "kernels_ms_per_step": {k: v[0] / prof_steps for k, v in kern.items()}}

    extras = {x for x in args.extras.split(",") if x}
    # ---- dense first-fit pass: every entry must be read (HBM-bound) -------
    if args.dense_log2 > 0 and "dense" in extras:
        qd = c2d_queue(seed=args.seed, n=1 << args.dense_log2)
        dd = torch.from_numpy(qd.demand).to(dev)
        dec = torch.zeros(qd.n, dtype=torch.uint8, device=dev)
        rc, r0 = cs.sched_scan(cs.SCHED_POLICY_MMU, dd, qd.capacity, dec, window_limit=args.dense_window)
        assert rc == 0
        # whole passes timed without kernel timing (its events cost time of
        # their own), then the kernels timed over as many passes again
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.dense_reps):
            rc, r = cs.sched_scan(cs.SCHED_POLICY_MMU, dd, qd.capacity, dec,
                                  window_limit=args.dense_window)
            assert rc == 0
        torch.cuda.synchronize()
        ddt = (time.perf_counter() - t1) / args.dense_reps
        cs.sched_profile(True)
        for _ in range(args.dense_reps):
            rc, r = cs.sched_scan(cs.SCHED_POLICY_MMU, dd, qd.capacity, dec,
                                  window_limit=args.dense_window)
            assert rc == 0
        torch.cuda.synchronize()
        rc, ms, launches = cs.sched_profile_read("k_round")
        rc, ms_w, launches_w = cs.sched_profile_read("k_window")
        cs.sched_profile(0)
        ok = first_fit_holds(qd.demand, qd.capacity, dec.cpu().numpy().astype(bool))
        bytes_pass = 9 * qd.n     # each entry read once (8 B) + its decision (1 B)
        kern_s = (ms + ms_w) * 1e-3 / args.dense_reps
        out["dense_scan"] = {
            "entries": qd.n, "rounds": r["rounds"], "pass_ms": ddt * 1e3,
            "kernels_ms": kern_s * 1e3, "round_launches_per_pass": launches / args.dense_reps,
            "window_launches_per_pass": launches_w / args.dense_reps, "window_limit": args.dense_window,
            "GBps_pass": bytes_pass / ddt / 1e9, "GBps_kernels": bytes_pass / kern_s / 1e9,
            "frac_of_peak": bytes_pass / kern_s / 1e9 / HBM_PEAK_GBS,
            # the grid round (the streaming scan kernel) alone: the single-wave
            # window walk in front of it decides the first few thousand entries,
            # so the round's bytes are those of the whole queue to < 0.1 %
            "window_walk_ms": ms_w / args.dense_reps, "round_kernel_ms": ms / args.dense_reps,
            "GBps_round_kernel": bytes_pass / (ms * 1e-3 / args.dense_reps) / 1e9,
            "round_frac_of_peak": bytes_pass / (ms * 1e-3 / args.dense_reps) / 1e9 / HBM_PEAK_GBS,
            "fixed_point_ok": bool(ok),
            # HBM bytes per grid round measured with FETCH_SIZE / WRITE_SIZE
            # (committed record; None once the kernel's source has changed)
            "round_traffic_bytes": traffic_for("k_round"), "round_algorithmic_bytes": bytes_pass}
        del dd, dec

    if "dense" in extras and args.dense_sweep:
        out["dense_sweep"] = dense_sweep(cs, torch, dev,
                                         [int(x) for x in args.dense_sweep.split(",") if x],
                                         args.seed, args.dense_window)
    if "tenants" in extras:
        out["tenants"] = tenant_measure(cs, torch, dev)
        # the triad over 6 GiB is the achievable-bandwidth reference: every
        # HBM-bound figure is also reported as a fraction of it
        ach = out["tenants"]["triad"]["GBps"]
        out["hbm_achieved_GBps"] = ach
        out["tenants"]["hist"]["frac_of_achieved"] = out["tenants"]["hist"]["GBps"] / ach
        if "dense_scan" in out:
            ds = out["dense_scan"]
            ds["frac_of_achieved"] = ds["GBps_kernels"] / ach
            ds["round_frac_of_achieved"] = ds["GBps_round_kernel"] / ach
        print(f"[bench] tenants: {json.dumps(out['tenants'])}", file=sys.stderr, flush=True)
    if "slab" in extras:
        out["slab"] = slab_measure(cs, torch, dev)
        print(f"[bench] slab: {json.dumps(out['slab'])}", file=sys.stderr, flush=True)

    if args.cosched:
        torch.cuda.empty_cache()
        free, _ = torch.cuda.mem_get_info()
        out["coschedule"] = {}
        for name in [x for x in args.cosched.split(",") if x]:
            if name == "hol":
                out["coschedule"][name] = hol_run(cs, args.cosched_streams)
            else:
                out["coschedule"][name] = cosched_run(cs, name,
                                                      args.c5_jobs if name == "c5" else args.c4_jobs,
                                                      int(free), args.cosched_streams,
                                                      args.tune_cache or tune_cache_path(torch))
            print(f"[bench] {name}: {json.dumps(out['coschedule'][name])}", file=sys.stderr,
                  flush=True)

    if args.cpu_seconds > 0:
        cb, ref_pass = cpu_baseline_c2(q, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["parity_last_step"] = ref_pass == [(int(a), int(b)) for a, b in last]
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
