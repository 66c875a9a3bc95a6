"""Host-side logic of bench.py, on the CPU: the first-fit property it checks
the dense passes against, the nearest-rank percentile of the serving
figures, the HBM-traffic record it builds from rocprofv3 counter files (and
drops once the kernel's source has changed), and its refusal of more than one
GPU."""
import csv
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import sched as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _queue(rng, n):
    d = rng.integers(1, 100, n).astype(np.int64)
    d[rng.random(n) < 0.1] = -1  # withdrawn requests
    return d


def test_first_fit_check_accepts_the_oracle(bench):
    rng = np.random.default_rng(11)
    for _ in range(200):
        n = int(rng.integers(1, 120))
        d = _queue(rng, n)
        R = int(rng.integers(0, 2500))
        admit, _ = S.mmu_pass(d, R)
        assert bench.first_fit_holds(d, R, admit)


def test_first_fit_check_rejects_every_single_change(bench):
    """Flipping any one decision of a first-fit result breaks the property:
    dropping an admitted entry leaves room that the next fitting entry, or
    the dropped one, should have taken; adding one either overflows or takes
    an entry that first fit skipped because it did not fit."""
    rng = np.random.default_rng(12)
    for _ in range(40):
        n = int(rng.integers(1, 60))
        d = _queue(rng, n)
        R = int(rng.integers(0, 1500))
        admit, _ = S.mmu_pass(d, R)
        for i in range(n):
            bad = admit.copy()
            bad[i] = not bad[i]
            assert not bench.first_fit_holds(d, R, bad), (d.tolist(), R, i)


def test_first_fit_check_on_fifo_prefix_and_empty_cases(bench):
    d = np.array([3, 4, 5, 100, 1, 1], dtype=np.int64)
    # R = 12: 3 + 4 + 5 fill it exactly; 100 does not fit, nor does anything after
    assert bench.first_fit_holds(d, 12, [1, 1, 1, 0, 0, 0])
    # R = 14: the two 1s behind the 100 are backfilled
    assert bench.first_fit_holds(d, 14, [1, 1, 1, 0, 1, 1])
    assert not bench.first_fit_holds(d, 14, [1, 1, 1, 0, 0, 0])
    assert bench.first_fit_holds(d, 0, [0] * 6)
    assert bench.first_fit_holds(np.zeros(0, dtype=np.int64), 5, [])
    # a withdrawn entry (-1) is never admitted
    assert not bench.first_fit_holds(np.array([-1, 2]), 5, [1, 1])


def test_nearest_rank(bench):
    x = list(range(10, 0, -1))          # 10 .. 1, unsorted on purpose
    assert bench.nearest_rank(x, 50) == 5.0
    assert bench.nearest_rank(x, 90) == 9.0
    assert bench.nearest_rank(x, 99) == 10.0
    assert bench.nearest_rank(x, 100) == 10.0
    assert bench.nearest_rank(x, 1) == 1.0
    assert bench.nearest_rank([7.5], 99) == 7.5
    assert np.isnan(bench.nearest_rank([], 50))


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                          "Counter_Value"])
        w.writeheader()
        for i, (kernel, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter,
                        "Counter_Value": value})


def test_traffic_record_scales_by_the_calibration_copy(bench, tmp_path):
    """Counters in KiB per dispatch, scaled by what they read for a copy of
    known size: a 256 MiB copy whose counter reads half its bytes doubles
    every reading.  Other kernels and smaller copies are ignored."""
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    chain = "schedk::k_chain(schedk::DevCtl*, long)"
    _counter_csv(fetch, "FETCH_SIZE", [(chain, 100.0), ("schedk::k_round(long)", 9e5),
                                       (chain, 120.0), ("__amd_rocclr_copyBuffer", 4.0),
                                       ("__amd_rocclr_copyBuffer", 131072.0)])
    _counter_csv(write, "WRITE_SIZE", [(chain, 300.0), ("__amd_rocclr_copyBuffer", 131072.0),
                                       (chain, 280.0)])
    rec = bench.traffic_record(str(fetch), str(write), 256, "k_chain")
    assert rec["fetch"]["dispatches"] == 2 and rec["write"]["dispatches"] == 2
    assert rec["fetch"]["scale"] == pytest.approx(2.0)
    assert rec["fetch"]["bytes_per_launch"] == pytest.approx(110.0 * 1024 * 2)
    assert rec["write"]["bytes_per_launch"] == pytest.approx(290.0 * 1024 * 2)
    assert rec["bytes_per_launch"] == pytest.approx(400.0 * 1024 * 2)
    src = os.path.join(ROOT, bench.KERNEL_SOURCE["k_chain"])
    with open(src, "rb") as f:
        assert rec["source_sha256"] == hashlib.sha256(f.read()).hexdigest()


def test_traffic_record_is_dropped_when_the_source_changes(bench, tmp_path, monkeypatch):
    rel = bench.KERNEL_SOURCE["k_chain"]
    src = tmp_path / rel
    src.parent.mkdir(parents=True)
    src.write_text("kernel source, first version\n")
    (tmp_path / "profiles").mkdir()
    rec = {"kernel": "k_chain", "source": rel, "bytes_per_launch": 4321.0,
           "source_sha256": hashlib.sha256(src.read_bytes()).hexdigest()}
    (tmp_path / "profiles" / "k_chain_c2_traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_for("k_chain") == 4321.0
    assert bench.traffic_for("k_round") is None      # no record
    src.write_text("kernel source, second version\n")
    assert bench.traffic_for("k_chain") is None


def test_committed_traffic_records_are_well_formed(bench):
    for kernel in ("k_chain", "k_round"):
        path = os.path.join(ROOT, "profiles", f"{kernel}_c2_traffic.json")
        with open(path) as f:
            rec = json.load(f)
        assert rec["kernel"] == kernel and rec["source"] == bench.KERNEL_SOURCE[kernel]
        assert len(rec["source_sha256"]) == 64
        assert rec["bytes_per_launch"] == pytest.approx(
            rec["fetch"]["bytes_per_launch"] + rec["write"]["bytes_per_launch"])
        assert rec["bytes_per_launch"] > 0


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), ([], {"WORLD_SIZE": "4"})])
def test_more_than_one_gpu_is_refused(argv, env):
    e = dict(os.environ, **env)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv],
                       capture_output=True, text=True, env=e, timeout=120)
    assert r.returncode == 2
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in out["error"]
