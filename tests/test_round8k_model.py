"""CPU model of an earlier 8192-entry-tile build of the grid-round kernel
(tests/cpu_models/round8k_model.cpp), run on the inputs of the admission
test that was running when that build hung on the GPU: single-tile queues
scanned without the window walk.  Every thread of the modelled workgroup
must pass the same barriers in every round (the source-level condition for
its barriers to match), and the decisions must equal the oracle's FIFO and
first-fit passes (Sec. V, Policies 1 and 2)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import sched as S
from workloads import random_queue

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_models", "round8k_model.cpp")


@pytest.fixture(scope="module")
def model(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path_factory.mktemp("round8k") / "round8k")
    subprocess.run([gxx, "-std=c++20", "-O2", "-pthread", "-o", exe, SRC], check=True)
    return exe


def _run(exe, pol, d, R):
    inp = f"{pol} {d.size} {R}\n" + " ".join(map(str, d.tolist())) + "\n"
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    lines = out.stdout.split("\n")
    return lines[1], lines[3]


@pytest.mark.parametrize("n", [1, 2, 255, 4097])
@pytest.mark.parametrize("pol", [0, 1])
def test_round8k_barriers_and_decisions(model, n, pol):
    wl = 0                                   # the test ran the grid round alone
    rng = np.random.default_rng(n * 7 + wl)  # that test's queue for this size
    d = random_queue(int(rng.integers(1 << 30)), n, 1000, holes=0.05)
    tot = int(d[d >= 0].sum())
    for R in sorted({0, 1, 999, tot // 3, max(tot - 1, 0), tot, tot + 5}):
        dec, status = _run(model, pol, d, R)
        assert status == "barriers consistent", (n, pol, R)
        ref, _ = (S.fifo_pass if pol == 0 else S.mmu_pass)(d, R)
        got = np.array([c == "1" for c in dec], dtype=bool)
        assert np.array_equal(got, ref), (n, pol, R)
        # entries not admitted are rejected ('0') or, after a FIFO pass ends,
        # left to the caller ('?', which write_all then zeroes)
        assert set(dec) <= {"0", "1", "?"}
