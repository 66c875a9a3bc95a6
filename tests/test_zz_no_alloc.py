"""The scan entry point that allocates nothing (sched_scan_noalloc): the same
decisions and results as sched_scan on the same inputs, on two calls in a
row (the second smaller), without any change in the device's free memory
after the first call on the device has set up."""
import numpy as np
import pytest
import torch

from oracle import sched as S
from workloads import c2d_queue, random_queue

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_04495_amd import cosched
    cosched.lib()
    return cosched


@pytest.mark.parametrize("policy", [0, 1])
def test_noalloc_scan_equals_scan(cs, policy):
    big = c2d_queue(seed=3, n=1 << 22)
    small = random_queue(11, 3 * 4096 + 17, 1000, holes=0.05)
    cases = [(big.demand, big.capacity, 64), (small, 200_000, 0)]
    inputs = []
    for d_np, R, wl in cases:
        d = torch.from_numpy(np.ascontiguousarray(d_np)).to(DEV)
        ref = torch.full((d_np.size,), 7, dtype=torch.uint8, device=DEV)
        got = torch.full((d_np.size,), 9, dtype=torch.uint8, device=DEV)
        rc, rr = cs.sched_scan(policy, d, R, ref, write_all=1, window_limit=wl)
        assert rc == 0
        inputs.append((d_np, d, R, wl, ref, rr, got))
    # the first call on a device sets up (it looks up the array's address, and
    # the runtime loads the code object that holds it); later calls must not
    # change the device's free memory
    one = torch.ones(1, dtype=torch.int64, device=DEV)
    one_dec = torch.zeros(1, dtype=torch.uint8, device=DEV)
    assert cs.sched_scan_noalloc(policy, one, 1, one_dec)[0] == 0
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    results = []
    for d_np, d, R, wl, ref, rr, got in inputs:      # two calls, the second smaller
        print(f"  policy={policy} n={d_np.size} R={R} wl={wl}", flush=True)
        results.append(cs.sched_scan_noalloc(policy, d, R, got, write_all=1, window_limit=wl))
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    # compared only now: the comparisons' temporaries go through torch's allocator
    for (rc, rg), (d_np, d, R, wl, ref, rr, got) in zip(results, inputs):
        assert rc == 0
        assert rg == rr
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())
    # the small case against the oracle as well
    d_np, d, R, wl, ref, rr, got = inputs[1]
    a, R2 = (S.fifo_pass if policy == 0 else S.mmu_pass)(d_np, R)
    assert np.array_equal(got.cpu().numpy().astype(bool), a) and rr["free_after"] == R2


def test_noalloc_scan_limits(cs):
    d = torch.ones(8, dtype=torch.int64, device=DEV)
    dec = torch.zeros(8, dtype=torch.uint8, device=DEV)
    r = cs.sched_scan_result_t()
    # more entries than the fixed workspace holds: refused before any work
    assert cs.lib().sched_scan_noalloc(1, (1 << 28) + 1, cs._ptr(d), 100, cs._ptr(dec), 0, 0, None,
                                       cs.C.byref(r)) == cs.SCHED_E_INVALID
    assert cs.sched_scan_noalloc(7, d, 100, dec)[0] == cs.SCHED_E_INVALID
    rc, out = cs.sched_scan_noalloc(1, d, 5, dec, write_all=1)
    assert rc == 0 and out["admitted"] == 5 and out["free_after"] == 0
