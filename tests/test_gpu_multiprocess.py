"""Clients in separate processes share one context (Sec. III-B, the
shared-memory approach): a child process attaches to the context this
process shared and both run life-cycle calls in one global order; every
result and every reservation equals one oracle Scheduler fed the same
order.  A blocking pre-allocation in the child is admitted by a pass that a
post-free in this process runs."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from oracle import sched as S

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_04495_amd import cosched
    cosched.lib()
    return cosched


class Child:
    def __init__(self, name):
        self.p = subprocess.Popen([sys.executable, "-u", os.path.join(HERE, "mp_client.py"), name],
                                  stdin=subprocess.PIPE, stdout=subprocess.PIPE, text=True)
        self.hello = self.reply()

    def send(self, cmd):
        self.p.stdin.write(cmd + "\n")
        self.p.stdin.flush()

    def reply(self):
        line = self.p.stdout.readline()
        assert line, "the client process ended"
        return json.loads(line)

    def call(self, cmd):
        self.send(cmd)
        return self.reply()

    def close(self):
        try:
            if self.p.poll() is None:
                self.call("quit")
            self.p.wait(timeout=60)
        finally:
            if self.p.poll() is None:
                self.p.kill()


@pytest.mark.parametrize("policy", [0, 1, 3])
def test_two_processes_share_one_context(cs, policy):
    C = 10_000
    name = f"/sched-test-{os.getpid()}-{policy}"
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=C, max_jobs=64, queue_capacity=4096)
    assert rc == 0
    child = None
    try:
        assert cs.sched_share(ctx, name) == 0
        assert cs.sched_share(ctx, name) == cs.SCHED_E_INVALID        # already shared
        child = Child(name)
        assert child.hello["rc"] == 0
        ref = S.Scheduler(C, policy)
        rng = np.random.default_rng(policy + 7)
        jobs = []
        for k in range(16):                    # job handles are common to both processes
            pr = int(rng.integers(0, 3)) if policy >= 2 else 0
            if k % 2:
                r = child.call(f"register {pr} 50")
                rc, j = r["rc"], r["job"]
            else:
                rc, j = cs.sched_register(ctx, pr, 50)
            assert rc == 0 and j == ref.register(pr, 50)
            jobs.append(j)
        for step in range(200):
            j = jobs[int(rng.integers(len(jobs)))]
            in_child = bool(rng.integers(2))
            if rng.random() < 0.55:
                b = int(rng.integers(1, 4000))
                got = (child.call(f"admit {j} {b} {cs.SCHED_NONBLOCK}")["rc"] if in_child else
                       cs.sched_admit(ctx, j, 0, b, cs.SCHED_NONBLOCK))
                assert got == ref.admit(j, 0, b), f"step {step} admit"
            else:
                res = ref.jobs[j]["res"]
                b = 0 if rng.random() < 0.5 else int(rng.integers(0, res + 2))
                got = (child.call(f"release {j} {b}")["rc"] if in_child else
                       cs.sched_release(ctx, j, -1, b))
                assert got == ref.release(j, -1, b), f"step {step} release"
            for jj in jobs:
                want = ref.jobs[jj]["res"]
                assert cs.sched_reservation(ctx, jj) == (0, want)
            if step % 50 == 0:
                r = child.call(f"reservation {j}")
                assert r["rc"] == 0 and r["res"] == ref.jobs[j]["res"]
        # withdraw what still waits (a wait with timeout 0) and free everything,
        # then a blocking request in the child that only a post-free in this
        # process can serve
        for jj in jobs:
            n = ref.withdraw(jj)
            assert cs.sched_wait(ctx, jj, 0) == (S.TIMEOUT if n else S.OK)
        for jj in jobs:
            assert cs.sched_release(ctx, jj, -1, 0) == ref.release(jj, -1, 0) == 0
        assert cs.sched_stats(ctx)[1]["used"] == ref.used == 0
        a, b = jobs[0], jobs[1]
        assert cs.sched_admit(ctx, a, 0, 7000, 0) == ref.admit(a, 0, 7000) == 0
        r = child.call(f"admit {b} 5000 {cs.SCHED_NONBLOCK}")
        assert r["rc"] == ref.admit(b, 0, 5000) == cs.SCHED_NOT_READY
        child.send(f"wait {b} 10000")          # blocks in the child
        assert cs.sched_release(ctx, a, -1, 0) == ref.release(a, -1, 0) == 0
        assert child.reply()["rc"] == 0        # admitted by this process's pass
        assert ref.jobs[b]["res"] == 5000
        assert cs.sched_reservation(ctx, b) == (0, 5000)
        rc, st = cs.sched_stats(ctx)
        assert rc == 0 and st["used"] == 5000
    finally:
        if child:
            child.close()
        cs.sched_destroy(ctx)
    # the name is gone with the context
    assert cs.sched_attach(name)[0] == cs.SCHED_E_INVALID


@pytest.mark.parametrize("policy", [0, 1])
def test_dead_client_is_reclaimed(cs, policy):
    """A client process that holds reservations and has a request waiting is
    killed (SIGKILL: it runs no clean-up).  The sanity check of the process
    that shares the context finds its jobs' owner gone, withdraws the waiting
    request, returns the reservations and admits the request that waited
    behind them -- as the oracle's sanity check does (Sec. III-B, third
    robustness feature; Sec. IV)."""
    import signal
    C = 10_000
    name = f"/sched-dead-{os.getpid()}-{policy}"
    rc, ctx = cs.sched_create(policy=policy, capacity_bytes=C, max_jobs=16, queue_capacity=4096)
    assert rc == 0
    child = None
    dead = set()
    ref = S.Scheduler(C, policy, alive=lambda pid: pid not in dead)
    try:
        assert cs.sched_share(ctx, name) == 0
        child = Child(name)
        assert child.hello["rc"] == 0
        pid = child.hello["pid"]
        held = []
        for b, want in ((3000, S.OK), (4000, S.OK), (5000, S.NOT_READY)):
            r = child.call("register 0 60000")
            assert r["rc"] == 0 and r["job"] == ref.register(0, 60000)
            j = r["job"]
            held.append(j)
            assert child.call(f"own {j}")["rc"] == 0 and ref.set_owner(j, pid) == 0
            got = child.call(f"admit {j} {b} {cs.SCHED_NONBLOCK}")["rc"]
            assert got == ref.admit(j, 0, b) == want
        rc, k = cs.sched_register(ctx, 0, 60000)
        assert rc == 0 and k == ref.register(0, 60000)
        # does not fit beside the child's 7000 bytes; the child is alive
        assert cs.sched_admit(ctx, k, 0, 6000, cs.SCHED_NONBLOCK) == ref.admit(k, 0, 6000) \
            == cs.SCHED_NOT_READY
        assert cs.sched_stats(ctx)[1]["used"] == ref.used == 7000
        child.p.send_signal(signal.SIGKILL)
        assert child.p.wait(timeout=60) == -signal.SIGKILL
        dead.add(pid)
        rc, nj, nb = cs.sched_sanity_check(ctx)
        assert rc == 0 and (nj, nb) == ref.sanity(ref.alive) == (3, 7000)
        for j in held + [k]:
            assert cs.sched_reservation(ctx, j) == (0, ref.jobs[j]["res"])
        assert ref.jobs[k]["res"] == 6000
        assert cs.sched_wait(ctx, k, 0) == S.OK            # nothing of k waits
        assert cs.sched_stats(ctx)[1]["used"] == ref.used == 6000
        # a second check finds nothing more
        assert cs.sched_sanity_check(ctx)[:3] == (0, 0, 0)
    finally:
        if child and child.p.poll() is None:
            child.p.kill()
            child.p.wait(timeout=60)
        cs.sched_destroy(ctx)
