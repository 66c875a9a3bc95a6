"""CPU oracle for the memory-safe co-scheduler -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct statement of what the scheduler computes,
written from the paper (Reano, Silla, Nikolopoulos, Varghese, "Intra-node
Memory Safe GPU Co-Scheduling", IEEE TPDS 2017; arXiv:1712.04495):

* ``sched``     -- admission passes under the four notification policies of
                   Sec. V, the scheduler state of Sec. III-B ("shared memory
                   data") and the life-cycle checks of Sec. IV.
* ``schedule``  -- a virtual-clock replay of a whole job mix through that
                   scheduler (arrivals, releases, passes).
* ``slab``      -- a sequential simulator of the quota-checked slab
                   sub-allocator and an invariant checker for logs of
                   concurrent allocator phases.
* ``tenants``   -- references for the synthetic tenant jobs (fp32 triad,
                   int32 histogram, bf16 GEMM in fp64).
* ``c2seq``     -- the release/admit rounds of ``sched`` restated as a plain
                   sequential C loop (``c2seq.c``, gcc -O2), to time the
                   oracle as compiled code on one host core.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline
leg may import this package.  It shares no code with the HIP path in
``paper_1712_04495_amd/``; the only common module is the seeded input
generator ``workloads``.  The product path never calls into it.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against brute force, closed forms or invariants, except where a function's
docstring says "parity unpinned".
"""
