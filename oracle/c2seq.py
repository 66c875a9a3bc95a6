"""ctypes front end of ``c2seq.c`` -- CPU oracle, TEST INFRASTRUCTURE ONLY.

``c2seq.c`` states the release/admit rounds of the admission microbenchmark
(Sec. V Policies 1 and 2, Sec. IV post-free) as a plain sequential C loop,
so the oracle can also be timed as compiled code on one host core.  Its
results must equal ``sched.release_rounds`` (pinned in
``tests/test_oracle_c2seq.py``).  Built with gcc -O2; nothing here is used by
the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_DIR, "c2seq.c")
LIB = os.path.join(_DIR, "libc2seq.so")
CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-Wall"]

_lib = None


def build() -> str:
    """Compiles c2seq.c into libc2seq.so next to it (gcc -O2)."""
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-o", tmp, SRC], check=True)
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        p64 = C.POINTER(C.c_int64)
        L.c2seq_release_rounds.restype = C.c_int
        L.c2seq_release_rounds.argtypes = [C.c_int64, p64, C.c_int64, C.POINTER(C.c_uint8),
                                           C.c_int32, C.c_int32, p64, p64, p64, p64]
        _lib = L
    return _lib


def release_rounds(demand, capacity: int, coins, rounds: int, policy: int = 1):
    """Same contract as ``sched.release_rounds``; returns a list of
    (admitted ids int64[], R_after, released count) per round."""
    d = np.ascontiguousarray(demand, dtype=np.int64)
    n = d.size
    co = np.ascontiguousarray(coins, dtype=np.uint8).reshape(-1)
    if rounds > 1 and co.size < (rounds - 1) * n:
        raise ValueError("coins must hold (rounds - 1) * n entries")
    if co.size == 0:
        co = np.zeros(1, np.uint8)
    cnt = np.zeros(max(rounds, 1), np.int64)
    Ra = np.zeros(max(rounds, 1), np.int64)
    rel = np.zeros(max(rounds, 1), np.int64)
    ids = np.zeros(max(n, 1), np.int64)
    p64 = C.POINTER(C.c_int64)
    rc = lib().c2seq_release_rounds(n, d.ctypes.data_as(p64), int(capacity),
                                    co.ctypes.data_as(C.POINTER(C.c_uint8)), rounds, policy,
                                    cnt.ctypes.data_as(p64), Ra.ctypes.data_as(p64),
                                    rel.ctypes.data_as(p64), ids.ctypes.data_as(p64))
    if rc != 0:
        raise ValueError("c2seq_release_rounds refused its arguments")
    out, off = [], 0
    for r in range(rounds):
        k = int(cnt[r])
        out.append((ids[off:off + k].copy(), int(Ra[r]), int(rel[r])))
        off += k
    return out
