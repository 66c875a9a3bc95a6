"""References for the synthetic tenant jobs -- CPU oracle (test infrastructure).

The paper's tenants were third-party CUDA applications (Sec. VI); they are
replaced here by three synthetic kinds whose results have plain definitions:

* STREAM triad  a = b + s*c  in fp32, s = 3;
* histogram of uint32 keys into 4096 (or fewer) int32 bins;
* C = A B^T with bf16 inputs, computed here in fp64 from the exact inputs.

Input contents come from a counter-based generator, SplitMix64 (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
output i of the generator whose state starts at s0 is
    z = s0 + (i + 1) * 0x9E3779B97F4A7C15
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z ^ (z >> 31)
(all mod 2**64), with s0 = seed << 32.  The device implements the same
published definition independently.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_state(s0: int, idx) -> np.ndarray:
    """Output number ``idx`` (0-based, array) of SplitMix64 whose state starts at s0."""
    i = np.asarray(idx, dtype=np.uint64)
    s0 = np.uint64(int(s0) & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        z = s0 + (i + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, idx) -> np.ndarray:
    """Output number ``idx`` of SplitMix64 seeded with state seed << 32."""
    return splitmix64_state(int(seed) << 32, idx)


# --------------------------------------------------------------------------
# Triad
# --------------------------------------------------------------------------
TRIAD_SCALAR = 3.0


def triad_inputs(seed: int, idx):
    """b, c in [1, 2) with 16 fractional bits: b from hash bits 0..15, c from
    bits 16..31.  Exactly representable in fp32."""
    h = splitmix64(seed, idx)
    b = 1.0 + (h & np.uint64(0xFFFF)).astype(np.float64) / 65536.0
    c = 1.0 + ((h >> np.uint64(16)) & np.uint64(0xFFFF)).astype(np.float64) / 65536.0
    return b, c


def triad_ref(seed: int, idx):
    """a = b + 3 c computed in fp64.  With these inputs the exact value has at
    most 19 significant bits, so it is also the correctly rounded fp32 result
    of either a fused or an unfused multiply-add."""
    b, c = triad_inputs(seed, idx)
    return b + TRIAD_SCALAR * c


# --------------------------------------------------------------------------
# Histogram
# --------------------------------------------------------------------------
def hist_keys(seed: int, n: int, start: int = 0):
    """uint32 keys: the low 32 bits of SplitMix64 outputs start .. start+n-1."""
    return (splitmix64(seed, np.arange(start, start + n, dtype=np.uint64))
            & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def hist_ref(seed: int, n: int, bins: int = 4096, mask: int = 4095, chunk: int = 1 << 24):
    """Counts of (key & mask) over n keys, as numpy bincount in chunks."""
    out = np.zeros(bins, dtype=np.int64)
    for s in range(0, n, chunk):
        k = hist_keys(seed, min(chunk, n - s), s)
        out += np.bincount((k & np.uint32(mask)).astype(np.int64), minlength=bins)
    return out


# --------------------------------------------------------------------------
# GEMM  C[m, n] = sum_k A[m, k] * Bt[n, k]
# --------------------------------------------------------------------------
def gemm_operand(seed: int, rows, K: int):
    """Rows of a K-major bf16 operand: element (r, k) is
    ((h(r*K + k) & 255) - 128) / 64, an exact bf16 value in [-2, 2)."""
    rows = np.asarray(rows, dtype=np.uint64)
    idx = rows[:, None] * np.uint64(K) + np.arange(K, dtype=np.uint64)[None, :]
    h = splitmix64(seed, idx)
    return ((h & np.uint64(0xFF)).astype(np.float64) - 128.0) / 64.0


def gemm_ref_entries(seed_a: int, seed_b: int, K: int, m_idx, n_idx):
    """fp64 reference for the entries (m_idx[i], n_idx[i])."""
    m_idx = np.asarray(m_idx, dtype=np.int64)
    n_idx = np.asarray(n_idx, dtype=np.int64)
    um, im = np.unique(m_idx, return_inverse=True)
    un, inn = np.unique(n_idx, return_inverse=True)
    A = gemm_operand(seed_a, um, K)
    B = gemm_operand(seed_b, un, K)
    return np.einsum("ik,ik->i", A[im], B[inn])


def gemm_ref_full(seed_a: int, seed_b: int, M: int, N: int, K: int):
    """Full fp64 product for small sizes (numpy matmul as the contraction)."""
    A = gemm_operand(seed_a, np.arange(M), K)
    B = gemm_operand(seed_b, np.arange(N), K)
    return A @ B.T


def bf16_round(x):
    """Round fp64 values to bf16 (round to nearest even) and back, for pins."""
    f = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> np.uint64(16)) & np.uint64(1)
    r = ((f + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# Output digest and GEMM sample positions reported by the serving loop
# --------------------------------------------------------------------------
# Not part of the method: an encoding of a job's output that the serving
# loop computes on the device, so that results inside a mix can be checked
# element by element without copying them out.
DIGEST_KEY = 0x6A09E667F3BCC908
SAMPLE_KEY = 0xBB67AE8584CAA73B
GEMM_SAMPLES = 8


def position_digest(words, chunk: int = 1 << 24) -> int:
    """sum_i (s_i | 1) * w_i mod 2^64 over 32-bit words w (uint32 array, or
    an fp32 array taken by its bit patterns), s_i = SplitMix64 output i for
    state DIGEST_KEY.  The multipliers are odd, so changing one word always
    changes the digest."""
    w = np.ascontiguousarray(words)
    if w.dtype == np.float32:
        w = w.view(np.uint32)
    w = w.astype(np.uint32, copy=False).ravel()
    total = np.uint64(0)
    with np.errstate(over="ignore"):
        for s in range(0, w.size, chunk):
            part = w[s:s + chunk].astype(np.uint64)
            mult = splitmix64_state(DIGEST_KEY, np.arange(s, s + part.size, dtype=np.uint64))
            total = total + np.sum((mult | np.uint64(1)) * part, dtype=np.uint64)
    return int(total)


def gemm_sample_positions(seed: int, N: int):
    """Row-major positions of the GEMM_SAMPLES entries of C reported for a
    GEMM job: SplitMix64 output k for state (seed << 32) ^ SAMPLE_KEY, mod N^2;
    returned as (rows, cols)."""
    s0 = ((int(seed) << 32) ^ SAMPLE_KEY) & 0xFFFFFFFFFFFFFFFF
    p = splitmix64_state(s0, np.arange(GEMM_SAMPLES, dtype=np.uint64)) % np.uint64(N * N)
    p = p.astype(np.int64)
    return p // N, p % N
