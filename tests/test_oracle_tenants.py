"""Pins for the tenant references (oracle/tenants.py)."""
from collections import Counter

import numpy as np

from oracle import tenants as T


def test_splitmix64_published_vectors():
    # Outputs of the reference SplitMix64 generator for state 0 and state 1234567
    # (published test vectors of the algorithm).
    assert [int(x) for x in T.splitmix64_state(0, np.arange(5))] == [
        0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
        0xF88BB8A8724C81EC, 0x1B39896A51A8749B]
    assert [int(x) for x in T.splitmix64_state(1234567, np.arange(5))] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]
    # the seeded form is the state form with s0 = seed << 32
    assert np.array_equal(T.splitmix64(3, np.arange(10)), T.splitmix64_state(3 << 32, np.arange(10)))


def test_triad_inputs_exact_and_ranges():
    idx = np.arange(1 << 16)
    b, c = T.triad_inputs(7, idx)
    assert b.min() >= 1.0 and b.max() < 2.0 and c.min() >= 1.0 and c.max() < 2.0
    assert np.array_equal(b.astype(np.float32).astype(np.float64), b)
    a = T.triad_ref(7, idx)
    # fp32 unfused (mul then add) and fused both give the exact value
    b32, c32 = b.astype(np.float32), c.astype(np.float32)
    unfused = b32 + np.float32(3.0) * c32
    assert np.array_equal(unfused.astype(np.float64), a)
    assert np.all((a >= 4.0) & (a < 8.0))


def test_hist_against_counter():
    n = 5000
    keys = T.hist_keys(11, n)
    cnt = Counter(int(k) & 4095 for k in keys)
    ref = T.hist_ref(11, n)
    assert ref.sum() == n
    assert all(ref[b] == cnt.get(b, 0) for b in range(4096))
    skew = T.hist_ref(11, n, bins=4096, mask=63)
    assert skew.sum() == n and np.all(skew[64:] == 0)
    # chunking does not change the result
    assert np.array_equal(T.hist_ref(11, n, chunk=333), ref)


def test_gemm_operand_exact_bf16():
    A = T.gemm_operand(5, np.arange(4), 64)
    assert np.array_equal(T.bf16_round(A), A)
    assert A.min() >= -2.0 and A.max() < 2.0
    assert np.all((A * 64) == np.round(A * 64))


def test_bf16_round_known_values():
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, -2.5, 1.0 + 2**-7])
    exp = np.array([1.0, 1.0, 1.0 + 2**-6, -2.5, 1.0 + 2**-7])
    assert np.array_equal(T.bf16_round(vals), exp)


def test_gemm_small_brute_force():
    M, N, K = 3, 4, 5
    A = T.gemm_operand(1, np.arange(M), K)
    B = T.gemm_operand(2, np.arange(N), K)
    C = T.gemm_ref_full(1, 2, M, N, K)
    for m in range(M):
        for n in range(N):
            s = 0.0
            for k in range(K):
                s += A[m, k] * B[n, k]
            assert C[m, n] == s
    mi = np.array([0, 2, 1, 2])
    ni = np.array([3, 0, 1, 3])
    assert np.array_equal(T.gemm_ref_entries(1, 2, K, mi, ni), C[mi, ni])


# ---- output digest (position-keyed) ---------------------------------------
def test_position_digest_single_word_and_zeros():
    # one word: (s_0 | 1) * w mod 2^64, s_0 the first SplitMix64 output of the
    # key state; all-zero output digests to 0
    s0 = int(T.splitmix64_state(T.DIGEST_KEY, np.arange(1))[0])
    for w in (1, 7, 0xFFFFFFFF):
        assert T.position_digest(np.array([w], np.uint32)) == ((s0 | 1) * w) % 2**64
    assert T.position_digest(np.zeros(1000, np.uint32)) == 0


def test_position_digest_sees_every_change():
    rng = np.random.default_rng(3)
    w = rng.integers(0, 2**32, 777, dtype=np.uint64).astype(np.uint32)
    d = T.position_digest(w)
    for i in range(w.size):
        for delta in (1, 2**31, int(rng.integers(1, 2**32))):
            v = w.copy()
            v[i] = np.uint32((int(v[i]) + delta) % 2**32)
            assert T.position_digest(v) != d, (i, delta)
    # moving words: swaps of unequal words and a rotation are seen
    for _ in range(500):
        i, j = rng.integers(0, w.size, 2)
        if w[i] == w[j]:
            continue
        v = w.copy()
        v[i], v[j] = v[j], v[i]
        assert T.position_digest(v) != d
    assert T.position_digest(np.roll(w, 1)) != d


def test_position_digest_is_linear_and_chunk_free():
    # additive in the words (mod 2^64) and independent of the chunking
    rng = np.random.default_rng(4)
    a = rng.integers(0, 2**31, 5000, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 2**31, 5000, dtype=np.uint64).astype(np.uint32)
    assert T.position_digest(a + b) == (T.position_digest(a) + T.position_digest(b)) % 2**64
    assert T.position_digest(a, chunk=7) == T.position_digest(a)
    f = np.array([1.0, 4.5, 7.25], np.float32)
    assert T.position_digest(f) == T.position_digest(f.view(np.uint32))


def test_gemm_sample_positions_in_range_and_seeded():
    for N in (256, 1024, 8192):
        r, c = T.gemm_sample_positions(5, N)
        assert r.size == T.GEMM_SAMPLES and np.all((r >= 0) & (r < N) & (c >= 0) & (c < N))
    r1, c1 = T.gemm_sample_positions(5, 4096)
    r2, c2 = T.gemm_sample_positions(6, 4096)
    assert not (np.array_equal(r1, r2) and np.array_equal(c1, c2))
    # position k is SplitMix64 output k of the keyed state, row-major
    s0 = ((5 << 32) ^ T.SAMPLE_KEY) % 2**64
    p = [int(x) % (4096 * 4096) for x in T.splitmix64_state(s0, np.arange(T.GEMM_SAMPLES))]
    assert [int(a) * 4096 + int(b) for a, b in zip(r1, c1)] == p
