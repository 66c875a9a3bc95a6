"""Tenant kernels vs the oracle references: triad bit-exact (its values are
exact in fp32), histogram bit-exact, bf16 GEMM within 2e-2 relative of the
fp64 product of the exact bf16 inputs."""
import numpy as np
import pytest
import torch

from oracle import tenants as T

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def cs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1712_04495_amd import cosched
    cosched.lib()
    return cosched


@pytest.mark.parametrize("n", [1, 3, 4, 1023, 4096 * 257 + 5, 3_000_001])
def test_triad_exact(cs, n):
    b = torch.empty(n, dtype=torch.float32, device=DEV)
    c = torch.empty_like(b)
    a = torch.full_like(b, -1.0)
    assert cs.sched_triad_fill(b, c, 7) == 0
    assert cs.sched_triad(a, b, c, 3.0, 10) == 0
    torch.cuda.synchronize()
    idx = np.arange(n)
    bb, cc = T.triad_inputs(7, idx)
    assert np.array_equal(b.cpu().numpy().astype(np.float64), bb)
    assert np.array_equal(c.cpu().numpy().astype(np.float64), cc)
    assert np.array_equal(a.cpu().numpy().astype(np.float64), T.triad_ref(7, idx))


def test_triad_large_sampled(cs):
    n = (1 << 28) + 12345                       # 1 GiB per array
    b = torch.empty(n, dtype=torch.float32, device=DEV)
    c = torch.empty_like(b)
    a = torch.empty_like(b)
    assert cs.sched_triad_fill(b, c, 11) == 0
    assert cs.sched_triad(a, b, c, 3.0, 2) == 0
    rng = np.random.default_rng(0)
    idx = np.unique(np.concatenate([rng.integers(0, n, 100_000), np.arange(n - 64, n)]))
    got = a[torch.from_numpy(idx).to(DEV)].cpu().numpy().astype(np.float64)
    assert np.array_equal(got, T.triad_ref(11, idx))


@pytest.mark.parametrize("n,mask", [(0, 4095), (1, 4095), (7, 4095), (1 << 20, 4095),
                                    (3 * (1 << 20) + 3, 63), (1 << 24, 4095)])
def test_hist_exact(cs, n, mask):
    keys = torch.empty(max(n, 1), dtype=torch.int32, device=DEV)[:n]
    bins = torch.full((4096,), 123, dtype=torch.int32, device=DEV)
    assert cs.sched_hist_fill(keys, 5) == 0
    assert cs.sched_hist(keys, bins, mask) == 0
    torch.cuda.synchronize()
    ref = T.hist_ref(5, n, mask=mask)
    got = bins.cpu().numpy().astype(np.int64)
    assert np.array_equal(got, ref) and got.sum() == n


def _gemm(cs, M, N, K, sa=1, sb=2):
    A = torch.empty(M * K, dtype=torch.int16, device=DEV)
    B = torch.empty(N * K, dtype=torch.int16, device=DEV)
    C = torch.full((M * N,), float("nan"), dtype=torch.float32, device=DEV)
    assert cs.sched_gemm_fill(A, M, K, sa) == 0
    assert cs.sched_gemm_fill(B, N, K, sb) == 0
    assert cs.sched_gemm_bf16(A, B, C, M, N, K) == 0
    torch.cuda.synchronize()
    return A, B, C.view(M, N)


def test_gemm_operands_exact(cs):
    A = torch.empty(4 * 64, dtype=torch.int16, device=DEV)
    assert cs.sched_gemm_fill(A, 4, 64, 9) == 0
    got = A.view(torch.bfloat16).float().cpu().numpy().astype(np.float64).reshape(4, 64)
    assert np.array_equal(got, T.gemm_operand(9, np.arange(4), 64))


# 128-tile kernel: (128, 128, 64), (256, 384, 192); 256-tile kernel: the
# others -- one k-tile (256, 256, 64), an odd count of k-tiles (512, 768, 320)
# and (256, 512, 192), a single tile column (4096, 256, 576), all with the
# plain tile order, and (2048, 2048, 128) with the XCD-grouped one.
@pytest.mark.parametrize("M,N,K", [(128, 128, 64), (256, 384, 192), (256, 256, 64),
                                   (256, 512, 192), (512, 768, 320), (4096, 256, 576),
                                   (1024, 1024, 1024), (2048, 2048, 128)])
def test_gemm_full(cs, M, N, K):
    _check_full(cs, M, N, K)


# Every entry of grids with more 256-tiles than the device has CUs, so that
# CUs run tiles one after another: (4096, 8192, 192) is 512 tiles in the XCD
# bands with an odd k-tile count, (8192, 4096, 64) 512 tiles of one k-tile
# each, (3072, 6144, 128) 288 tiles in the plain order.
@pytest.mark.parametrize("M,N,K", [(4096, 8192, 192), (8192, 4096, 64), (3072, 6144, 128)])
def test_gemm_full_many_tiles(cs, M, N, K):
    assert (M // 256) * (N // 256) > torch.cuda.get_device_properties(0).multi_processor_count
    _check_full(cs, M, N, K)


def _check_full(cs, M, N, K):
    _, _, C = _gemm(cs, M, N, K)
    ref = T.gemm_ref_full(1, 2, M, N, K)
    got = C.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() <= 2e-2, err.max()
    A = np.abs(T.gemm_operand(1, np.arange(M), K))
    B = np.abs(T.gemm_operand(2, np.arange(N), K))
    _assert_fp32_bound(got, ref, A @ B.T, K)


def _assert_fp32_bound(got, ref, abs_dot, K):
    """The operands are exact bf16 values with 8 significant bits, so every
    product a*b is exact in fp32 and the only error is the fp32 accumulation:
    for any summation order |c - r| <= gamma_K * sum_k |a_k b_k| with
    gamma_K = K u / (1 - K u), u = 2^-24.  A dropped or repeated k-step moves
    an entry by a whole product, far beyond this bound."""
    u = 2.0 ** -24
    gamma = K * u / (1 - K * u)
    bad = np.abs(got - ref) > gamma * abs_dot
    assert not bad.any(), (np.argwhere(bad)[:3], np.abs(got - ref).max())


@pytest.mark.parametrize("N", [2048, 4096, 8192])
def test_gemm_sampled(cs, N):
    _, _, C = _gemm(cs, N, N, N, 3, 4)
    rng = np.random.default_rng(N)
    mi = rng.integers(0, N, 512)
    ni = rng.integers(0, N, 512)
    mi[:2] = [0, N - 1]
    ni[:2] = [0, N - 1]
    ref = T.gemm_ref_entries(3, 4, N, mi, ni)
    got = C[torch.from_numpy(mi).to(DEV), torch.from_numpy(ni).to(DEV)].cpu().numpy()
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    assert err.max() <= 2e-2, err.max()
    A = np.abs(T.gemm_operand(3, mi, N))
    B = np.abs(T.gemm_operand(4, ni, N))
    _assert_fp32_bound(got.astype(np.float64), ref, np.einsum("ik,ik->i", A, B), N)


def test_tenant_bad_args(cs):
    x = torch.zeros(130, dtype=torch.int16, device=DEV)
    c = torch.zeros(4, dtype=torch.float32, device=DEV)
    assert cs.sched_gemm_bf16(x, x, c, 100, 128, 64) == cs.SCHED_E_INVALID
    k = torch.zeros(8, dtype=torch.int32, device=DEV)
    assert cs.sched_hist(k, torch.zeros(4096, dtype=torch.int32, device=DEV), 4096) == cs.SCHED_E_INVALID


def _sparse_rows(n, K, offsets):
    """k positions of the nonzero entries of each of n rows: for each offset
    function f, column f(r) (all within [0, K))."""
    return [sorted({f(r) % K for f in offsets}) for r in range(n)]


@pytest.mark.parametrize("K", [(1 << 22) - 64, 1 << 22])
def test_gemm_large_k_offsets(cs, K):
    """The 256-tile kernel addresses a 256-row panel with 32-bit byte offsets
    and takes K < 2^22; K = 2^22 - 64 puts its largest offsets within 0.4 % of
    2^31, and K = 2^22 goes to the 128-tile kernel.  Sparse exact operands (1.0
    in A, 2.0 in B) hit columns at the start, the middle and the last 64 of
    every row; the product is a small integer, exact in fp32."""
    M = N = 256
    a_cols = _sparse_rows(M, K, [lambda r: r % 64, lambda r: K // 2 + (7 * r) % 64,
                                 lambda r: K - 64 + r % 64])
    b_cols = _sparse_rows(N, K, [lambda r: (3 * r) % 64, lambda r: K // 2 + (5 * r) % 64,
                                 lambda r: K - 64 + r % 64])
    A = torch.zeros(M * K, dtype=torch.int16, device=DEV)
    B = torch.zeros(N * K, dtype=torch.int16, device=DEV)
    ia = torch.tensor([r * K + k for r in range(M) for k in a_cols[r]], dtype=torch.int64)
    ib = torch.tensor([r * K + k for r in range(N) for k in b_cols[r]], dtype=torch.int64)
    A[ia.to(DEV)] = 0x3F80  # bf16 1.0
    B[ib.to(DEV)] = 0x4000  # bf16 2.0
    C = torch.full((M * N,), float("nan"), dtype=torch.float32, device=DEV)
    assert cs.sched_gemm_bf16(A, B, C, M, N, K) == 0
    torch.cuda.synchronize()
    got = C.view(M, N).cpu().numpy().astype(np.float64)
    del A, B, C
    torch.cuda.empty_cache()
    # reference: the dense product restricted to the columns that hold nonzeros
    cols = sorted({k for r in a_cols for k in r} | {k for r in b_cols for k in r})
    pos = {k: i for i, k in enumerate(cols)}
    Ad = np.zeros((M, len(cols)))
    Bd = np.zeros((N, len(cols)))
    for r in range(M):
        Ad[r, [pos[k] for k in a_cols[r]]] = 1.0
    for r in range(N):
        Bd[r, [pos[k] for k in b_cols[r]]] = 2.0
    ref = Ad @ Bd.T
    assert ref.max() > 0 and np.array_equal(got, ref)
