"""GPU unit tests of the two building blocks, through the kernel-level C entry points.

Each is compared with a plain float64 CPU computation of the same operation:
the MFMA GEMM (every layout, triangular and split-K mode, float64 and float32
operands, ragged sizes spanning several 128-tiles), the blocked Cholesky
fused with the inverse of its factor, and the outer-blocked Cholesky with
blocked triangular solves that forms the smoother gain.
"""
import numpy as np
import pytest
import torch

from paper_1107_4192_amd import kfmeg

pytestmark = pytest.mark.gpu

F = kfmeg


def _op(X, trans):
    return X.T if trans else X


CASES = [
    (1, 1, 1, 0), (15, 17, 3, 0), (64, 64, 64, 0), (128, 128, 16, 0), (130, 257, 33, 0),
    (306, 500, 500, 0), (129, 129, 200, F.G_TA), (200, 77, 129, F.G_TB), (257, 140, 65, F.G_TA | F.G_TB),
    (300, 300, 70, F.G_LOWER), (300, 300, 70, F.G_LOWER | F.G_MIRROR), (300, 300, 70, F.G_LOWER | F.G_MIRROR | F.G_TA),
    (306, 306, 5124, F.G_TB),
    # lower outputs of 9 and 17 tile rows: groups of 8 tile rows, the last one partial
    (1100, 1100, 40, F.G_LOWER | F.G_MIRROR), (2100, 2100, 20, F.G_LOWER | F.G_TB),
]


def _padded(X, dev="cuda"):
    """Copy X into a buffer whose leading dimension is a multiple of 16 (the fast path's layout)."""
    r, c = X.shape
    buf = torch.full((r, (c + 15) // 16 * 16), float("nan"), dtype=X.dtype, device=dev)
    buf[:, :c] = X.to(dev)
    return buf[:, :c]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("M,N,K,flags", CASES)
@pytest.mark.parametrize("ksplit", [1, 3])
@pytest.mark.parametrize("padded", [False, True])
def test_gemm_layouts(dtype, M, N, K, flags, ksplit, padded):
    g = torch.Generator().manual_seed(M * 7919 + N * 31 + K + flags * 101 + ksplit)
    ta, tb = bool(flags & F.G_TA), bool(flags & F.G_TB)
    A = torch.randn((K, M) if ta else (M, K), generator=g, dtype=torch.float64)
    B = torch.randn((N, K) if tb else (K, N), generator=g, dtype=torch.float64)
    Cin = torch.randn((M, N), generator=g, dtype=torch.float64)
    alpha, beta = -0.75, 1.25
    Ad, Bd = A.to(dtype), B.to(dtype)
    ref = alpha * (_op(Ad.double(), ta) @ _op(Bd.double(), tb)) + beta * Cin
    if padded:   # NaN padding: any read past the logical extent would poison the result
        C = F.kfd_gemm(_padded(Ad), _padded(Bd), M, N, K, flags, alpha, beta, Cin.cuda(), ksplit=ksplit).cpu()
    else:
        C = F.kfd_gemm(Ad.cuda(), Bd.cuda(), M, N, K, flags, alpha, beta, Cin.cuda(), ksplit=ksplit).cpu()
    tol = (1e-13 if dtype == torch.float64 else 2e-6) * K ** 0.5 * 4 + (1e-14 if dtype == torch.float64 else 1e-6)
    if flags & F.G_LOWER:
        low = torch.tril(torch.ones(M, N, dtype=torch.bool))
        assert (C[low] - ref[low]).abs().max() <= tol * max(1.0, ref.abs().max())
        if flags & F.G_MIRROR:
            assert torch.equal(C, C.T)
        else:
            assert torch.equal(C[~low], torch.zeros_like(C[~low]))
    else:
        assert (C - ref).abs().max() <= tol * max(1.0, ref.abs().max())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,k", [(200, 200), (300, 130), (129, 257)])
@pytest.mark.parametrize("padded", [False, True])
def test_gemm_triangular_operands(dtype, n, k, padded):
    g = torch.Generator().manual_seed(n + k)
    dev = _padded if padded else (lambda X: X.cuda())
    # A lower triangular (n x n) times B (n x k)
    A = torch.tril(torch.randn(n, n, generator=g, dtype=torch.float64)).to(dtype)
    B = torch.randn(n, k, generator=g, dtype=torch.float64).to(dtype)
    C = F.kfd_gemm(dev(A), dev(B), n, k, n, F.G_ALOWER).cpu()
    ref = A.double() @ B.double()
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert (C - ref).abs().max() <= tol * ref.abs().max()
    # G^T L with L lower (B lower: B(k,j) = 0 for k < j)
    G = torch.randn(n, k, generator=g, dtype=torch.float64).to(dtype)
    L = torch.tril(torch.randn(n, n, generator=g, dtype=torch.float64)).to(dtype)
    C = F.kfd_gemm(dev(G), dev(L), k, n, n, F.G_TA | F.G_BLOWER).cpu()
    ref = G.double().T @ L.double()
    assert (C - ref).abs().max() <= tol * ref.abs().max()
    # X L^T with L lower: B(k,j) = L[j][k], upper in (k,j)
    X = torch.randn(k, n, generator=g, dtype=torch.float64).to(dtype)
    C = F.kfd_gemm(dev(X), dev(L), k, n, n, F.G_TB | F.G_BUPPER).cpu()
    ref = X.double() @ L.double().T
    assert (C - ref).abs().max() <= tol * ref.abs().max()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("K,ksplit", [(20, 4), (3, 3), (33, 6), (50, 8)])
def test_gemm_split_slices_past_k(dtype, K, ksplit):
    """Split-K slices are whole multiples of 16 in k, so the last slices can start past K
    (K = 20 in 4 slices: [0, 16), [16, 20), then two empty ones). An empty slice must add
    nothing, also where its (negative) span is not a multiple of 16."""
    g = torch.Generator().manual_seed(K * 31 + ksplit)
    M, N = 200, 140
    A = torch.randn((M, K), generator=g, dtype=torch.float64)
    B = torch.randn((N, K), generator=g, dtype=torch.float64)
    Ad, Bd = A.to(dtype), B.to(dtype)
    ref = Ad.double() @ Bd.double().T
    for dev in (lambda X: X.cuda(), _padded):
        C = F.kfd_gemm(dev(Ad), dev(Bd), M, N, K, F.G_TB, 1.0, 0.0, ksplit=ksplit).cpu()
        tol = (1e-13 if dtype == torch.float64 else 2e-6) * K ** 0.5 * 4 + 1e-6
        assert (C - ref).abs().max() <= tol * max(1.0, ref.abs().max())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("flags", [0, F.G_TB, F.G_TA, F.G_TB | F.G_LOWER | F.G_MIRROR])
@pytest.mark.parametrize("full,k", [(0, 2), (7, 3), (20, 4), (35, 2)])
def test_gemm_tail_split(dtype, flags, full, k):
    # 6 x 6 tiles (21 lower): whole tiles first, the rest split along K with a tile-wise reduction
    M = N = 700
    K = 530
    g = torch.Generator().manual_seed(full * 13 + k + flags)
    ta, tb = bool(flags & F.G_TA), bool(flags & F.G_TB)
    A = torch.randn((K, M) if ta else (M, K), generator=g, dtype=torch.float64).to(dtype)
    B = torch.randn((N, K) if tb else (K, N), generator=g, dtype=torch.float64).to(dtype)
    Cin = torch.randn((M, N), generator=g, dtype=torch.float64)
    tiles = 21 if flags & F.G_LOWER else 36
    full = min(full, tiles)
    ref = -0.5 * (_op(A.double(), ta) @ _op(B.double(), tb)) + 2.0 * Cin
    C = F.kfd_gemm_tail(_padded(A), _padded(B), M, N, K, flags, -0.5, 2.0, Cin.cuda(), full=full, k=k).cpu()
    whole = F.kfd_gemm(_padded(A), _padded(B), M, N, K, flags, -0.5, 2.0, Cin.cuda()).cpu()
    tol = (1e-13 if dtype == torch.float64 else 2e-6) * K ** 0.5 * 4
    if flags & F.G_LOWER:
        low = torch.tril(torch.ones(M, N, dtype=torch.bool))
        assert (C[low] - ref[low]).abs().max() <= tol * ref.abs().max()
        assert torch.equal(C, C.T)
    else:
        assert (C - ref).abs().max() <= tol * ref.abs().max()
    # whole tiles are the same computation as without splitting: bitwise equal there
    assert torch.equal(C[:128, :128], whole[:128, :128]) or full == 0


def test_gemm_padded_leading_dimension():
    g = torch.Generator().manual_seed(5)
    big = torch.randn(300, 400, generator=g, dtype=torch.float64)
    A = big[:, :150]            # lda = 400
    B = torch.randn(150, 260, generator=g, dtype=torch.float64)
    C = F.kfd_gemm(big.cuda()[:, :150], B.cuda(), 300, 260, 150).cpu()
    assert (C - A @ B).abs().max() <= 1e-12 * (A @ B).abs().max()


def test_gemm_mfma_fragment_layout_single_tile():
    # One 16 x 16 x 4 product with distinct entries pins the lane layout of the MFMA operands and result.
    A = torch.arange(16 * 4, dtype=torch.float64).reshape(16, 4) / 7.0
    B = (torch.arange(4 * 16, dtype=torch.float64).reshape(4, 16) - 30.0) / 3.0
    C = F.kfd_gemm(A.cuda(), B.cuda(), 16, 16, 4).cpu()
    assert torch.allclose(C, A @ B, rtol=1e-15, atol=1e-13)


def _spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.logspace(-np.log10(cond), 0, n)
    A = (U * ev) @ U.T
    return (A + A.T) / 2


@pytest.mark.parametrize("n", [1, 2, 17, 63, 64, 65, 127, 128, 129, 200, 306, 500,
                               1024, 1025, 1300, 2100])   # up to nine 256-column panels
def test_chol_inv(n):
    A = _spd(n, n)
    # the strict upper triangle is never read: fill it with garbage
    W = torch.tril(torch.tensor(A, device="cuda")) + torch.triu(torch.full((n, n), 7.0, device="cuda", dtype=torch.float64), 1)
    Z = F.kfd_chol_inv(W)
    L = np.tril(W.cpu().numpy())          # the strict upper triangle of W is not part of the result
    Li = Z.cpu().numpy()
    Lref = np.linalg.cholesky(A)
    assert np.abs(L - Lref).max() <= 1e-12 * np.abs(Lref).max() * max(1, n) ** 0.5
    assert np.array_equal(np.triu(Li, 1), np.zeros((n, n)))
    assert np.abs(Li @ Lref - np.eye(n)).max() <= 1e-11 * max(1, n) ** 0.5 * 30


@pytest.mark.parametrize("n,row", [(150, 100), (150, 101), (1300, 1100), (70, 64), (70, 65)])
def test_chol_inv_reports_first_bad_pivot(n, row):
    A = _spd(n, 3, cond=10)
    A[row, row] = -1.0
    W = torch.tensor(A, device="cuda")
    with pytest.raises(kfmeg.KFError) as ei:
        F.kfd_chol_inv(W)
    assert ei.value.status == kfmeg.KF_ENOTPD
    assert f"pivot row {row}" in str(ei.value)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("n,k", [(200, 200), (300, 130), (129, 257)])
def test_gemm_a_upper_transposed(dtype, n, k):
    # U^T X with U lower triangular: A(i,k) = U[k][i], zero for k < i (upper in (i,k))
    g = torch.Generator().manual_seed(3 * n + k)
    U = torch.tril(torch.randn(n, n, generator=g, dtype=torch.float64)).to(dtype)
    X = torch.randn(n, k, generator=g, dtype=torch.float64).to(dtype)
    C = F.kfd_gemm(_padded(U), _padded(X), n, k, n, F.G_TA | F.G_AUPPER).cpu()
    ref = U.double().T @ X.double()
    tol = 1e-12 if dtype == torch.float64 else 2e-5
    assert (C - ref).abs().max() <= tol * ref.abs().max()


@pytest.mark.parametrize("n,nb", [(1, 1024), (63, 1024), (300, 128), (300, 64), (1000, 256), (1025, 1024),
                                  (2100, 1024), (2100, 512)])
def test_blocked_spd_solve(n, nb):
    """The smoother gain's factorisation and solves: several outer blocks with a ragged last one."""
    A = _spd(n, 7 * n + nb, cond=1e3)
    rng = np.random.default_rng(n)
    B = rng.normal(size=(n, n))
    W = torch.tril(torch.tensor(A, device="cuda")) + torch.triu(torch.full((n, n), 7.0, device="cuda",
                                                                            dtype=torch.float64), 1)
    X = F.kfd_spd_solve(W, torch.tensor(B, device="cuda"), nb).cpu().numpy()
    L = np.tril(W.cpu().numpy())
    Lref = np.linalg.cholesky(A)
    assert np.abs(L - Lref).max() <= 1e-12 * np.abs(Lref).max() * max(1, n) ** 0.5
    ref = np.linalg.solve(A, B)
    assert np.abs(X - ref).max() <= 1e-9 * np.abs(ref).max()      # cond 1e3
    assert np.abs(A @ X - B).max() <= 1e-11 * np.abs(B).max() * max(1, n) ** 0.5


@pytest.mark.parametrize("n,nb,row", [(300, 128, 200), (300, 128, 5), (2100, 1024, 2050)])
def test_blocked_spd_solve_reports_bad_pivot(n, nb, row):
    A = _spd(n, 3, cond=10)
    A[row, row] = -1.0
    W = torch.tensor(A, device="cuda")
    with pytest.raises(kfmeg.KFError) as ei:
        F.kfd_spd_solve(W, torch.eye(n, dtype=torch.float64, device="cuda"), nb)
    assert ei.value.status == kfmeg.KF_ENOTPD
    assert f"pivot row {row}" in str(ei.value)
