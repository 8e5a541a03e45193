"""Stage-by-stage parity of the HIP building blocks (FP64) against plain
numpy/scipy definitions: GEMM, Cholesky, triangular inverse, band reduction,
bulge chase, divide and conquer, and the full symmetric eigensolver.

Sizes span several tiles and a ragged tail (128-wide tiles and panels, 64
band, 32-row D&C leaves)."""
import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    assert torch.cuda.is_available()
    from paper_2407_11993_amd import kernels
    return kernels


def _np(t):
    return t.detach().cpu().numpy()


def _sym(n, seed, spread=1.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) * spread
    return (A + A.T) / 2


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    return A @ A.T / n + np.eye(n)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (17, 33, 5), (130, 70, 200),
                                   (257, 129, 64), (64, 64, 4096), (2100, 2100, 300),
                                   (16500, 61, 300), (16500, 64, 8192)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm(K, m, n, k, ta, tb):
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    A = rng.standard_normal((k, m) if ta else (m, k))
    B = rng.standard_normal((n, k) if tb else (k, n))
    C0 = rng.standard_normal((m, n))
    ref = 0.5 * ((A.T if ta else A) @ (B.T if tb else B)) - 2.0 * C0
    out = _np(K.gemm(A, B, ta, tb, alpha=0.5, beta=-2.0, C=C0))
    scale = np.abs(A).max() * np.abs(B).max() * k + 2 * np.abs(C0).max()
    assert np.abs(out - ref).max() <= 1e-15 * scale * 4


MMK_LOWER, MMK_A_LOWER, MMK_A_UPPER, MMK_B_LOWER = 1, 2, 4, 8


# the structure flags on both tile sizes (2100 x 2200 uses 128 x 128 tiles)
@pytest.mark.parametrize("m,n,k", [(300, 260, 280), (2100, 2200, 2150), (16500, 64, 1100)])
@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False)])
@pytest.mark.parametrize("flags,b_band", [(MMK_LOWER, -1), (MMK_A_LOWER, -1), (MMK_A_UPPER, -1),
                                          (MMK_B_LOWER, -1), (0, 40),
                                          (MMK_LOWER | MMK_A_LOWER, 70)])
def test_gemm_tri(K, m, n, k, ta, tb, flags, b_band):
    rng = np.random.default_rng(m + n + k + flags + b_band)
    opA = rng.standard_normal((m, k))
    opB = rng.standard_normal((k, n))
    if flags & MMK_A_LOWER:
        opA = np.tril(opA)
    if flags & MMK_A_UPPER:
        opA = np.triu(opA)
    if flags & MMK_B_LOWER:
        opB = np.tril(opB)
    if b_band >= 0:
        opB = np.triu(opB, -b_band)
    C0 = rng.standard_normal((m, n))
    ref = 0.5 * (opA @ opB) - 2.0 * C0
    if flags & MMK_LOWER:
        ref = np.where(np.tril(np.ones((m, n), dtype=bool)), ref, C0)
    out = _np(K.gemm_tri(opA.T.copy() if ta else opA, opB.T.copy() if tb else opB, ta, tb,
                         alpha=0.5, beta=-2.0, C=C0, flags=flags, b_band=b_band))
    scale = np.abs(opA).max() * np.abs(opB).max() * k + 2 * np.abs(C0).max()
    assert np.abs(out - ref).max() <= 1e-15 * scale * 4


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (130, 70), (257, 129), (2100, 2100),
                                 (4096, 1030), (16400, 64)])
def test_symm_lower(K, m, n):
    """The upper triangle of A holds NaN: a read of it would show in C."""
    rng = np.random.default_rng(m + 5 * n)
    S = _sym(m, m + 1)
    A = np.tril(S) + np.triu(np.full((m, m), np.nan), 1)
    B = rng.standard_normal((m, n))
    C0 = rng.standard_normal((m, n))
    ref = 0.5 * (S @ B) - 2.0 * C0
    out = _np(K.symm_lower(A, B, alpha=0.5, beta=-2.0, C=C0))
    scale = np.abs(S).max() * np.abs(B).max() * m + 2 * np.abs(C0).max()
    assert np.abs(out - ref).max() <= 1e-15 * scale * 4


# 2600: the trailing updates run on 128 x 128 tiles (lower output, B transposed)
@pytest.mark.parametrize("n", [1, 5, 128, 129, 300, 513, 2600])
def test_potrf(K, n):
    A = _spd(n, n)
    G, info = K.potrf(A)
    G = _np(G)
    assert info == -1
    assert np.all(np.triu(G, 1) == 0)
    assert np.abs(G - np.linalg.cholesky(A)).max() < 1e-12
    assert np.abs(G @ G.T - A).max() < 1e-13 * np.abs(A).max() * max(1, np.sqrt(n))


# diagonal blocks are factored in pairs: the first failing pivot is reported
# from either block of a pair
@pytest.mark.parametrize("n,piv", [(200, 150), (400, 100), (400, 150), (400, 300)])
def test_potrf_reports_pivot(K, n, piv):
    A = _spd(n, 1)
    A[piv, piv] = -5.0
    _, info = K.potrf(A)
    assert info == piv


# 4300: the top-level products run on 128 x 128 tiles (triangular operands)
@pytest.mark.parametrize("n", [1, 100, 128, 129, 300, 700, 4300])
def test_trtri(K, n):
    G = np.linalg.cholesky(_spd(n, n + 11))
    Gi = _np(K.trtri(G))
    assert np.all(np.triu(Gi, 1) == 0)
    ref = sla.solve_triangular(G, np.eye(n), lower=True)
    assert np.abs(Gi - ref).max() < 1e-12 * np.abs(ref).max()


def _band_dense(AB, n, nb):
    B = np.zeros((n, n))
    for d in range(nb + 1):
        for j in range(n - d):
            B[j + d, j] = AB[j, d]
            B[j, j + d] = AB[j, d]
    return B


# panels are reduced in pairs (an odd count ends with a single one); 2600 runs
# the updates on 128-row tiles
@pytest.mark.parametrize("n,nb", [(3, 1), (70, 16), (200, 64), (333, 64), (129, 32),
                                  (140, 16), (2600, 64)])
def test_sy2sb_preserves_spectrum(K, n, nb):
    A = _sym(n, n + nb)
    AB = _np(K.sy2sb(A, nb))
    assert np.all(AB[:, nb + 1:] == 0)
    # only the lower triangle is read: NaN above it changes nothing
    Au = np.tril(A) + np.triu(np.full((n, n), np.nan), 1)
    assert np.array_equal(_np(K.sy2sb(Au, nb)), AB)
    B = _band_dense(AB, n, nb)
    ev = np.linalg.eigvalsh(A)
    eb = np.linalg.eigvalsh(B)
    assert np.abs(ev - eb).max() < 1e-13 * np.abs(ev).max() * np.sqrt(n)


@pytest.mark.parametrize("n,nb", [(3, 1), (5, 2), (150, 8), (200, 64), (301, 64)])
def test_sb2st_preserves_spectrum(K, n, nb):
    rng = np.random.default_rng(n)
    B = np.zeros((n, n))
    for d in range(nb + 1):
        v = rng.standard_normal(n - d)
        B += np.diag(v, -d) + (np.diag(v, d) if d else 0)
    AB = np.zeros((n, 2 * nb + 1))
    for d in range(nb + 1):
        AB[:n - d, d] = np.diag(B, -d)
    d_, e_ = K.sb2st(AB, nb)
    T = np.diag(_np(d_)) + np.diag(_np(e_), 1) + np.diag(_np(e_), -1)
    ev = np.linalg.eigvalsh(B)
    assert np.abs(np.linalg.eigvalsh(T) - ev).max() < 1e-13 * np.abs(ev).max() * np.sqrt(n)


def _check_eig(A, w, Z, tol=1e-13):
    n = A.shape[0]
    scale = max(np.abs(np.linalg.eigvalsh(A)).max(), 1e-300)
    assert np.all(np.diff(w) >= 0)
    assert np.abs(w - np.linalg.eigvalsh(A)).max() < tol * scale * max(1, np.sqrt(n))
    assert np.abs(Z.T @ Z - np.eye(n)).max() < tol * 10 * max(1, np.sqrt(n))
    assert np.abs(A @ Z - Z * w).max() < tol * 10 * scale * max(1, np.sqrt(n))


@pytest.mark.parametrize("n", [1, 2, 5, 31, 32, 33, 64, 100, 257, 600])
def test_stedc_random(K, n):
    rng = np.random.default_rng(n + 100)
    d = rng.standard_normal(n)
    e = rng.standard_normal(max(n - 1, 0))
    w, Z = K.stedc(d, e)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    _check_eig(T, _np(w), _np(Z))


@pytest.mark.parametrize("kind", ["zero_couplings", "repeated", "graded", "wilkinson"])
def test_stedc_structured(K, kind):
    n = 200
    rng = np.random.default_rng(7)
    if kind == "zero_couplings":
        d = rng.standard_normal(n)
        e = rng.standard_normal(n - 1)
        e[::7] = 0.0
    elif kind == "repeated":
        d = np.repeat(rng.standard_normal(n // 10), 10)
        e = 1e-3 * rng.standard_normal(n - 1)
        e[9::10] = 0.0
    elif kind == "graded":
        d = 10.0 ** np.linspace(-8, 4, n)
        e = np.sqrt(d[:-1] * d[1:]) * 0.1
    else:
        m = (n - 1) / 2
        d = np.abs(np.arange(n) - m)
        e = np.ones(n - 1)
    w, Z = K.stedc(d, e)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    _check_eig(T, _np(w), _np(Z))


@pytest.mark.parametrize("n", [1, 3, 50, 200, 301])
def test_syevd(K, n):
    A = _sym(n, 3 * n + 1)
    w, Z = K.syevd(A)
    _check_eig(A, _np(w), _np(Z))


@pytest.mark.parametrize("n,nb", [(200, 16), (230, 40), (700, 64)])
def test_syevd_band_widths(K, n, nb):
    # nb < 64 takes the back-transform path without window reuse; n = 700
    # chains many consecutive blocks per group of 64 sweeps
    A = _sym(n, 5 * n + nb)
    w, Z = K.syevd(A, nb=nb)
    _check_eig(A, _np(w), _np(Z))


def test_syevd_clustered(K):
    n = 256
    rng = np.random.default_rng(3)
    Qr, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([np.full(60, 1.0), np.full(60, 2.0), rng.uniform(3, 4, n - 120)])
    A = (Qr * lam) @ Qr.T
    A = (A + A.T) / 2
    w, Z = K.syevd(A)
    _check_eig(A, _np(w), _np(Z), tol=5e-13)


def _check_eig_gpu(apply_A, w, Z, scale, tol):
    """Residual and orthogonality on the GPU (torch products) for sizes where
    a dense numpy check would take minutes; w sorted."""
    import torch
    n = Z.shape[0]
    assert bool(torch.all(w[1:] >= w[:-1]))
    eye = torch.eye(n, dtype=torch.float64, device=Z.device)
    orth = float((Z.T @ Z - eye).abs().max())
    res = float((apply_A(Z) - Z * w).abs().max())
    assert orth < tol * np.sqrt(n), orth
    assert res < tol * scale * np.sqrt(n), res


def test_stedc_two_row_chunks(K):
    """n = 12,000: the merges are applied to the eigenvector matrix in two
    chunks of rows (11,184 and a ragged 816)."""
    import torch
    n = 12000
    rng = np.random.default_rng(12)
    d = rng.standard_normal(n)
    e = rng.standard_normal(n - 1)
    e[::997] = 0.0  # a few exact splits deflate whole subproblems
    w, Z = K.stedc(d, e)
    ref = sla.eigvalsh_tridiagonal(d, e)
    scale = np.abs(ref).max()
    assert np.abs(_np(w) - ref).max() < 1e-13 * scale * np.sqrt(n)
    dt = torch.as_tensor(d, device="cuda")
    et = torch.as_tensor(e, device="cuda")

    def T_times(X):
        Y = dt[:, None] * X
        Y[:-1] += et[:, None] * X[1:]
        Y[1:] += et[:, None] * X[:-1]
        return Y
    _check_eig_gpu(T_times, w, Z, scale, 1e-13)


def test_syevd_two_row_chunks(K):
    """n = 11,700, a dense symmetric matrix with a known spectrum (clusters
    included): the back-transform of the leaves, then the merges in two
    chunks of rows."""
    import torch
    n = 11700
    g = torch.Generator(device="cuda").manual_seed(5)
    Qr, _ = torch.linalg.qr(torch.randn(n, n, dtype=torch.float64, device="cuda", generator=g))
    lam = torch.cat([torch.full((300,), 1.0), torch.full((200,), -2.0),
                     torch.linspace(-5.0, 7.0, n - 500)]).to(torch.float64).cuda()
    A = (Qr * lam) @ Qr.T
    A = (A + A.T) / 2
    w, Z = K.syevd(A)
    ref = torch.sort(lam).values
    assert float((w - ref).abs().max()) < 1e-13 * 7.0 * np.sqrt(n)
    _check_eig_gpu(lambda X: A @ X, w, Z, 7.0, 1e-13)
