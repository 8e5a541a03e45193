"""The algebra of the decomposition's standard form taken from the
resistance side (Sec. 3.2, eq. generalized_eigenvalues_discrete: the pencil
L_i v = tau R_i v), checked in dense numpy against the oracle on a small
electrode plate, on the CPU.  This pins the reading the GPU path is built
on, independently of its kernels:

* R_i = K^T R K = R'' - V Y^T - Y V^T restricted to the kept unknowns, with
  R'' = R[m:, m:] and the electrode term of rank 2m from the Householder
  complement K = H[:, m:] (H = I - V T V^T, the QR of E^T);
* R'' = Hc Hc^T and R_i = Hc A Hc^T with A = I + Z S Z^T, Z = Hc^{-1}[V, Y],
  S = -[[0, I], [I, 0]];
* A^{-1/2} = I + Z Gamma Z^T with Gamma from two small eigendecompositions
  (of Z^T Z and of the 2m x 2m core), so that
  C' = A^{-1/2} Hc^{-1} L_i Hc^{-T} A^{-1/2} = F^{-1} L_i F^{-T}
  (F = Hc A^{1/2}) has the time constants tau = 1 / lambda as eigenvalues;
* V = F^{-T} Q' T^{-1/2}, columns reversed, is L_i-orthonormal and
  diagonalises R_i to diag(lambda).

The oracle's eigenvalues come from its own Cholesky of L_i and Jacobi, so a
wrong sign, factor or transpose anywhere above fails the comparison."""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_2407_11993_amd import inputs


def _householder_complement(E):
    """H = I - V T V^T from the QR of E^T (m = rows of E), as the library
    forms it: V unit lower trapezoidal, T upper triangular."""
    n, m = E.shape[1], E.shape[0]
    (raw, tau), _ = sla.qr(E.T, mode="raw")
    V = np.tril(raw[:, :m], -1)
    V[np.arange(m), np.arange(m)] = 1.0
    T = np.zeros((m, m))
    for c in range(m):  # forward compact-WY recurrence
        T[:c, c] = -tau[c] * T[:c, :c] @ (V[:, :c].T @ V[:, c])
        T[c, c] = tau[c]
    return V, T


def _two_sided(A, V, T):
    """Y with H^T A H = A - V Y^T - Y V^T (H = I - V T V^T)."""
    X = A @ V
    return X @ T - 0.5 * V @ (T.T @ V.T @ X @ T)


@pytest.mark.parametrize("ew", [3, 4])
def test_rside_standard_form_matches_oracle(orc, ew):
    w = inputs.electrode_plate(10, 14, ew, T=10, tau_D=60.0, coil_period=120.0)
    L = orc.assemble_L(w.xyz, w.h)
    R = w.R.to_dense()
    E = w.E.to_dense()
    m = E.shape[0]
    n0 = w.n - m
    V, T = _householder_complement(E)
    K = (np.eye(w.n) - V @ T @ V.T)[:, m:]
    YL, YR = _two_sided(L, V, T), _two_sided(R, V, T)
    Li = (L - V @ YL.T - YL @ V.T)[m:, m:]
    Ri = (R - V @ YR.T - YR @ V.T)[m:, m:]
    assert np.abs(Li - K.T @ L @ K).max() < 1e-13 * np.abs(L).max()
    assert np.abs(Ri - K.T @ R @ K).max() < 1e-13 * np.abs(R).max()

    Hc = np.linalg.cholesky(R[m:, m:])
    Z = sla.solve_triangular(Hc, np.hstack([V[m:], YR[m:]]), lower=True)
    S = -np.block([[np.zeros((m, m)), np.eye(m)], [np.eye(m), np.zeros((m, m))]])
    A = np.eye(n0) + Z @ S @ Z.T
    assert np.abs(Hc @ A @ Hc.T - Ri).max() < 1e-12 * np.abs(Ri).max()

    # Gamma: Z^T Z = W diag(d) W^T; the core B = I + D^{1/2} W^T S W D^{1/2}
    d, W = np.linalg.eigh(Z.T @ Z)
    ds = np.sqrt(np.maximum(d, 0.0))
    B = np.eye(2 * m) + ds[:, None] * (W.T @ S @ W) * ds[None, :]
    db, Wb = np.linalg.eigh(B)
    assert db.min() > 0  # A is positive definite
    core = Wb @ np.diag(1.0 / np.sqrt(db) - 1.0) @ Wb.T
    Gamma = W @ (core / ds[:, None] / ds[None, :]) @ W.T
    Aih = np.eye(n0) + Z @ Gamma @ Z.T
    assert np.abs(Aih @ A @ Aih - np.eye(n0)).max() < 1e-12

    X = sla.solve_triangular(Hc, sla.solve_triangular(Hc, Li, lower=True).T, lower=True).T
    Cp = Aih @ X @ Aih
    tau, Qp = np.linalg.eigh(0.5 * (Cp + Cp.T))
    assert tau.min() > 0
    lam = 1.0 / tau[::-1]
    pb = orc.Problem(L, R, w.M, w.P, E=E)
    lam_ref = orc.modal_eigen(pb, want_V=False)
    assert np.max(np.abs(lam - lam_ref) / lam_ref) < 1e-10

    Vm = sla.solve_triangular(Hc.T, Qp + Z @ (Gamma @ (Z.T @ Qp)), lower=False)
    Vm = (Vm / np.sqrt(tau)[None, :])[:, ::-1]
    assert np.abs(Vm.T @ Li @ Vm - np.eye(n0)).max() < 1e-11
    assert np.abs(Vm.T @ Ri @ Vm - np.diag(lam)).max() < 1e-11 * lam.max()
