"""Plain FP64 CPU oracle (ctypes wrapper around ``oracle.c``).

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
definition that the GPU library is checked against.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does, and it shares no code with the GPU library.

Every function follows the paper's equations (Ventre et al., "Modal
Decomposition in Numerical Computation of Eddy Current Transients"):

* ``assemble_L``        -- the dense SPD inductance stand-in (Sec. 3.1, L_jk).
* ``cholesky``          -- Z = C C^T (Sec. 3.3.1).
* ``jacobi_eig``        -- cyclic Jacobi (Golub & Van Loan 8.5) for C = Q Lam Q^T.
* ``standard_form``     -- C = G^{-1} Ri G^{-T} for the pencil of Sec. 3.2.
* ``null_basis``        -- K, an orthonormal basis of ker E (Sec. 3.1).
* ``theta_direct``      -- the Cholesky theta-method (Sec. 3.3.1, eq. time_integration).
* ``theta_modal``       -- the modal theta-method (Sec. 3.3.2).
* ``modal_eigen``       -- eigenvalues and Li-normalised eigenvectors (Sec. 3.2).
* ``time_constants``    -- the eigenvalues tau of Li v = tau Ri v as the paper writes
                           them (Sec. 3.2), from the standard form on Ri's side.
* ``exact_modal``       -- the decoupled modal equations of Sec. 3.2 integrated in
                           closed form over each step, waveforms linear between
                           samples (the analytical route of Sec. 3.3 left to later work).
* ``exact_phi``         -- the two step integrals that closed form uses.
* ``mode_weights``      -- the modal forcing and probe weights (Sec. 3.2).
* ``select_modes``      -- the modes kept by the selective solution of Sec. 3.2
                           (coupling score above a relative tolerance); the
                           modal steppers take the kept set as ``keep``.
* ``phasors_direct``    -- steady-state probe phasors under sinusoidal sources: one
                           complex solve of the unreduced system per frequency (the
                           frequency-domain method of Sec. 4.6).
* ``adjoint_direct``    -- gradient of a probe-signal misfit through the
                           theta-method (adjoint recursion, every state kept).
* ``ldlt_inertia``      -- Sylvester inertia of a symmetric matrix (Bunch-Kaufman
                           LDL^T).
* ``inertia``           -- the number of eigenvalues of the pencil of Sec. 3.2
                           below, at and above a shift sigma (inertia of Ri - sigma Li).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_i64 = ctypes.c_int64


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` with gcc into ``liboracle.so`` (plain -O2, FP64)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
             "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.orc_assemble_L.argtypes = [_i64, _dp, ctypes.c_double, _dp]
        lib.orc_cholesky.argtypes = [_i64, _dp]
        lib.orc_cholesky.restype = _i64
        lib.orc_forward.argtypes = [_i64, _dp, _dp]
        lib.orc_backward_T.argtypes = [_i64, _dp, _dp]
        lib.orc_jacobi.argtypes = [_i64, _dp, _dp, _dp, ctypes.c_int]
        lib.orc_jacobi.restype = ctypes.c_int
        lib.orc_null_basis.argtypes = [_i64, _i64, _dp, _dp]
        lib.orc_null_basis.restype = ctypes.c_int
        lib.orc_standard_form.argtypes = [_i64, _dp, _dp, _dp]
        lib.orc_theta_direct.argtypes = [
            ctypes.POINTER(_Problem), ctypes.c_double, ctypes.c_double, _i64,
            _dp, _dp, _dp, _dp]
        lib.orc_theta_direct.restype = ctypes.c_int
        lib.orc_theta_modal.argtypes = [
            ctypes.POINTER(_Problem), ctypes.c_double, ctypes.c_double, _i64,
            _dp, _dp, _dp, _dp, _dp, _u8p]
        lib.orc_theta_modal.restype = ctypes.c_int
        lib.orc_exact_modal.argtypes = [
            ctypes.POINTER(_Problem), ctypes.c_double, _i64, _dp, _dp, _dp, _dp, _u8p]
        lib.orc_exact_modal.restype = ctypes.c_int
        lib.orc_mode_weights.argtypes = [ctypes.POINTER(_Problem), _dp, _dp, _dp]
        lib.orc_mode_weights.restype = ctypes.c_int
        lib.orc_exact_phi.argtypes = [ctypes.c_double, ctypes.c_double, _dp, _dp]
        lib.orc_modal_eigen.argtypes = [
            ctypes.POINTER(_Problem), _dp, _dp, ctypes.POINTER(ctypes.c_int)]
        lib.orc_modal_eigen.restype = ctypes.c_int
        lib.orc_time_constants.argtypes = [ctypes.POINTER(_Problem), _dp]
        lib.orc_time_constants.restype = ctypes.c_int
        lib.orc_adjoint_direct.argtypes = [
            _i64, _dp, _dp, _i64, _dp, _dp, ctypes.c_double, ctypes.c_double, _i64,
            _dp, _dp, _dp, _dp, _dp]
        lib.orc_adjoint_direct.restype = ctypes.c_int
        lib.orc_ldlt_inertia.argtypes = [_i64, _dp, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_inertia.argtypes = [ctypes.POINTER(_Problem), ctypes.c_double,
                                    ctypes.POINTER(ctypes.c_int64)]
        lib.orc_inertia.restype = ctypes.c_int
        _lib = lib
    return _lib


class _Problem(ctypes.Structure):
    _fields_ = [("n", _i64), ("m", _i64), ("n_src", _i64), ("n_probe", _i64),
                ("L", _dp), ("R", _dp), ("E", _dp), ("M", _dp), ("P", _dp)]


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


# ---------------------------------------------------------------------------
# elementary pieces
# ---------------------------------------------------------------------------
def assemble_L(xyz, h: float) -> np.ndarray:
    """L_ij = h / sqrt(|x_i - x_j|^2 + h^2) (dense SPD inductance stand-in)."""
    xyz = _f64(xyz)
    n = xyz.shape[0]
    out = np.empty((n, n))
    _load().orc_assemble_L(n, _ptr(xyz), float(h), _ptr(out))
    return out


def cholesky(A) -> np.ndarray:
    """Lower Cholesky factor; raises ValueError with the failing pivot."""
    G = _f64(A).copy()
    piv = _load().orc_cholesky(G.shape[0], _ptr(G))
    if piv >= 0:
        raise ValueError(f"not positive definite at pivot {piv}")
    return G


def forward(G, b) -> np.ndarray:
    G = _f64(G)
    x = _f64(b).copy()
    _load().orc_forward(G.shape[0], _ptr(G), _ptr(x))
    return x


def backward_T(G, b) -> np.ndarray:
    G = _f64(G)
    x = _f64(b).copy()
    _load().orc_backward_T(G.shape[0], _ptr(G), _ptr(x))
    return x


def jacobi_eig(A, max_sweeps: int = 100):
    """Cyclic Jacobi: returns (lam ascending, Q, sweeps)."""
    A = _f64(A).copy()
    n = A.shape[0]
    Q = np.empty((n, n))
    lam = np.empty(n)
    sw = _load().orc_jacobi(n, _ptr(A), _ptr(Q), _ptr(lam), int(max_sweeps))
    if sw < 0:
        raise RuntimeError("Jacobi did not converge")
    return lam, Q, sw


def null_basis(E) -> np.ndarray:
    E = _f64(np.atleast_2d(E))
    m, n = E.shape
    K = np.empty((n, n - m))
    if _load().orc_null_basis(m, n, _ptr(E), _ptr(K)):
        raise ValueError("E is rank deficient")
    return K


def standard_form(G, Ri) -> np.ndarray:
    G = _f64(G)
    Ri = _f64(Ri)
    C = np.empty_like(G)
    _load().orc_standard_form(G.shape[0], _ptr(G), _ptr(Ri), _ptr(C))
    return C


# ---------------------------------------------------------------------------
# problems and the two theta-methods
# ---------------------------------------------------------------------------
class Problem:
    """Dense problem statement  R I + L I' + E^T phi = -M0 i0',  E I = iD.

    L, R: n x n; E: m x n (m = Ne - 1, may be 0); M: n x n_src;
    P: n_probe x n probe rows.
    """

    def __init__(self, L, R, M, P, E=None):
        self.L = _f64(L)
        self.R = _f64(R)
        n = self.L.shape[0]
        self.M = _f64(np.asarray(M).reshape(n, -1))
        self.P = _f64(np.atleast_2d(P))
        if E is None or np.size(E) == 0:
            self.E = np.zeros((0, n))
        else:
            self.E = _f64(np.atleast_2d(E))
        self.n = n
        self.m = self.E.shape[0]
        self.n_src = self.M.shape[1]
        self.n_probe = self.P.shape[0]

    def _struct(self) -> _Problem:
        dummy = np.zeros(1)
        self._keep = dummy
        return _Problem(self.n, self.m, self.n_src, self.n_probe,
                        _ptr(self.L), _ptr(self.R),
                        _ptr(self.E) if self.m else _ptr(dummy),
                        _ptr(self.M) if self.n_src else _ptr(dummy),
                        _ptr(self.P) if self.n_probe else _ptr(dummy))

    def _waves(self, T, i_src, i_D):
        i_src = _f64(np.zeros((T + 1, 0)) if i_src is None else
                     np.asarray(i_src).reshape(T + 1, -1))
        i_D = _f64(np.zeros((T + 1, 0)) if i_D is None else
                   np.asarray(i_D).reshape(T + 1, -1))
        assert i_src.shape[1] == self.n_src and i_D.shape[1] == self.m
        if i_src.size == 0:
            i_src = np.zeros(1)
        if i_D.size == 0:
            i_D = np.zeros(1)
        return i_src, i_D


_ERR = {1: "electrode matrix E is rank deficient",
        2: "matrix not positive definite",
        3: "Jacobi did not converge"}


def theta_direct(pb: Problem, theta: float, dt: float, T: int, i_src=None,
                 i_D=None, want_I: bool = False):
    """Cholesky theta-method; returns signal (T x n_probe) [, I_hist]."""
    i_src, i_D = pb._waves(T, i_src, i_D)
    sig = np.zeros((T, max(pb.n_probe, 1)))
    I_hist = np.zeros((T + 1, pb.n)) if want_I else None
    st = pb._struct()
    rc = _load().orc_theta_direct(ctypes.byref(st), float(theta), float(dt),
                                  int(T), _ptr(i_src), _ptr(i_D), _ptr(sig),
                                  _ptr(I_hist))
    if rc:
        raise RuntimeError(_ERR.get(rc, str(rc)))
    sig = sig[:, :pb.n_probe]
    return (sig, I_hist) if want_I else sig


def _keep(pb: Problem, keep):
    if keep is None:
        return None
    k = np.ascontiguousarray(np.asarray(keep, dtype=bool).astype(np.uint8))
    assert k.shape == (pb.n - pb.m,)
    return k


def theta_modal(pb: Problem, theta: float, dt: float, T: int, i_src=None,
                i_D=None, want_I: bool = False, keep=None):
    """Modal theta-method; returns (signal, lam) [+ I_hist].  keep (n0
    booleans, modes in ascending eigenvalue order) steps only those modes."""
    i_src, i_D = pb._waves(T, i_src, i_D)
    kp = _keep(pb, keep)
    sig = np.zeros((T, max(pb.n_probe, 1)))
    lam = np.zeros(pb.n - pb.m)
    I_hist = np.zeros((T + 1, pb.n)) if want_I else None
    st = pb._struct()
    rc = _load().orc_theta_modal(ctypes.byref(st), float(theta), float(dt),
                                 int(T), _ptr(i_src), _ptr(i_D), _ptr(sig),
                                 _ptr(lam), _ptr(I_hist),
                                 None if kp is None else kp.ctypes.data_as(_u8p))
    if rc:
        raise RuntimeError(_ERR.get(rc, str(rc)))
    sig = sig[:, :pb.n_probe]
    return (sig, lam, I_hist) if want_I else (sig, lam)


def exact_modal(pb: Problem, dt: float, T: int, i_src=None, i_D=None,
                want_I: bool = False, keep=None):
    """Modal stepping with exact per-mode integration of waveforms that are
    linear between samples; returns signal (T x n_probe) [, I_hist].  keep
    as in theta_modal."""
    i_src, i_D = pb._waves(T, i_src, i_D)
    kp = _keep(pb, keep)
    sig = np.zeros((T, max(pb.n_probe, 1)))
    I_hist = np.zeros((T + 1, pb.n)) if want_I else None
    st = pb._struct()
    rc = _load().orc_exact_modal(ctypes.byref(st), float(dt), int(T), _ptr(i_src),
                                 _ptr(i_D), _ptr(sig), _ptr(I_hist),
                                 None if kp is None else kp.ctypes.data_as(_u8p))
    if rc:
        raise RuntimeError(_ERR.get(rc, str(rc)))
    sig = sig[:, :pb.n_probe]
    return (sig, I_hist) if want_I else sig


def exact_phi(lam: float, dt: float):
    """(phi1, phi2): the integrals of exp(-lam (dt - s)) and of s exp(-lam (dt - s))
    over [0, dt] that the exact step uses."""
    a = np.zeros(1)
    b = np.zeros(1)
    _load().orc_exact_phi(float(lam), float(dt), _ptr(a), _ptr(b))
    return float(a[0]), float(b[0])


def phasors_direct(pb: Problem, omegas, amp_src, amp_D=None):
    """Steady-state phasors of the probe signals P dI/dt for sources
    i0_c(t) = Re{amp_src[w, c] exp(j omega_w t)} and electrode currents
    iD_a(t) = Re{amp_D[w, a] exp(j omega_w t)}: for every frequency the
    unreduced circuit system of Sec. 3.1 in phasor form,
        (R + j omega L) I + E^T phi = -j omega M0 I0,   E I = ID,
    is solved directly (complex LU), and the probe phasor is j omega P I.
    Returns n_w x n_probe complex."""
    omegas = np.asarray(omegas, dtype=np.float64).reshape(-1)
    n, m = pb.n, pb.m
    amp_src = np.asarray(amp_src, dtype=np.complex128).reshape(len(omegas), pb.n_src)
    if m:
        amp_D = np.asarray(amp_D, dtype=np.complex128).reshape(len(omegas), m)
    out = np.zeros((len(omegas), pb.n_probe), dtype=np.complex128)
    for w, om in enumerate(omegas):
        A = np.zeros((n + m, n + m), dtype=np.complex128)
        A[:n, :n] = pb.R + 1j * om * pb.L
        rhs = np.zeros(n + m, dtype=np.complex128)
        rhs[:n] = -1j * om * (pb.M @ amp_src[w])
        if m:
            A[:n, n:] = pb.E.T
            A[n:, :n] = pb.E
            rhs[n:] = amp_D[w]
        I = np.linalg.solve(A, rhs)[:n]
        out[w] = 1j * om * (pb.P @ I)
    return out


def mode_weights(pb: Problem):
    """(lam, W, Pw): eigenvalues (ascending), the modal forcing weights
    W = V^T [R_D | L_D | K^T M0] (n0 x (2m + n_src)) and the modal probe weights
    Pw = (P K V)^T (n0 x n_probe), V the Li-normalised eigenvectors (Sec. 3.2)."""
    n0 = pb.n - pb.m
    nf = 2 * pb.m + pb.n_src
    lam = np.zeros(n0)
    W = np.zeros((n0, max(nf, 1)))
    Pw = np.zeros((n0, max(pb.n_probe, 1)))
    st = pb._struct()
    rc = _load().orc_mode_weights(ctypes.byref(st), _ptr(lam), _ptr(W), _ptr(Pw))
    if rc:
        raise RuntimeError(_ERR.get(rc, str(rc)))
    return lam, W[:, :nf], Pw[:, :pb.n_probe]


def select_modes(pb: Problem, tol: float):
    """Selective solution of the decoupled modal equations (Sec. 3.2, reading
    13): mode n is kept when its coupling score
        score_n = max_j |W(n, j)| * max_p |Pw(n, p)|
    exceeds tol times the largest score (tol >= 0; every source and electrode
    column counts with unit amplitude).  A mode with score 0 is never excited
    or never seen, so tol = 0 drops only modes that cannot change a probe
    signal.  Returns (keep, score), keep a boolean per mode in ascending
    eigenvalue order."""
    assert tol >= 0
    _, W, Pw = mode_weights(pb)
    a = np.abs(W).max(axis=1) if W.shape[1] else np.zeros(W.shape[0])
    b = np.abs(Pw).max(axis=1) if Pw.shape[1] else np.zeros(Pw.shape[0])
    score = a * b
    top = score.max() if score.size else 0.0
    return score > tol * top, score


def modal_eigen(pb: Problem, want_V: bool = True):
    """Eigenvalues (ascending) and Li-normalised eigenvectors of (Ri, Li)."""
    n0 = pb.n - pb.m
    lam = np.zeros(n0)
    V = np.zeros((n0, n0)) if want_V else None
    sw = ctypes.c_int(0)
    st = pb._struct()
    rc = _load().orc_modal_eigen(ctypes.byref(st), _ptr(lam), _ptr(V),
                                 ctypes.byref(sw))
    if rc:
        raise RuntimeError(_ERR.get(rc, str(rc)))
    return (lam, V) if want_V else lam


def time_constants(pb: Problem):
    """The pencil's eigenvalues as the paper writes them (Sec. 3.2, eq.
    generalized_eigenvalues_discrete: Li v = tau Ri v), in its order
    tau_1 >= tau_2 >= ... (Sec. 2.3), from the standard form on Ri's side:
    Ri = H H^T, Jacobi on H^{-1} Li H^{-T}."""
    n0 = pb.n - pb.m
    tau = np.zeros(n0)
    st = pb._struct()
    rc = _load().orc_time_constants(ctypes.byref(st), _ptr(tau))
    if rc:
        raise RuntimeError(_ERR.get(rc, str(rc)))
    return np.sort(tau)[::-1].copy()


def adjoint_direct(L, R, M, P, theta: float, dt: float, T: int, i_src, obs):
    """Misfit J = sum_c sum_k (s_c^{k+1} - obs[c, k])^2 over runs c (source
    column c of M, probe row c of P, shared waveform i_src of T+1 samples) and
    its gradients: dJ/dR (n x n, every entry independent) and dJ/di (T+1)."""
    L = _f64(L)
    R = _f64(R)
    n = L.shape[0]
    M = _f64(np.asarray(M).reshape(n, -1))
    C = M.shape[1]
    P = _f64(np.atleast_2d(P))
    assert P.shape == (C, n)
    i_src = _f64(np.asarray(i_src).reshape(T + 1))
    obs = _f64(np.asarray(obs).reshape(C, T))
    J = np.zeros(1)
    dJdR = np.zeros((n, n))
    dJdi = np.zeros(T + 1)
    rc = _load().orc_adjoint_direct(n, _ptr(L), _ptr(R), C, _ptr(M), _ptr(P), float(theta),
                                    float(dt), int(T), _ptr(i_src), _ptr(obs), _ptr(J),
                                    _ptr(dJdR), _ptr(dJdi))
    if rc:
        raise RuntimeError(_ERR.get(rc, str(rc)))
    return float(J[0]), dJdR, dJdi


def ldlt_inertia(A):
    """(negative, zero, positive) eigenvalue counts of the symmetric matrix A
    (only its lower triangle is read), from the block-diagonal D of its
    Bunch-Kaufman factorisation P A P^T = L D L^T (Sylvester's law of inertia)."""
    A = _f64(A).copy()
    counts = (ctypes.c_int64 * 3)()
    _load().orc_ldlt_inertia(A.shape[0], _ptr(A), counts)
    return int(counts[0]), int(counts[1]), int(counts[2])


def inertia(pb: Problem, sigma: float):
    """(#{lam_n < sigma}, #{lam_n = sigma}, #{lam_n > sigma}) for the
    eigenvalues lam = 1/tau of the reduced pencil Ri v = lam Li v (Sec. 3.2),
    from the inertia of Ri - sigma Li, a congruence of C - sigma I.  Costs one
    dense factorisation (n0^3 / 3); safe to call from several threads."""
    counts = (ctypes.c_int64 * 3)()
    st = pb._struct()
    if _load().orc_inertia(ctypes.byref(st), float(sigma), counts):
        raise RuntimeError(_ERR[1])
    return int(counts[0]), int(counts[1]), int(counts[2])
