"""The inductance matrix handed to the library as a dense matrix (Sec. 3.1:
L is the Galerkin matrix L_jk of eq. discrete_version_1a, an input of the
problem), through the C ABI, against the CPU oracle.

The matrices here are NOT the smooth kernel the generator produces: the
kernel matrix plus a random symmetric positive semi-definite low-rank term
and a random positive diagonal, so that a library that ignored the given
matrix (or read its upper triangle, or the wrong block after the electrode
reduction) fails.  Tolerances as in the other end-to-end tests: signals
1e-9 of max|s| against the oracle's direct theta-stepper, modal against
Cholesky 1e-8, eigenvalues 1e-10 relative (element-wise, no crack)."""
import numpy as np
import pytest

from paper_2407_11993_amd import inputs

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _perturbed_L(orc, w, seed):
    """Kernel matrix + (0.3 / k) B B^T + diag(0.05 + 0.1 u), B ~ N(0, 1)^{n x k}."""
    rng = np.random.default_rng(seed)
    n, k = w.n, 5
    B = rng.standard_normal((n, k))
    return orc.assemble_L(w.xyz, w.h) + (0.3 / k) * B @ B.T + np.diag(0.05 + 0.1 * rng.random(n))


CASES = {
    "plain": lambda: inputs.plate(10, 12, seed=2, T=300, wave="sin", thetas=(0.5, 1.0)),
    "two-electrodes": lambda: inputs.electrode_plate(10, 14, 4, T=300, tau_D=60.0,
                                                     coil_period=120.0),
    "two-electrodes-rho": lambda: inputs.electrode_plate(12, 9, 3, T=250, tau_D=40.0,
                                                         coil_period=70.0, seed=3),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, orc):
    import torch
    assert torch.cuda.is_available()
    from paper_2407_11993_amd import Solver
    w = CASES[request.param]()
    w.L = _perturbed_L(orc, w, seed=11)
    s = Solver(w)
    s.decompose()
    E = None if w.E is None else w.E.to_dense()
    return w, s, orc.Problem(w.L, w.R.to_dense(), w.M, w.P, E=E)


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_borrowed_L_signals_match_oracle(case, orc, theta):
    w, s, pb = case
    i_D = w.i_D if w.m else None
    s.reset()
    ref = orc.theta_direct(pb, theta, w.dt, w.T, w.i_src, i_D)
    sm = _np(s.step_modal(theta, w.dt, w.T, w.i_src, i_D))
    sc = _np(s.step_cholesky(theta, w.dt, w.T, w.i_src, i_D))
    assert _rel(sm, ref) < 1e-9
    assert _rel(sc, ref) < 1e-9
    assert _rel(sm, sc) < 1e-8


def test_borrowed_L_eigenvalues_match_oracle(case, orc):
    w, s, pb = case
    lam_ref = orc.modal_eigen(pb, want_V=False)
    lam = _np(s.eigenvalues())
    assert lam.shape == lam_ref.shape == (w.n - w.m,)
    assert np.max(np.abs(lam - lam_ref) / lam_ref) < 1e-10


def test_borrowed_L_projected_decomposition(case, orc):
    from paper_2407_11993_amd import Solver
    w, _, pb = case
    i_D = w.i_D if w.m else None
    s = Solver(w)
    s.decompose(projected=True)
    ref = orc.theta_direct(pb, 0.5, w.dt, w.T, w.i_src, i_D)
    assert _rel(_np(s.step_modal(0.5, w.dt, w.T, w.i_src, i_D)), ref) < 1e-9
    s.close()


def test_borrowed_L_is_not_written(case):
    w, s, _ = case
    # the solver's device copy is what the library borrows; it was read by
    # setup, the decomposition and the Cholesky factorisations above
    assert np.array_equal(_np(s._L), np.ascontiguousarray(w.L.T))


def test_borrowed_kernel_matrix_equals_generated(orc):
    """Handing over the generator's own matrix gives the generated run's
    signals (up to the rounding of the two assemblies)."""
    from paper_2407_11993_amd import Solver
    w = inputs.electrode_plate(9, 12, 3, T=200, tau_D=50.0, coil_period=90.0)
    a = Solver(w)
    a.decompose()
    sa = _np(a.step_modal(0.5, w.dt, w.T, w.i_src, w.i_D))
    w.L = orc.assemble_L(w.xyz, w.h)
    b = Solver(w)
    b.decompose()
    sb = _np(b.step_modal(0.5, w.dt, w.T, w.i_src, w.i_D))
    assert _rel(sb, sa) < 1e-12
    a.close()
    b.close()


def _expect_invalid(w, what):
    from paper_2407_11993_amd import Solver, _lib
    with pytest.raises(_lib.MMError) as ei:
        Solver(w)
    assert ei.value.code == 1, what
    assert "NaN or Inf" in str(ei.value), what


@pytest.mark.parametrize("where", ["L", "R", "M0", "P", "E", "xyz"])
def test_non_finite_inputs_are_rejected(orc, where):
    w = inputs.electrode_plate(8, 10, 3, T=10)
    if where == "L":
        w.L = orc.assemble_L(w.xyz, w.h)
        w.L[7, 3] = np.nan  # lower triangle
    elif where == "R":
        w.R.val = w.R.val.copy()
        w.R.val[5] = np.inf
    elif where == "M0":
        w.M = w.M.copy()
        w.M[4, 0] = np.nan
    elif where == "P":
        w.P = w.P.copy()
        w.P[0, 9] = -np.inf
    elif where == "E":
        w.E.val = w.E.val.copy()
        w.E.val[1] = np.nan
    else:
        w.xyz = w.xyz.copy()
        w.xyz[3, 1] = np.nan
    _expect_invalid(w, where)


def test_non_finite_dt_is_rejected():
    import torch
    from paper_2407_11993_amd import Solver, _lib
    w = inputs.plate(6, 6, seed=1, T=10)
    s = Solver(w)
    s.decompose()
    with pytest.raises(_lib.MMError) as ei:
        s.step_modal(0.5, float("inf"), 4, torch.zeros((5, 1), dtype=torch.float64,
                                                       device="cuda"))
    assert ei.value.code == 1
    s.close()


def test_indefinite_L_is_rejected(orc):
    """A borrowed L with a negative direction: the time constants of
    Li v = tau Ri v are then not all positive, and the decomposition reports
    MM_E_NOT_SPD rather than returning negative or infinite eigenvalues."""
    from paper_2407_11993_amd import Solver, _lib
    w = inputs.plate(8, 9, seed=4, T=10)
    L = orc.assemble_L(w.xyz, w.h)
    u = np.random.default_rng(5).standard_normal(w.n)
    u /= np.linalg.norm(u)
    w.L = L - (np.linalg.eigvalsh(L)[-1] + 1.0) * np.outer(u, u)
    s = Solver(w)
    for projected in (False, True):
        with pytest.raises(_lib.MMError) as ei:
            s.decompose(projected=projected)
        assert ei.value.code == 3, projected
        assert "L_i" in str(ei.value)
    s.close()
