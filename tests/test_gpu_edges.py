"""Edge cases of the boundary against the CPU oracle.

* Problems smaller than every tile, block and band of the path (N = 1, 2, 3
  and 7 cells: one cell, a band of width 0 or 1 for the band reduction, no
  bulge to chase, a single leaf for the divide and conquer, one partial
  block for the Cholesky method's solves), with the full and the projected
  decomposition: eigenvalues to 1e-10 relative, signals of both
  theta-methods to 1e-9 of max|s| (Sec. 3.2, Sec. 3.3).
* The same with two electrodes on plates of 2, 4 and 12 cells (N0 = 1, 3 and
  11 after the reduction: the electrode term's rank 2 then exceeds or nears
  N0, and its low-rank factor is singular).
* Zero-step calls: an empty signal, and the state left as it was, so that a
  run cut as 15 + 0 + 25 steps gives the 40-step run's signal (both
  methods)."""
import numpy as np
import pytest

from paper_2407_11993_amd import inputs

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("projected", [False, True])
@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 2), (1, 3), (7, 1)])
def test_tiny_problems_match_oracle(orc, nx, ny, projected):
    from paper_2407_11993_amd import Solver
    w = inputs.plate(nx, ny, seed=1, T=30, wave="sin", thetas=(0.5,))
    pb = orc.Problem(orc.assemble_L(w.xyz, w.h), w.R.to_dense(), w.M, w.P)
    lam_ref = orc.modal_eigen(pb, want_V=False)
    ref = orc.theta_direct(pb, 0.5, w.dt, w.T, w.i_src)
    s = Solver(w)
    s.decompose(projected=projected)
    lam = _np(s.eigenvalues())
    assert lam.shape == lam_ref.shape == (w.n,)
    assert np.max(np.abs(lam - lam_ref) / lam_ref) < 1e-10
    sm = _np(s.step_modal(0.5, w.dt, w.T, w.i_src))
    s.reset()
    sc = _np(s.step_cholesky(0.5, w.dt, w.T, w.i_src))
    assert sm.shape == sc.shape == ref.shape == (w.T, 1)
    assert _rel(sm, ref) < 1e-9
    assert _rel(sc, ref) < 1e-9
    s.close()


@pytest.mark.parametrize("projected", [False, True])
@pytest.mark.parametrize("nx,ny,ew", [(1, 2, 1), (2, 2, 1), (3, 4, 2)])
def test_tiny_electrode_problems_match_oracle(orc, nx, ny, ew, projected):
    from paper_2407_11993_amd import Solver
    w = inputs.electrode_plate(nx, ny, ew, T=30, tau_D=20.0, coil_period=40.0)
    pb = orc.Problem(orc.assemble_L(w.xyz, w.h), w.R.to_dense(), w.M, w.P,
                     E=w.E.to_dense())
    lam_ref = orc.modal_eigen(pb, want_V=False)
    ref = orc.theta_direct(pb, 0.5, w.dt, w.T, w.i_src, w.i_D)
    s = Solver(w)
    s.decompose(projected=projected)
    lam = _np(s.eigenvalues())
    assert lam.shape == lam_ref.shape == (w.n - w.m,)
    assert np.max(np.abs(lam - lam_ref) / lam_ref) < 1e-10
    sm = _np(s.step_modal(0.5, w.dt, w.T, w.i_src, w.i_D))
    s.reset()
    sc = _np(s.step_cholesky(0.5, w.dt, w.T, w.i_src, w.i_D))
    assert _rel(sm, ref) < 1e-9
    assert _rel(sc, ref) < 1e-9
    s.close()


@pytest.mark.parametrize("method", ["modal", "cholesky"])
def test_zero_steps_leave_the_state(method):
    from paper_2407_11993_amd import Solver
    w = inputs.plate(6, 7, seed=2, T=40, wave="sin", thetas=(0.5,))
    s = Solver(w)
    s.decompose()
    step = s.step_modal if method == "modal" else s.step_cholesky
    whole = _np(step(0.5, 1.0, 40, w.i_src))
    s.reset()
    first = _np(step(0.5, 1.0, 15, w.i_src[:16]))
    empty = step(0.5, 1.0, 0, w.i_src[15:16])
    assert tuple(empty.shape) == (0, w.n_probe)
    rest = _np(step(0.5, 1.0, 25, w.i_src[15:]))
    assert _rel(np.vstack([first, rest]), whole) < 1e-14
    s.close()


def test_unbanded_numbering_is_rejected():
    """R's factor is taken banded (block bidiagonal with blocks of the
    bandwidth, at most 8192): a 100 x 100 plate numbered in random order has
    a bandwidth near N and is refused with MM_E_INVALID by both
    decompositions, before any large allocation; the Cholesky method, which
    needs no band, still runs."""
    import scipy.sparse as sp
    from paper_2407_11993_amd import Solver, _lib
    w = inputs.plate(100, 100, seed=3, T=5, wave="sin", thetas=(0.5,))
    perm = np.random.default_rng(7).permutation(w.n)
    R = sp.csr_matrix((w.R.val, w.R.col, w.R.rowptr), shape=w.R.shape)[perm][:, perm].tocsr()
    R.sort_indices()
    w.R = inputs.CSR(R.shape, R.indptr.astype(np.int64), R.indices.astype(np.int32),
                     R.data.astype(np.float64))
    w.xyz = w.xyz[perm]
    w.M = w.M[perm]
    w.P = w.P[:, perm]
    s = Solver(w)
    for projected in (False, True):
        with pytest.raises(_lib.MMError) as ei:
            s.decompose(projected=projected)
        assert ei.value.code == 1 and "bandwidth" in str(ei.value)
    sc = _np(s.step_cholesky(0.5, w.dt, w.T, w.i_src))
    assert sc.shape == (w.T, 1) and np.all(np.isfinite(sc))
    s.close()
