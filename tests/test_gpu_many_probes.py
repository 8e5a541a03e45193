"""Many probes per run (Sec. 4.4 observes the field at 301 sensing points):
above 8 probes the stepping calls write the amplitude (modal) or current
(Cholesky) increments of a chunk of steps and take the chunk's signals as
one matrix product P~^T dY.  Against the CPU oracle at small sizes (1e-9 of
max|s| per probe), against the 8-probe path and across chunk boundaries at
N = 16,384, and between the two methods (1e-8)."""
import numpy as np
import pytest

from paper_2407_11993_amd import inputs

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _rel_cols(a, b):
    """max over probes of max_k |a - b| / max_k |b| (per-probe scale)."""
    return float((np.abs(a - b).max(axis=0) / np.abs(b).max(axis=0)).max())


def _with_probes(w, n_side, lift=1.5):
    """The workload observed by n_side^2 point probes on a grid above the
    plate (couplings by the same kernel as the coil), the coil first."""
    nx, ny = w.dims[0], w.dims[1]
    xs = np.linspace(0.5, nx - 1.5, n_side)
    ys = np.linspace(0.5, ny - 1.5, n_side)
    rows = [w.P[0]]
    for yv in ys:
        for xv in xs:
            rows.append(inputs.coil_coupling(w.xyz, (xv, yv, lift)))
    w.P = np.vstack(rows)
    return w


CASES = {
    "plate-crack": lambda: inputs.plate(14, 11, seed=4, crack=((4, 9), (5, 7), 1e3), T=260,
                                        wave="sin", thetas=(0.5,)),
    "electrodes": lambda: inputs.electrode_plate(12, 9, 3, T=250, tau_D=40.0, coil_period=70.0,
                                                 seed=3),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_many_probes_match_oracle(orc, case):
    from paper_2407_11993_amd import Solver
    w = _with_probes(CASES[case](), 6)  # 37 probes
    i_D = w.i_D if w.m else None
    E = None if w.E is None else w.E.to_dense()
    pb = orc.Problem(orc.assemble_L(w.xyz, w.h), w.R.to_dense(), w.M, w.P, E=E)
    ref = orc.theta_direct(pb, 0.5, w.dt, w.T, w.i_src, i_D)
    ref_x = orc.exact_modal(pb, w.dt, w.T, w.i_src, i_D)
    s = Solver(w)
    s.decompose()
    sm = _np(s.step_modal(0.5, w.dt, w.T, w.i_src, i_D))
    s.reset()
    sx = _np(s.step_modal_exact(w.dt, w.T, w.i_src, i_D))
    s.reset()
    sc = _np(s.step_cholesky(0.5, w.dt, w.T, w.i_src, i_D))
    assert sm.shape == ref.shape == (w.T, 37)
    assert _rel_cols(sm, ref) < 1e-9
    assert _rel_cols(sx, ref_x) < 1e-9
    assert _rel_cols(sc, ref) < 1e-9
    # selective stepping with every mode of non-zero score kept
    s.reset()
    s.select_modes(0.0)
    ss = _np(s.step_modal_selective(0.5, w.dt, w.T, w.i_src, i_D))
    assert _rel_cols(ss, ref) < 1e-9
    s.close()


def test_many_probes_across_chunks_at_16384():
    """N = 16,384, 20,000 steps: two chunks of increments per call.  Twelve
    probes in one call against the same probes in two calls of six (the
    register path), and the Cholesky method's twelve against the modal ones."""
    import torch
    from paper_2407_11993_amd import Solver
    T = 20000
    w = _with_probes(inputs.plate_128x128_crack(T=T), 3, lift=2.0)  # 10 probes
    w.P = np.vstack([w.P, inputs.coil_coupling(w.xyz, (30.5, 90.5, 1.0))[None],
                     inputs.coil_coupling(w.xyz, (100.5, 20.5, 3.0))[None]])
    i_src = torch.as_tensor(w.i_src, dtype=torch.float64, device="cuda")
    s = Solver(w)
    s.decompose(projected=True)
    many = _np(s.step_modal(0.5, w.dt, T, i_src))
    s.close()
    parts = []
    for sl in (slice(0, 6), slice(6, 12)):
        w6 = inputs.plate_128x128_crack(T=1)
        w6.P = w.P[sl]
        s6 = Solver(w6)
        s6.decompose(projected=True)
        parts.append(_np(s6.step_modal(0.5, w.dt, T, i_src)))
        s6.close()
    few = np.hstack(parts)
    assert many.shape == few.shape == (T, 12)
    assert _rel_cols(many, few) < 1e-11
    s = Solver(w)
    sc = _np(s.step_cholesky(0.5, w.dt, T, i_src))
    assert _rel_cols(sc, few) < 1e-8
    s.close()


@pytest.mark.parametrize("case", sorted(CASES) + ["tiny"])
def test_projected_many_columns_match_oracle(orc, case):
    """More forcing and probe columns than the bulge chase carries along (32):
    the projected decomposition keeps the chase's reflectors and applies Q2^T
    to the columns afterwards (a wavefront of launches over the blocks of 64
    sweeps; "tiny" has fewer than 66 unknowns, a band narrower than 64 and one
    block per launch).  Against the oracle and the full decomposition."""
    from paper_2407_11993_amd import Solver
    if case == "tiny":
        w = inputs.plate(7, 8, seed=6, T=200, wave="sin", thetas=(0.5,))
    else:
        w = CASES[case]()
    w = _with_probes(w, 6)  # 37 probes
    assert w.M.shape[1] + 2 * w.m + w.n_probe > 32
    i_D = w.i_D if w.m else None
    E = None if w.E is None else w.E.to_dense()
    pb = orc.Problem(orc.assemble_L(w.xyz, w.h), w.R.to_dense(), w.M, w.P, E=E)
    ref = orc.theta_direct(pb, 0.5, w.dt, w.T, w.i_src, i_D)
    s = Solver(w)
    s.decompose(projected=True)
    sp = _np(s.step_modal(0.5, w.dt, w.T, w.i_src, i_D))
    s.close()
    f = Solver(w)
    f.decompose()
    sf = _np(f.step_modal(0.5, w.dt, w.T, w.i_src, i_D))
    f.close()
    assert sp.shape == ref.shape == (w.T, 37)
    assert _rel_cols(sp, ref) < 1e-9
    assert _rel_cols(sp, sf) < 1e-11


def test_301_probes_projected_at_16384():
    """N = 16,384 (the crack plate) observed at 301 points (the number of
    Sec. 4.4) on a line 2 cells above the plate, over the crack: the
    projected decomposition with 302 columns against the full one, and the
    Cholesky method against both (1e-8)."""
    from paper_2407_11993_amd import Solver
    T = 3000
    w = inputs.plate_128x128_crack(T=T)
    xs = np.linspace(0.5, w.dims[0] - 1.5, 301)
    w.P = np.vstack([inputs.coil_coupling(w.xyz, (x, w.dims[1] / 2.0 - 0.5, 2.0))
                     for x in xs])
    s = Solver(w)
    s.decompose(projected=True)
    sp = _np(s.step_modal(0.5, w.dt, T, w.i_src))
    s.close()
    f = Solver(w)
    f.decompose()
    sf = _np(f.step_modal(0.5, w.dt, T, w.i_src))
    f.reset()
    sc = _np(f.step_cholesky(0.5, w.dt, T, w.i_src))
    f.close()
    assert sp.shape == sf.shape == (T, 301)
    assert _rel_cols(sp, sf) < 1e-10
    assert _rel_cols(sc, sf) < 1e-8
