"""Time-parallel modal stepping (mm_step_modal_scan) through the C ABI.

Against the oracle: the 8x8x8 block's stored signals (theta = 1/2 and 1)
within 1e-9 of max|s|.  Against the sequential stepper (same decomposition):
within 1e-11 of max|s| (the chunk chaining reorders rounding), for theta and
exact integration, with electrodes, over 200,000 steps (about a thousand
chunks), for horizons shorter than one chunk, and continuing from the state."""
import os

import numpy as np
import pytest

from paper_2407_11993_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.fixture(scope="module")
def block8():
    import torch
    assert torch.cuda.is_available()
    from paper_2407_11993_amd import Solver
    w = inputs.block_8x8x8()
    s = Solver(w)
    s.decompose()
    return w, s


@pytest.mark.parametrize("theta,tag", [(0.5, "cn"), (1.0, "be")])
def test_scan_matches_oracle_block8(block8, theta, tag):
    w, s = block8
    ref = np.loadtxt(os.path.join(GOLDEN, f"block8_signal_direct_{tag}.txt"))[:, None]
    s.reset()
    got = _np(s.step_modal_scan(theta, w.dt, w.T, w.i_src))
    assert _rel(got, ref) < 1e-9
    s.reset()
    seq = _np(s.step_modal(theta, w.dt, w.T, w.i_src))
    assert _rel(got, seq) < 1e-11


@pytest.mark.parametrize("T", [1, 7, 31, 200000])
def test_scan_matches_sequential_block8(block8, T):
    w, s = block8
    t = np.arange(T + 1)
    i_src = np.sin(2 * np.pi * t / 997.0)[:, None] * np.exp(-t / 5e4)[:, None]
    for exact in (False, True):
        s.reset()
        got = _np(s.step_modal_scan(0.5, 1.0, T, i_src, exact=exact))
        s.reset()
        seq = _np(s.step_modal_exact(1.0, T, i_src) if exact else s.step_modal(0.5, 1.0, T, i_src))
        assert _rel(got, seq) < 1e-11, (T, exact)


def test_scan_continues_the_state(block8):
    w, s = block8
    T1, T2 = 1500, 500
    s.reset()
    seq = _np(s.step_modal(0.5, w.dt, T1 + T2, w.i_src[:T1 + T2 + 1]))
    s.reset()
    a = _np(s.step_modal_scan(0.5, w.dt, T1, w.i_src[:T1 + 1]))
    b = _np(s.step_modal(0.5, w.dt, T2, w.i_src[T1:T1 + T2 + 1]))
    assert _rel(np.vstack([a, b]), seq) < 1e-11


def test_scan_with_electrodes():
    from paper_2407_11993_amd import Solver
    w = inputs.electrode_plate(12, 9, 3, T=3000, tau_D=40.0, coil_period=70.0, seed=3)
    s = Solver(w)
    s.decompose()
    for exact in (False, True):
        s.reset()
        got = _np(s.step_modal_scan(0.5, w.dt, w.T, w.i_src, w.i_D, exact=exact))
        s.reset()
        seq = _np(s.step_modal_exact(w.dt, w.T, w.i_src, w.i_D) if exact
                  else s.step_modal(0.5, w.dt, w.T, w.i_src, w.i_D))
        assert _rel(got, seq) < 1e-11, exact
    s.close()


def test_scan_rejects_bad_arguments(block8):
    from paper_2407_11993_amd import _lib
    w, s = block8
    with pytest.raises(_lib.MMError) as e:
        s.step_modal_scan(1.5, w.dt, 10, w.i_src[:11])
    assert e.value.code == 1  # MM_E_INVALID: theta outside [0, 1]
