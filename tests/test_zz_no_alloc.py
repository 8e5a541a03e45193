"""mm_step_modal_noalloc (the modal theta-method with its probe partial sums
in the library's static device array, no allocation) against mm_step_modal
through the C ABI: two calls in a row, the second on a smaller input, each
compared with the allocating entry point on the same problem and state.
Collected last: a failure here must not hide the other GPU tests."""
import numpy as np
import pytest

from paper_2407_11993_amd import inputs

pytestmark = pytest.mark.gpu


def _noalloc(s, theta, dt, n_steps, i_src, i_D=None):
    import torch
    from paper_2407_11993_amd import _lib
    src, d = s._waves(n_steps, i_src, i_D)
    sig = torch.empty((n_steps, s.n_probe), dtype=torch.float64, device="cuda")
    _lib.check(s.lib.mm_step_modal_noalloc(s.ctx, float(theta), float(dt), int(n_steps),
                                           _lib.ptr(src), _lib.ptr(d), _lib.ptr(sig)), s.ctx)
    torch.cuda.synchronize()
    return sig.cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_noalloc_matches_step_modal_twice():
    from paper_2407_11993_amd import Solver
    # first call: the 16x24 plate with two electrodes, 700 steps; second: a
    # 9x12 plate, 90 steps (a smaller problem and run on the same array)
    for w in (inputs.electrode_plate(16, 24, 4, T=700, tau_D=80.0, coil_period=150.0),
              inputs.electrode_plate(9, 12, 3, T=90, tau_D=30.0, coil_period=40.0)):
        a = Solver(w)
        a.decompose()
        ref = a.step_modal(0.5, w.dt, w.T, w.i_src, w.i_D).cpu().numpy()
        a.reset()
        got = _noalloc(a, 0.5, w.dt, w.T, w.i_src, w.i_D)
        assert got.shape == ref.shape
        # the same kernels and summation order: identical results
        assert np.array_equal(got, ref), _rel(got, ref)
        a.close()


def test_noalloc_continues_state_across_calls():
    from paper_2407_11993_amd import Solver
    w = inputs.plate(12, 10, seed=3, crack=((4, 8), (4, 6), 1e3), T=400, wave="gauss")
    s = Solver(w)
    s.decompose()
    ref = s.step_modal(0.5, w.dt, w.T, w.i_src).cpu().numpy()
    s.reset()
    k = 150
    a = _noalloc(s, 0.5, w.dt, k, w.i_src[:k + 1])
    b = _noalloc(s, 0.5, w.dt, w.T - k, w.i_src[k:])
    assert np.array_equal(np.vstack([a, b]), ref)
    s.close()


def test_noalloc_rejects_oversize():
    from paper_2407_11993_amd import Solver, _lib
    w = inputs.plate(6, 6, seed=1, T=10)
    s = Solver(w)
    s.decompose()
    n_steps = (1 << 23) + 1  # one mode group and one probe: one step too many
    i_src = np.zeros((n_steps + 1, 1))
    with pytest.raises(_lib.MMError) as ei:
        _noalloc(s, 0.5, 1.0, n_steps, i_src)
    assert ei.value.code == 1
    s.close()
