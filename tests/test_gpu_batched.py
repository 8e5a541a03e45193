"""Batched modal runs (many sources and waveforms of uneven length in one
launch, replayed as one HIP graph) against the CPU oracle run by run."""
import numpy as np
import pytest

from paper_2407_11993_amd import inputs

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def _coil_plate(nx=12, ny=10, n_coils=6, seed=11):
    base = inputs.plate(nx, ny, seed=seed, crack=((3, 7), (4, 6), 1e3), T=1)
    rng = np.random.default_rng(seed)
    coils = [(rng.uniform(0, nx - 1), rng.uniform(0, ny - 1), 2.0) for _ in range(n_coils)]
    M = np.stack([inputs.coil_coupling(base.xyz, p) for p in coils], axis=1)
    base.M = M
    base.P = M.T.copy()
    return base


def _waves(lens, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for T in lens:
        t = np.arange(T + 1, dtype=np.float64)
        if rng.random() < 0.5:
            out.append(np.sin(2 * np.pi * t / rng.uniform(20, 80)))
        else:
            out.append(np.exp(-((t - T / 4) / rng.uniform(5, 20)) ** 2))
    return out


@pytest.fixture(scope="module")
def setup(orc):
    import torch
    assert torch.cuda.is_available()
    from paper_2407_11993_amd import Solver
    w = _coil_plate()
    s = Solver(w)
    s.decompose()
    L = orc.assemble_L(w.xyz, w.h)
    R = w.R.to_dense()
    return w, s, L, R


LENS = [150, 0, 37, 200, 5, 120, 64]
SRC = [0, 1, 2, 3, 4, 5, 2]
PRB = [0, 1, 2, 3, 4, 5, 4]


def _ref(orc, w, L, R, theta, lens, src, prb, waves):
    out = []
    for T, c, p, wv in zip(lens, src, prb, waves):
        if T == 0:
            out.append(np.zeros(0))
            continue
        pb = orc.Problem(L, R, w.M[:, c:c + 1], w.P[p:p + 1])
        out.append(orc.theta_direct(pb, theta, 1.0, T, wv[:, None])[:, 0])
    return out


@pytest.mark.parametrize("theta", [0.5, 1.0])
def test_batch_matches_oracle_run_by_run(setup, orc, theta):
    w, s, L, R = setup
    waves = _waves(LENS)
    b = s.batch(theta, 1.0, LENS, SRC, PRB, np.concatenate(waves))
    b.run()
    ref = _ref(orc, w, L, R, theta, LENS, SRC, PRB, waves)
    for r, T in enumerate(LENS):
        got = _np(b.signal(r))
        assert got.shape == (T,)
        if T:
            assert _rel(got, ref[r]) < 1e-9, r


def test_every_tile_agrees(setup):
    w, s, L, R = setup
    waves = np.concatenate(_waves(LENS))
    outs = []
    for tile in range(6):
        b = s.batch(0.5, 1.0, LENS, SRC, PRB, waves, tile=tile)
        outs.append(_np(b.run()).copy())
        assert (b.threads, b.modes) == [(256, 1), (256, 2), (256, 4), (128, 4), (256, 8),
                                        (128, 8)][tile]
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() <= 1e-12 * np.abs(outs[0]).max()


def test_sequential_single_runs_are_bit_identical(setup):
    w, s, L, R = setup
    waves = _waves(LENS, seed=9)
    b = s.batch(0.5, 1.0, LENS, SRC, PRB, np.concatenate(waves), tile=2)
    full = _np(b.run()).copy()
    for r, T in enumerate(LENS):
        one = s.batch(0.5, 1.0, [T], [SRC[r]], [PRB[r]], waves[r], tile=2)
        got = _np(one.run())[:T]
        assert np.array_equal(got, full[b.offsets[r]:b.offsets[r + 1]])


def test_replay_and_refill(setup, orc):
    import torch
    w, s, L, R = setup
    lens = [80, 33]
    w1 = _waves(lens, seed=1)
    w2 = _waves(lens, seed=2)
    b = s.batch(0.5, 1.0, lens, [1, 4], [1, 4], np.concatenate(w1))
    a1 = _np(b.run()).copy()
    a2 = _np(b.run()).copy()
    assert np.array_equal(a1, a2)
    b.waves.copy_(torch.from_numpy(np.concatenate(w2)).to(b.waves.device))
    a3 = _np(b.run()).copy()
    ref = _ref(orc, w, L, R, 0.5, lens, [1, 4], [1, 4], w2)
    assert _rel(a3[:80], ref[0]) < 1e-9
    assert _rel(a3[80:], ref[1]) < 1e-9


def test_batch_errors(setup):
    from paper_2407_11993_amd import Solver, _lib
    w, s, L, R = setup
    with pytest.raises(_lib.MMError) as e:
        s.batch(0.5, 1.0, [10], [6], [0], np.zeros(11))  # source out of range
    assert e.value.code == 1
    with pytest.raises(_lib.MMError) as e:
        s.batch(0.5, 1.0, [10], [0], [0], np.zeros(11), tile=6)
    assert e.value.code == 1
    fresh = Solver(w)
    with pytest.raises(_lib.MMError) as e:
        fresh.batch(0.5, 1.0, [10], [0], [0], np.zeros(11))
    assert e.value.code == 5  # MM_E_STATE: not decomposed


def test_single_run_calls_reject_many_sources(setup):
    from paper_2407_11993_amd import Solver, _lib
    w = _coil_plate(n_coils=9)
    s = Solver(w)
    s.decompose()
    with pytest.raises(_lib.MMError) as e:
        s.step_modal(0.5, 1.0, 5, np.zeros((6, 9)))
    assert e.value.code == 1 and "mm_batch" in str(e.value)
