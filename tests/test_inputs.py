"""Host-side input generators (no GPU)."""
import numpy as np

from paper_2407_11993_amd import inputs


def test_resistance_model_reproduces_the_assembly():
    for dims, seed in (((7, 5, 1), 3), ((4, 3, 3), 8)):
        n = dims[0] * dims[1] * dims[2]
        rho = inputs.rho_loguniform(n, seed)
        rowptr, col, (ent, cel, coef), const = inputs.resistance_model(dims)
        R = inputs.resistance_csr(dims, rho)
        vals = const.copy()
        np.add.at(vals, ent, coef * rho[cel])
        assert np.array_equal(rowptr, R.rowptr) and np.array_equal(col, R.col)
        assert np.abs(vals - R.val).max() < 1e-14 * np.abs(R.val).max()


def test_adjoint_workloads_have_the_stated_shapes():
    """The full and quarter-size adjoint workloads: plate sizes, coil counts,
    the two defects only in the reference field, the shared pulse."""
    for cfg, n, C, T, (a, b) in ((inputs.adjoint_plate_128x256(T=50), 128 * 256, 64, 50, (1e3, 5.0)),
                                 (inputs.adjoint_plate_32x64(T=40), 32 * 64, 8, 40, (1e3, 5.0))):
        assert cfg["xyz"].shape == (n, 3)
        assert cfg["M"].shape == (n, C)
        assert cfg["i_src"].shape == (T + 1,)
        diff = cfg["rho_ref"] != cfg["rho_bg"]
        assert set(np.unique(cfg["rho_ref"][diff])) == {a, b}
        assert np.all((cfg["rho_bg"] >= 0.5) & (cfg["rho_bg"] <= 2.0))
