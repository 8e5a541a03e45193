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
