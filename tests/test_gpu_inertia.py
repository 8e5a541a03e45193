"""Eigenvalues of the 128x128 plate with a crack (N = 16,384, the crack
signature workload: log-uniform resistivity, a 10x3-cell crack of
resistivity 1e3, kappa ~ 1e8) against stored Sylvester inertia counts.

For each shift sigma of a fixed logarithmic grid the oracle counted the
negative pivots of a Bunch-Kaufman LDL^T of R - sigma L, i.e. the number of
generalized eigenvalues below sigma (Sec. 3.2, eq. generalized_eigenvalues_
discrete, congruent to C - sigma I); tests/golden/make_inertia_golden.py
wrote them calling only the oracle.  The library's eigenvalues must give the
same count at every shift, except for eigenvalues within the two methods'
error of sigma (none, in practice), which may fall on either side.  This is
the size the oracle's Jacobi cannot reach, so it is the eigenvalue check at
scale."""
import os

import numpy as np
import pytest

from paper_2407_11993_amd import inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "plate128_crack_inertia.txt")


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="inertia counts not written")
def test_eigenvalue_counts_match_inertia():
    from paper_2407_11993_amd import Solver
    rows = np.atleast_2d(np.loadtxt(GOLDEN))
    w = inputs.plate_128x128_crack(T=1)
    s = Solver(w)
    s.decompose(projected=True)
    lam = s.eigenvalues().cpu().numpy()
    s.close()
    n0 = lam.size
    assert n0 == w.n and np.all(np.diff(lam) >= 0) and lam[0] > 0
    tau_max = 1.0 / lam[0]
    checked = 0
    for sigma, below, at, above in rows:
        assert int(below + at + above) == n0
        # the library's backward error (a few hundred eps of tau_max in tau,
        # i.e. 1e-13 tau_max lam^2 in lam) plus the inertia factorisation's
        # (1e-8 relative)
        win = 1e-8 * sigma + 1e-13 * tau_max * sigma * sigma
        count = int(np.searchsorted(lam, sigma, side="left"))
        near = int(np.sum(np.abs(lam - sigma) <= win))
        assert count - near <= int(below) <= count + near, (sigma, count, near, below)
        checked += near == 0
    assert checked >= rows.shape[0] - 2
