"""Write the stored expected values for the 8x8x8 block (N = 512).

Run from the repository root:  python tests/golden/make_golden.py
Every value is computed by the CPU oracle (oracle/) on the seeded inputs of
paper_2407_11993_amd.inputs; nothing here comes from the GPU library.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_11993_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    oracle.build(force=False)
    w = inputs.block_8x8x8()
    L = oracle.assemble_L(w.xyz, w.h)
    pb = oracle.Problem(L, w.R.to_dense(), w.M, w.P)
    for theta in (0.5, 1.0):
        sig_d = oracle.theta_direct(pb, theta, w.dt, w.T, w.i_src)
        tag = "cn" if theta == 0.5 else "be"
        np.savetxt(os.path.join(HERE, f"block8_signal_direct_{tag}.txt"),
                   sig_d, fmt="%.17e",
                   header=f"8x8x8 block, Cholesky theta-method, theta={theta}, "
                          f"dt=1, T={w.T}; oracle.theta_direct")
    lam = oracle.modal_eigen(pb, want_V=False)
    np.savetxt(os.path.join(HERE, "block8_eigenvalues.txt"), lam, fmt="%.17e",
               header="8x8x8 block, eigenvalues of (Ri, Li) ascending; "
                      "oracle.modal_eigen (Jacobi)")


if __name__ == "__main__":
    main()
