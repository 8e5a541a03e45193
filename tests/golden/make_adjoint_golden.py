"""Write the stored expected values of the adjoint on the 32x64 plate with
8 coils and T = 2000 steps (the quarter-size adjoint workload).

Run from the repository root:  python tests/golden/make_adjoint_golden.py
(about half an hour on one core).  The observations are the oracle's direct
theta-method signals of every coil on the reference field (the two defects);
the gradient is the oracle's physical-space adjoint at the background field.
Every value comes from oracle/; nothing here comes from the GPU library.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_11993_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
THETA = 0.5
N_SAMPLED = 512  # stored dJ/dR entries: the largest 64 and 448 at random (seed 55)


def main():
    oracle.build(force=False)
    cfg = inputs.adjoint_plate_32x64()
    T, M, dims, xyz = cfg["T"], cfg["M"], cfg["dims"], cfg["xyz"]
    C = M.shape[1]
    L = oracle.assemble_L(xyz, inputs.H_KERNEL)
    R_ref = inputs.resistance_csr(dims, cfg["rho_ref"]).to_dense()
    obs = np.empty((C, T))
    for c in range(C):
        pb = oracle.Problem(L, R_ref, M[:, c:c + 1], M[:, c][None, :])
        obs[c] = oracle.theta_direct(pb, THETA, 1.0, T, cfg["i_src"][:, None])[:, 0]
        print(f"observations: coil {c}", flush=True)
    np.savetxt(os.path.join(HERE, "adjoint_mini_obs.txt"), obs.reshape(-1), fmt="%.17e",
               header=f"{cfg['name']}: s_obs[c * T + k], T={T}, coils={C}, reference field; "
                      f"oracle.theta_direct, theta={THETA}, dt=1")
    Rcsr = inputs.resistance_csr(dims, cfg["rho_bg"])
    J, G, gi = oracle.adjoint_direct(L, Rcsr.to_dense(), M, M.T, THETA, 1.0, T, cfg["i_src"],
                                     obs)
    rows = np.repeat(np.arange(Rcsr.shape[0]), np.diff(Rcsr.rowptr))
    g = G[rows, Rcsr.col]
    top = np.argsort(-np.abs(g))[:64]
    rest = np.setdiff1d(np.arange(g.size), top)
    pick = np.sort(np.concatenate([top, np.random.default_rng(55).choice(
        rest, N_SAMPLED - top.size, replace=False)]))
    np.savetxt(os.path.join(HERE, "adjoint_mini_dJdR.txt"),
               np.column_stack([pick, g[pick]]), fmt=["%d", "%.17e"],
               header=f"{cfg['name']}: J={J:.17e} max_abs_dJdR={np.abs(g).max():.17e} "
                      f"nnz={g.size}; columns: index into R's stored entries (CSR order), "
                      f"dJ/dR there; oracle.adjoint_direct at the background field, "
                      f"theta={THETA}, dt=1")
    np.savetxt(os.path.join(HERE, "adjoint_mini_dJdi.txt"), gi, fmt="%.17e",
               header=f"{cfg['name']}: dJ/d i_src(t_k), k = 0..{T}; oracle.adjoint_direct")


if __name__ == "__main__":
    main()
