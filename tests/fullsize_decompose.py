"""The full decomposition at the paper-scale plate (256 x 384 cells with two
16-cell electrodes, N = 98,304, N0 = 98,303): mm_decompose forms the
eigenvector matrix V = G^{-T} Q (Sec. 3.2 eq. modal_decomposition_discrete),
and the reconstructed current I = K V y + A_D i_D (Sec. 3.1 eq.
current_electrodes) after 500 steps of theta = 1/2 is compared with the
Cholesky method's current after the same steps (within 1e-8 of the largest
entry), as are the probe signals; E I = i_D is checked on the modal current.

Several minutes of one library call, so it is run on its own rather than by
pytest (which would hold its output):  python tests/fullsize_decompose.py
The library prints each phase of the decomposition as it ends (MM_TRACE=1).
Exits non-zero if a check fails."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
os.environ.setdefault("MM_TRACE", "1")


def _rel(a, b):
    return float((a - b).abs().max() / b.abs().max())


def main():
    import torch
    from paper_2407_11993_amd import Solver, _lib, inputs
    torch.cuda.set_device(0)
    T = 500
    w = inputs.plate_256x384_electrodes(T=T)
    print(f"full decomposition: N = {w.n}, T = {T}", flush=True)
    i_src = torch.as_tensor(w.i_src, dtype=torch.float64, device="cuda")
    i_D = torch.as_tensor(w.i_D, dtype=torch.float64, device="cuda")
    s = Solver(w)
    t0 = time.perf_counter()
    s.decompose()
    t_dec = time.perf_counter() - t0
    lam = s.eigenvalues().cpu().numpy()
    ok = lam.shape == (w.n - w.m,) and bool(np.all(lam > 0)) and bool(np.all(np.diff(lam) >= 0))
    sm = s.step_modal(0.5, w.dt, T, i_src, i_D)
    Im = s.current(_lib.MM_MODAL)
    sc = s.step_cholesky(0.5, w.dt, T, i_src, i_D)
    Ic = s.current(_lib.MM_CHOLESKY)
    Ed = torch.zeros(w.n, dtype=torch.float64, device="cuda")
    Ed[torch.as_tensor(w.E.col.astype(np.int64), device="cuda")] = torch.as_tensor(
        w.E.val, device="cuda")
    eid = abs(float(Ed @ Im) - float(w.i_D[-1, 0]))
    res = {"decompose_s": round(t_dec, 2), "lambda_min": float(lam[0]),
           "lambda_max": float(lam[-1]), "signals_rel": _rel(sm, sc),
           "currents_rel": _rel(Im, Ic), "EI_minus_iD": eid}
    print(f"full decomposition result: {res}", flush=True)
    ok = ok and res["signals_rel"] < 1e-8 and res["currents_rel"] < 1e-8
    ok = ok and eid < 1e-10 * max(1.0, abs(float(w.i_D[-1, 0])))
    s.close()
    print("full decomposition: " + ("PASSED" if ok else "FAILED"), flush=True)
    sys.exit(0 if ok else 1)


if __name__ == "__main__":
    main()
