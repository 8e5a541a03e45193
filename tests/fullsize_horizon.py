"""Modal against Cholesky theta-method over the whole horizon of the
paper-scale plate (256 x 384 cells with two 16-cell electrodes, N = 98,304,
theta = 1/2, dt = 1, 10^5 steps; Sec. 3.3.1 eq. time_integration against
Sec. 3.3.2).

The Cholesky run streams 77 GB per step for 10^5 steps (about 22 minutes on
one MI355X), longer than one GPU session allows, so it is split in two parts
joined by the stepping state (mm_get_state / mm_set_state):

  part 1:  setup, projected decomposition, all 10^5 modal steps (signal
           saved), Cholesky factorisation and steps 0 .. H-1 (signal and the
           state after step H saved);
  part 2:  setup, Cholesky factorisation, the state of part 1 restored,
           steps H .. T-1 (signal saved);
  compare: (CPU) max_k |s_modal - s_chol| / max_k |s_chol| over all steps,
           also per block of 10^4 steps.

Each part prints a line per block of Cholesky steps and writes its arrays
(.npy) and timings (.json) to --out.  Not collected by pytest (a run of
minutes of GPU time per part); the parity bar is the same as the full-size
test's, 1e-8 of max|s|.

  python tests/fullsize_horizon.py part1 --out DIR
  python tests/fullsize_horizon.py part2 --out DIR --state DIR/chol_state.npy
  python tests/fullsize_horizon.py compare --out DIR [--out2 DIR2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

BLOCK = 5000  # Cholesky steps per call (one progress line each)


def _say(msg):
    print(f"horizon: {msg}", flush=True)


def _chol_steps(s, w, i_src, i_D, k0, k1, sig):
    import torch
    for a in range(k0, k1, BLOCK):
        b = min(a + BLOCK, k1)
        t0 = time.perf_counter()
        sig[a:b] = s.step_cholesky(0.5, w.dt, b - a, i_src[a:b + 1],
                                   i_D[a:b + 1]).cpu().numpy()[:, 0]
        torch.cuda.synchronize()
        _say(f"Cholesky steps {a}..{b - 1} in {time.perf_counter() - t0:.1f} s")


def part(which, out, state_path, half):
    import torch
    from paper_2407_11993_amd import Solver, _lib, inputs
    torch.cuda.set_device(0)
    w = inputs.plate_256x384_electrodes()
    T = w.T
    H = half or T // 2
    i_src = torch.as_tensor(w.i_src, dtype=torch.float64, device="cuda")
    i_D = torch.as_tensor(w.i_D, dtype=torch.float64, device="cuda")
    rec = {"workload": w.name, "N": w.n, "T": T, "theta": 0.5, "dt": w.dt, "half": H}
    s = Solver(w)
    if which == "part1":
        t0 = time.perf_counter()
        s.decompose(projected=True)
        lam = s.eigenvalues().cpu().numpy()
        sm = s.step_modal(0.5, w.dt, T, i_src, i_D).cpu().numpy()[:, 0]
        rec["modal_s"] = time.perf_counter() - t0
        rec["lambda_min"], rec["lambda_max"] = float(lam[0]), float(lam[-1])
        np.save(os.path.join(out, "modal_signal.npy"), sm)
        _say(f"modal: decomposition and {T} steps in {rec['modal_s']:.1f} s, "
             f"lambda in [{lam[0]:.6e}, {lam[-1]:.6e}]")
        s.reset()
        k0, k1 = 0, H
    else:
        k0, k1 = H, T
    t0 = time.perf_counter()
    s.step_cholesky(0.5, w.dt, 0, i_src[:1], i_D[:1])  # the factorisation
    torch.cuda.synchronize()
    rec["cholesky_factor_s"] = time.perf_counter() - t0
    _say(f"Cholesky factorisation {rec['cholesky_factor_s']:.1f} s")
    if which == "part2":
        s.set_state(np.load(state_path), _lib.MM_CHOLESKY)
    sig = np.zeros(T)
    t0 = time.perf_counter()
    _chol_steps(s, w, i_src, i_D, k0, k1, sig)
    rec["cholesky_steps"] = [k0, k1]
    rec["cholesky_steps_s"] = time.perf_counter() - t0
    np.save(os.path.join(out, f"chol_signal_{k0}_{k1}.npy"), sig[k0:k1])
    if which == "part1":
        np.save(os.path.join(out, "chol_state.npy"), s.get_state(_lib.MM_CHOLESKY).cpu().numpy())
    with open(os.path.join(out, f"{which}.json"), "w") as f:
        json.dump(rec, f, indent=1)
    _say(f"{which} done: {json.dumps(rec)}")
    s.close()


def compare(out, out2):
    sm = np.load(os.path.join(out, "modal_signal.npy"))
    r1 = json.load(open(os.path.join(out, "part1.json")))
    r2 = json.load(open(os.path.join(out2, "part2.json")))
    c1 = np.load(os.path.join(out, "chol_signal_%d_%d.npy" % tuple(r1["cholesky_steps"])))
    c2 = np.load(os.path.join(out2, "chol_signal_%d_%d.npy" % tuple(r2["cholesky_steps"])))
    sc = np.concatenate([c1, c2])
    assert sc.size == sm.size == r1["T"]
    scale = np.abs(sc).max()
    diff = np.abs(sm - sc)
    blocks = [float(diff[a:a + 10000].max() / scale) for a in range(0, sc.size, 10000)]
    res = {"max_rel": float(diff.max() / scale), "l2_rel": float(np.linalg.norm(sm - sc)
                                                                 / np.linalg.norm(sc)),
           "per_10k_steps": blocks, "argmax_step": int(diff.argmax()),
           "max_abs_signal": float(scale),
           "largest_time_constant_steps": 1.0 / r1["lambda_min"],
           "cholesky_seconds_measured": r1["cholesky_factor_s"] + r1["cholesky_steps_s"]
           + r2["cholesky_steps_s"],
           "cholesky_step_ms": 1e3 * (r1["cholesky_steps_s"] + r2["cholesky_steps_s"])
           / r1["T"],
           "modal_seconds": r1["modal_s"]}
    print(json.dumps(res, indent=1))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["part1", "part2", "compare"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--out2", default=None)
    ap.add_argument("--state", default=None)
    ap.add_argument("--half", type=int, default=0)
    a = ap.parse_args()
    os.makedirs(a.out, exist_ok=True)
    if a.what == "compare":
        res = compare(a.out, a.out2 or a.out)
        sys.exit(0 if res["max_rel"] < 1e-8 else 1)
    part(a.what, a.out, a.state, a.half)


if __name__ == "__main__":
    main()
