"""Benchmark: end-to-end seconds of the modal vs the Cholesky theta-method.

One step = the whole hot path on one synthetic problem, every phase on the
GPU: problem setup and L assembly, the modal decomposition, modal stepping,
and the Cholesky method (one factorisation per theta and two triangular
solves per time step).  Default workload: the 256x384 plate with two
16-cell electrodes (N = 98,304, N0 = 98,303 after the electrode reduction),
T = 100,000 steps, theta = 1/2; the Cholesky method's steps are measured
over a block of steps and extrapolated to T.  Other workloads: the 128x128
plate with a crack (N = 16,384, T = 10,000, theta in {0.5, 1.0}), the
8x8x8 block, the batched coils and the adjoint gradient.

Prints one JSON line.  `value` is the modal method's end-to-end seconds for
the workload (lower is better); the Cholesky method's seconds, the speed-up,
the decomposition's FP64 TFLOP/s and the roofline of the dominant kernel are
reported beside it.
"""
from __future__ import annotations

import argparse
import copy
import math
import json
import os
import sys
import time

T_START = time.perf_counter()  # the wall-clock budget counts from here
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
SELECT_TOL = 1e-10  # relative coupling score of the selective run
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 matrix (= vector), published


def _workload(name: str, T: int | None):
    from paper_2407_11993_amd import inputs
    if name == "plate-128x128-crack":
        return inputs.plate_128x128_crack(T=T or 10000)
    if name == "block-8x8x8":
        return inputs.block_8x8x8(T=T or 2000)
    if name == "batched-coils-128x128":
        return inputs.batched_coils()
    raise SystemExit(f"unknown workload {name}")


# flops of one modal mode-step: w u (1), -a y + . (2), c (.) (1), y += dy (1),
# probe accumulation (2)
FLOPS_PER_MODE_STEP = 7.0


def run_electrodes(args):
    """The paper-scale plate with injected currents (256 x 384 cells,
    N = 98,304, two electrodes, 1e5 steps, theta = 1/2) or a smaller plate of
    the same kind: the modal method end to end (setup, projected
    decomposition, all steps), and the Cholesky method's factorisation plus a
    measured block of steps whose per-step time is extrapolated to all steps
    (reported as such).  The signals of the two methods are compared over the
    measured steps.

    One end-to-end run of the paper-scale plate takes about a minute, so
    --warmup and --steps are upper bounds: the warm-up runs use a 48 x 72
    plate of the same kind (compiling and loading every kernel the timed run
    uses), and timed runs are added while the wall-clock budget (--budget-s,
    counted from the start of the process, with room kept for the CPU
    baseline) leaves room for one more.  `steps` reports the runs timed."""
    import numpy as np
    import torch
    from paper_2407_11993_amd import Solver, inputs

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    w = _electrode_workload(args.workload, args.T)
    T = w.T
    print(f"bench: inputs of {w.name} ready (N={w.n}, T={T})", file=sys.stderr, flush=True)
    theta, dt = w.thetas[0], w.dt
    K = min(args.chol_steps, T)
    stream = torch.cuda.current_stream()
    tones_hz = [1, 50, 100, 150, 250, 300, 400, 600, 700, 800, 900, 1000, 1500, 2000, 2500,
                3000, 3500, 4000, 4500, 5000, 5500, 6000, 6500, 7000, 7500, 8000, 8500, 9000,
                9500, 10000]
    omegas = [2 * math.pi * f / 30000.0 for f in tones_hz]

    last_signal = [None]  # the coil signal of the latest run

    def one_step(w, K, tag):
        T = w.T
        # waveforms resident in HBM before the timed region of the run
        i_src = torch.as_tensor(w.i_src, dtype=torch.float64, device="cuda")
        i_D = torch.as_tensor(w.i_D, dtype=torch.float64, device="cuda")
        amps_src = [[1.0] * w.M.shape[1]] * len(omegas)
        amps_D = [[1.0] * w.m] * len(omegas) if w.m else None
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(16)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        s = Solver(w)
        ev[1].record(stream)
        s.decompose(projected=True)
        ev[2].record(stream)
        torch.cuda.synchronize()
        print(f"bench: {tag} N={w.n}, projected decomposition "
              f"{ev[1].elapsed_time(ev[2]) / 1e3:.2f} s", file=sys.stderr, flush=True)
        sm = s.step_modal(theta, dt, T, i_src, i_D)
        ev[3].record(stream)
        # the same run with exact per-mode integration (waveforms linear
        # between samples): no time-step error, same cost
        s.reset()
        ev[7].record(stream)
        sx = s.step_modal_exact(dt, T, i_src, i_D)
        ev[8].record(stream)
        torch.cuda.synchronize()
        exact_diff = float((sm - sx).abs().max() / sx.abs().max())
        # steady-state phasors of the probe at the paper's 30 tones (Sec. 4.3,
        # sampled at 30 kS/s as in Sec. 4.6, so w = 2 pi f / 30000 per step),
        # unit amplitudes
        ev[9].record(stream)
        s.phasors(omegas, amps_src, amps_D)
        ev[10].record(stream)
        torch.cuda.synchronize()
        # selective solution (Sec. 3.2): only the modes with a coupling score
        # above 1e-10 of the largest are stepped, the same run otherwise
        s.reset()
        ev[11].record(stream)
        kept = s.select_modes(SELECT_TOL)
        ev[12].record(stream)
        ss = s.step_modal_selective(theta, dt, T, i_src, i_D)
        ev[13].record(stream)
        # the kept modes again, parallel in time
        s.reset()
        ev[14].record(stream)
        sp = s.step_modal_selective(theta, dt, T, i_src, i_D, scan=True)
        ev[15].record(stream)
        torch.cuda.synchronize()
        sel = (int(kept.numel()), float((ss - sm).abs().max() / sm.abs().max()),
               float((sp - ss).abs().max() / ss.abs().max()))
        s.reset()
        ev[4].record(stream)
        s.step_cholesky(theta, dt, 0, i_src[:1], i_D[:1])  # the factorisation
        ev[5].record(stream)
        sc = s.step_cholesky(theta, dt, K, i_src[:K + 1], i_D[:K + 1])
        ev[6].record(stream)
        torch.cuda.synchronize()
        t = [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(6)]
        print(f"bench: {tag} Cholesky factorisation {t[4]:.2f} s, {K} steps {t[5]:.2f} s",
              file=sys.stderr, flush=True)
        agree = float((sm[:K] - sc).abs().max() / sc.abs().max())
        last_signal[0] = sm[:, 0].clone()
        s.close()
        return {"setup": t[0], "decompose": t[1], "modal_steps": t[2], "cholesky_factor": t[4],
                "cholesky_steps_measured": t[5],
                "modal_exact_steps": ev[7].elapsed_time(ev[8]) / 1e3,
                "modal_phasors_30_tones": ev[9].elapsed_time(ev[10]) / 1e3,
                "select_modes": ev[11].elapsed_time(ev[12]) / 1e3,
                "modal_selective_steps": ev[12].elapsed_time(ev[13]) / 1e3,
                "modal_selective_steps_scan": ev[14].elapsed_time(ev[15]) / 1e3}, \
            (agree, exact_diff, sel)

    def many_probe_run(w):
        """Sec. 4.4 observes the field at 301 points: the same run with the
        coil and 300 point probes on a line 2 cells above the plate's long
        axis, one projected decomposition of all forcing and probe columns
        (more than the bulge chase carries along: its reflectors are kept
        and Q2^T is applied afterwards) and the modal steps."""
        nx, ny = w.dims[0], w.dims[1]
        ys = [0.5 + (ny - 2.0) * i / 299.0 for i in range(300)]
        wp = copy.copy(w)
        wp.P = np.vstack([w.P[:1]] + [inputs.coil_coupling(w.xyz, (nx / 2.0 - 0.5, y, 2.0))[None]
                                      for y in ys])
        i_src = torch.as_tensor(w.i_src, dtype=torch.float64, device="cuda")
        i_D = torch.as_tensor(w.i_D, dtype=torch.float64, device="cuda")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        s = Solver(wp)
        ev[1].record(stream)
        s.decompose(projected=True)
        ev[2].record(stream)
        sp = s.step_modal(theta, dt, wp.T, i_src, i_D)
        ev[3].record(stream)
        torch.cuda.synchronize()
        t = [ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(3)]
        ref = last_signal[0]
        diff = float((sp[:, 0] - ref).abs().max() / ref.abs().max())
        s.close()
        print(f"bench: 301 probes, projected decomposition {t[1]:.2f} s, "
              f"{wp.T} steps {t[2]:.3f} s", file=sys.stderr, flush=True)
        return {"probes": wp.n_probe, "columns": int(wp.M.shape[1] + 2 * wp.m + wp.n_probe),
                "setup_s": round(t[0], 3), "decompose_s": round(t[1], 3),
                "modal_steps_s": round(t[2], 4),
                "end_to_end_s": round(sum(t), 3),
                "coil_signal_difference_vs_one_probe_run": diff}

    if args.warmup:
        ww = _electrode_workload("plate-48x72-electrodes", min(T, 2000))
        for i in range(args.warmup):
            one_step(ww, min(K, ww.T), f"warm-up {i + 1}/{args.warmup}")
    runs, walls = [], []
    t0 = time.perf_counter()
    reserve = 0.0 if args.no_cpu_baseline else args.cpu_reserve_s

    def many_estimate():  # seconds the 301-probe leg needs, from the last run
        if args.no_many_probes:
            return 0.0
        r = runs[-1][0]
        return 1.2 * (r["setup"] + r["decompose"]) + 15.0

    while len(runs) < args.steps:
        if walls:
            left = args.budget_s - (time.perf_counter() - T_START) - reserve
            if left < 1.1 * max(walls) + many_estimate():
                break
        ts = time.perf_counter()
        runs.append(one_step(w, K, f"timed run {len(runs) + 1}"))
        walls.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    many = None
    if not args.no_many_probes:
        left = args.budget_s - (time.perf_counter() - T_START) - reserve
        if left >= many_estimate():
            many = many_probe_run(w)
        else:
            many = {"skipped": f"{left:.0f} s of the budget left, "
                               f"{many_estimate():.0f} s needed"}
    n_timed = len(runs)
    avg = {k: sum(r[0][k] for r in runs) / len(runs) for k in runs[0][0]}
    agree = max(r[1][0] for r in runs)
    exact_diff = max(r[1][1] for r in runs)
    n_kept = runs[-1][1][2][0]
    sel_diff = max(r[1][2][1] for r in runs)
    sel_scan_diff = max(r[1][2][2] for r in runs)
    n0 = w.n - w.m
    per_step = avg["cholesky_steps_measured"] / K
    modal_s = avg["setup"] + avg["decompose"] + avg["modal_steps"]
    chol_s = avg["setup"] + avg["cholesky_factor"] + per_step * T
    trsv_bytes = 2 * 8.0 * n0 * (n0 + 1) / 2
    achieved = trsv_bytes / per_step / 1e9
    dec_flops = _decomp_flops(n0, _band_block(w.R), full=False)
    return {
        "metric": "end-to-end s, modal theta-method (Cholesky theta-method beside it)",
        "value": round(modal_s, 3), "unit": "s", "n_gpus": 1, "steps": n_timed,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall / n_timed, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "N": w.n, "N0": n0, "T": T, "theta": theta, "dt": dt,
                   "electrodes": w.m + 1, "probes": w.n_probe,
                   "decomposition": "eigenvalues and projected weights V^T [F, P] "
                                    "(the eigenvector matrix is not formed)",
                   "step": "one end-to-end run of both methods (warm-up runs on a 48x72 "
                           "plate with two electrodes, T = 2000)",
                   "steps_requested": args.steps},
        "cholesky_s_extrapolated": round(chol_s, 1),
        "cholesky_steps_measured": K,
        "speedup_modal_vs_cholesky": round(chol_s / modal_s, 2),
        "signal_agreement_modal_vs_cholesky": agree,
        # exact per-mode integration vs theta = 1/2 on the same samples: the
        # theta-method's time-step error on this run
        "signal_difference_exact_vs_theta": exact_diff,
        # the paper's 30-tone comparison: modal phasors vs the frequency-domain
        # method's one complex factorisation of R + j w L per tone, estimated as
        # 4x the measured real Cholesky factorisation (complex arithmetic)
        "phasors_30_tones_s": round(avg["modal_phasors_30_tones"], 6),
        "frequency_domain_direct_estimate_s": round(30 * 4 * avg["cholesky_factor"], 1),
        # the selective solution on the same run: modes kept at a relative
        # coupling score of SELECT_TOL, their steps, and the signal change
        "selective": {"tol": SELECT_TOL, "modes_kept": n_kept, "modes": n0,
                      "select_s": round(avg["select_modes"], 6),
                      "steps_s": round(avg["modal_selective_steps"], 6),
                      "steps_scan_s": round(avg["modal_selective_steps_scan"], 6),
                      "signal_difference_vs_all_modes": sel_diff,
                      "signal_difference_scan_vs_sequential": sel_scan_diff},
        # the same plate observed at 301 points (Sec. 4.4), run once after the
        # timed runs: its own projected decomposition and all modal steps
        "many_probes": many,
        "phases_s": {k: round(v, 3) for k, v in avg.items()},
        "decomposition_tflops": round(dec_flops / avg["decompose"] / 1e12, 3),
        # the same time against the 7/3 N0^3 flops of the standard form taken from
        # L's side (dense Cholesky, inverse and product, then the band reduction),
        # which this decomposition replaces by R's banded factor: a rate for
        # comparison with that design, not the flops performed
        "decomposition_tflops_lside_count": round(7.0 / 3.0 * float(n0) ** 3
                                                  / avg["decompose"] / 1e12, 3),
        "roofline": {"bound": "hbm", "kernel": "triangular solve pair (fwd+bwd per step)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        # the modal value's dominant phase: GEMM-bound (the banded standard
        # form and the band reduction), timed on the stream it runs on
        "roofline_decomposition": {
            "bound": "mfma", "kernel": "projected decomposition (all its kernels)",
            "achieved": round(dec_flops / avg["decompose"] / 1e12, 2),
            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(dec_flops / avg["decompose"] / 1e12 / FP64_PEAK_TFLOPS, 4),
            "traffic": None},
    }


def _electrode_workload(name, T):
    from paper_2407_11993_amd import inputs
    nx, ny = (int(v) for v in name.split("-")[1].split("x"))
    T = T or 100000
    if (nx, ny) == (256, 384):
        return inputs.plate_256x384_electrodes(T=T)
    return inputs.electrode_plate(nx, ny, 16, T=T, name=f"plate-{nx}x{ny}-electrodes")


def run_scan(args):
    """Few modes, many steps: the 8x8x8 block (N = 512) stepped for 10^6 steps
    (theta = 1/2) by the sequential modal kernel (one thread per mode over the
    whole horizon: two workgroups) and by the time-parallel scan.  The
    decomposition is shared and not timed."""
    import numpy as np
    import torch
    from paper_2407_11993_amd import Solver, inputs

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    T = args.T or 1_000_000
    w = inputs.block_8x8x8(T=10)
    t = np.arange(T + 1)
    i_src = torch.as_tensor(np.sin(2 * np.pi * t / 200.0)[:, None], dtype=torch.float64,
                            device="cuda")
    s = Solver(w)
    s.decompose()
    stream = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.reset()
        torch.cuda.synchronize()
        e0.record(stream)
        out = fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / 1e3

    for _ in range(args.warmup):
        timed(lambda: s.step_modal_scan(0.5, 1.0, T, i_src))
    t0 = time.perf_counter()
    runs = []
    for _ in range(args.steps):
        seq, t_seq = timed(lambda: s.step_modal(0.5, 1.0, T, i_src))
        scn, t_scan = timed(lambda: s.step_modal_scan(0.5, 1.0, T, i_src))
        agree = float((seq - scn).abs().max() / seq.abs().max())
        runs.append((t_seq, t_scan, agree))
        print(f"bench: sequential {t_seq:.3f} s, scan {t_scan:.4f} s", file=sys.stderr,
              flush=True)
    wall = time.perf_counter() - t0
    t_seq = sum(r[0] for r in runs) / len(runs)
    t_scan = sum(r[1] for r in runs) / len(runs)
    mode_steps = 2.0 * w.n * T  # the scan's work: every chunk is run twice
    achieved = FLOPS_PER_MODE_STEP * mode_steps / t_scan / 1e12
    s.close()
    return {
        "metric": "modal stepping s, few modes and many steps (time-parallel scan)",
        "value": round(t_scan, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall / args.steps, 1),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "scan-block-8x8x8", "N": w.n, "T": T, "theta": 0.5},
        "sequential_s": round(t_seq, 4), "speedup_scan_vs_sequential": round(t_seq / t_scan, 1),
        "signal_agreement_scan_vs_sequential": max(r[2] for r in runs),
        "roofline": {"bound": "alu", "kernel": "time-parallel modal stepping (both passes)",
                     "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": None},
    }


def run_batched(args):
    """Batched coils on the 128x128 crack plate: 256 coil positions with
    their own waveform lengths, stepped in one graph-captured batched launch,
    against 256 sequential solves of one run each (same tile).  The
    decomposition is shared and not timed."""
    import numpy as np
    import torch
    from paper_2407_11993_amd import Solver

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    w = _workload(args.workload, args.T)
    s = Solver(w)
    s.decompose()
    lens = np.asarray(w.lengths, dtype=np.int64)
    n_runs = lens.size
    runs = np.arange(n_runs)
    waves = np.concatenate([w.i_src[:lens[r] + 1, r] for r in runs])
    print(f"bench: decomposed N={w.n}; autotuning {n_runs} runs", file=sys.stderr, flush=True)
    b = s.batch(0.5, w.dt, lens, runs, runs, waves)
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3 / reps

    for _ in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    t_batch = timed(b.run, args.steps)
    print(f"bench: batched {t_batch:.4f} s per launch", file=sys.stderr, flush=True)
    tiles = [(256, 1), (256, 2), (256, 4), (128, 4), (256, 8), (128, 8)]
    tile = tiles.index((b.threads, b.modes))
    singles = [s.batch(0.5, w.dt, [lens[r]], [r], [r], w.i_src[:lens[r] + 1, r], tile=tile)
               for r in runs]

    def sequential():
        for one in singles:
            one.run()

    sequential()
    t_seq = timed(sequential, 1)
    agree = max(float((singles[r].run()[:lens[r]] - b.signal(r)).abs().max()) for r in runs)
    mode_steps = float(s.n0) * float(lens.sum())
    tflops = FLOPS_PER_MODE_STEP * mode_steps / t_batch / 1e12
    res = {
        "metric": "batched modal stepping, s per launch (all runs)",
        "value": round(t_batch, 5), "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * t_batch, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "N": w.n, "runs": int(n_runs),
                   "total_steps": int(lens.sum()), "lengths": [int(lens.min()), int(lens.max())],
                   "tile": [b.threads, b.modes]},
        "sequential_s": round(t_seq, 5), "speedup_batched_vs_sequential": round(t_seq / t_batch, 2),
        "mode_steps_per_s": mode_steps / t_batch,
        "max_abs_diff_batched_vs_sequential": agree,
        "roofline": {"bound": "alu", "kernel": "batched modal stepping",
                     "achieved": round(tflops, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP64_PEAK_TFLOPS, 4), "traffic": None},
    }
    for one in singles:
        one.close()
    b.close()
    return res


def run_adjoint(args):
    """Adjoint on the 128x256 plate: gradient of the 64-coil probe-signal
    misfit with respect to every cell's resistivity and the shared waveform
    (modal adjoint with checkpoints every 500 steps), evaluated at the
    background field, with observations from the reference field (two
    defects).  Timed: problem
    setup, decomposition and the adjoint (forward, backward, S GEMMs,
    V S V^T).  A few cells are checked by central differences."""
    import numpy as np
    import torch
    from paper_2407_11993_amd import Solver, inputs
    from paper_2407_11993_amd.autograd import MisfitProblem

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    cfg = inputs.adjoint_plate_128x256(T=args.T or 10000)
    T, M, dims = cfg["T"], cfg["M"], cfg["dims"]
    C = M.shape[1]
    dev = "cuda"
    stream = torch.cuda.current_stream()
    wave = torch.as_tensor(cfg["i_src"], device=dev)
    # observations: the reference field, all coils in one batched launch
    pb0 = MisfitProblem(dims, M, torch.zeros((C, T), device=dev, dtype=torch.float64))
    rho_ref = torch.as_tensor(cfg["rho_ref"], device=dev)
    R_ref = (torch.sparse.mm(pb0.A, rho_ref.reshape(-1, 1)).reshape(-1) + pb0.c).contiguous()
    s = Solver(pb0.workload(R_ref))
    s.decompose()
    runs = np.arange(C)
    b = s.batch(0.5, 1.0, [T] * C, runs, runs, wave.repeat(C))
    obs = b.run().reshape(C, T).clone()
    b.close()
    s.close()
    print(f"bench: observations from the reference field (N={cfg['xyz'].shape[0]})",
          file=sys.stderr, flush=True)
    pb = MisfitProblem(dims, M, obs, theta=0.5, ckpt_every=500)
    rho = torch.as_tensor(cfg["rho_bg"], device=dev)

    def solver_at(r):
        R_val = (torch.sparse.mm(pb.A, r.reshape(-1, 1)).reshape(-1) + pb.c).contiguous()
        return Solver(pb.workload(R_val))

    def misfit(r):  # forward only: one batched launch of all coils
        sv = solver_at(r)
        sv.decompose()
        bb = sv.batch(0.5, 1.0, [T] * C, runs, runs, wave.repeat(C))
        J = float(((bb.run().reshape(C, T) - obs) ** 2).sum())
        bb.close()
        sv.close()
        return J

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    sv = solver_at(rho)
    ev[1].record(stream)
    sv.decompose()
    ev[2].record(stream)
    J, gR, g_i = sv.adjoint(0.5, 1.0, T, runs, runs, wave, obs, 500)
    ev[3].record(stream)
    torch.cuda.synchronize()
    t_setup, t_dec, t_adj = (ev[i].elapsed_time(ev[i + 1]) / 1e3 for i in range(3))
    sv.close()
    g_rho = torch.sparse.mm(pb.At, gR.reshape(-1, 1)).reshape(-1)
    J = float(J)
    print(f"bench: decomposition {t_dec:.2f} s, adjoint {t_adj:.2f} s, J = {J:.6e}",
          file=sys.stderr, flush=True)
    J_fwd = misfit(rho)
    gmax = float(g_rho.abs().max())
    # cells with the largest |dJ/drho| (where the check is informative) and
    # random ones; relative step 1e-4 keeps the difference far above the
    # misfit's rounding while the central difference error stays O(h^2)
    rng = np.random.default_rng(55)
    top = torch.topk(g_rho.abs(), (args.fd_cells + 1) // 2).indices.cpu().numpy()
    rest = rng.choice(rho.numel(), args.fd_cells - top.size, replace=False)
    fd = []
    for cell in np.concatenate([top, rest]):
        h = 1e-4 * float(rho[cell])
        e = torch.zeros_like(rho)
        e[cell] = h
        d = (misfit(rho + e) - misfit(rho - e)) / (2 * h)
        fd.append({"cell": int(cell), "fd": d, "adjoint": float(g_rho[cell]),
                   "err_rel_max_g": abs(d - float(g_rho[cell])) / gmax,
                   "err_rel_cell": abs(d - float(g_rho[cell])) / max(abs(d), 1e-300)})
        print(f"bench: fd cell {cell}: {fd[-1]}", file=sys.stderr, flush=True)
    n = rho.numel()
    s_flops = 2.0 * n * n * C * T
    t_all = t_setup + t_dec + t_adj
    res = {
        "metric": "adjoint gradient of the 64-coil misfit, end-to-end s",
        "value": round(t_all, 3), "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(1e3 * t_all, 1), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["name"], "N": n, "coils": C, "T": T, "theta": 0.5,
                   "ckpt_every": 500},
        "phases_s": {"setup": round(t_setup, 3), "decompose": round(t_dec, 3),
                     "adjoint": round(t_adj, 3)},
        "J": J, "J_forward_batched": J_fwd, "max_abs_dJ_drho": gmax,
        "max_abs_dJ_di": float(g_i.abs().max()),
        "fd_check": fd,
        "roofline": {"bound": "mfma", "kernel": "adjoint (S = sum l zeta^T GEMMs dominate)",
                     "achieved": round(s_flops / t_adj / 1e12, 3),
                     "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(s_flops / t_adj / 1e12 / FP64_PEAK_TFLOPS, 4),
                     "traffic": None},
    }
    return res


def _band_block(R) -> int:
    """Block size of R's banded factor: R's lower bandwidth rounded up to a
    multiple of 64 (at least 64), as the library chooses it."""
    import numpy as np
    rows = np.repeat(np.arange(R.shape[0]), np.diff(R.rowptr))
    band = int((rows - R.col).max()) if R.col.size else 0
    return max(64, -(-max(band, 1) // 64) * 64)


def _decomp_flops(n: int, Bb: int, full: bool) -> float:
    """Algorithmic FP64 flops of the modal decomposition: the standard form
    from R's side, two block-bidiagonal solves with n right-hand sides
    (3 Bb n^2 each: the off-diagonal product 2 Bb^2 n and the triangular
    diagonal-block product Bb^2 n per block row), the band reduction 4n^3/3;
    with the eigenvectors also the back-transforms Q2 and Q1 (2n^3 each) and
    V = H^{-T} Q' (3 Bb n^2).  The divide and conquer's merges (at most
    4n^3/3, deflation dependent) and the bulge chase (O(n^2 b)) are not
    counted."""
    f = 6.0 * Bb * float(n) ** 2 + 4.0 / 3.0 * float(n) ** 3
    if full:
        f += 4.0 * float(n) ** 3 + 3.0 * Bb * float(n) ** 2
    return f


def run_gpu(args):
    import numpy as np
    import torch
    from paper_2407_11993_amd import Solver

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    w = _workload(args.workload, args.T)
    stream = torch.cuda.current_stream()
    # waveforms resident in HBM before the timed region
    i_src = torch.as_tensor(w.i_src, dtype=torch.float64, device="cuda")

    def one_step():
        ev = {k: torch.cuda.Event(enable_timing=True) for k in
              ("start", "setup", "decomp", "modal", "full_start", "full", "chol_start", "chol")}
        ev_f = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for _ in w.thetas]
        ev["start"].record(stream)
        s = Solver(w)
        ev["setup"].record(stream)
        s.decompose(projected=True)  # the signals need Q^T G^{-1} [F, P] only
        ev["decomp"].record(stream)
        sig_m = []
        for th in w.thetas:
            s.reset()
            sig_m.append(s.step_modal(th, w.dt, w.T, i_src))
        ev["modal"].record(stream)
        # the full decomposition (eigenvector matrix formed), timed for reference
        ev["full_start"].record(stream)
        s.decompose()
        ev["full"].record(stream)
        s.reset()
        ev["chol_start"].record(stream)
        sig_c = []
        for (f0, f1), th in zip(ev_f, w.thetas):
            s.reset()
            f0.record(stream)
            s.step_cholesky(th, w.dt, 0, i_src[:1])  # the factorisation of this theta
            f1.record(stream)
            sig_c.append(s.step_cholesky(th, w.dt, w.T, i_src))
        ev["chol"].record(stream)
        torch.cuda.synchronize()
        t = {
            "setup": ev["start"].elapsed_time(ev["setup"]) / 1e3,
            "decompose": ev["setup"].elapsed_time(ev["decomp"]) / 1e3,
            "modal_steps": ev["decomp"].elapsed_time(ev["modal"]) / 1e3,
            "decompose_full": ev["full_start"].elapsed_time(ev["full"]) / 1e3,
            "cholesky": ev["chol_start"].elapsed_time(ev["chol"]) / 1e3,
            "cholesky_factor": sum(a.elapsed_time(b) for a, b in ev_f) / 1e3,
        }
        s.close()
        print("bench: step done " + " ".join(f"{k}={v:.3f}s" for k, v in t.items()),
              file=sys.stderr, flush=True)
        return t, sig_m, sig_c

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times = []
    for _ in range(args.steps):
        t, sig_m, sig_c = one_step()
        times.append(t)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    agree = max(float((a - b).abs().max() / b.abs().max()) for a, b in zip(sig_m, sig_c))
    avg = {k: sum(x[k] for x in times) / len(times) for k in times[0]}
    modal_s = avg["setup"] + avg["decompose"] + avg["modal_steps"]
    # the Cholesky method needs the same problem setup (L assembly is inside
    # its factorisation)
    chol_s = avg["setup"] + avg["cholesky"]
    n = w.n
    nsteps_total = w.T * len(w.thetas)
    # dominant kernel group: the two triangular solves of every Cholesky step.
    # Algorithmic bytes per step: the lower triangle of the factor read once
    # per solve, 2 * 8 * n(n+1)/2.
    trsv_bytes = 2 * 8.0 * n * (n + 1) / 2
    per_step = (avg["cholesky"] - avg["cholesky_factor"]) / nsteps_total
    achieved = trsv_bytes / per_step / 1e9
    res = {
        "metric": "end-to-end s, modal theta-method (Cholesky theta-method beside it)",
        "value": round(modal_s, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "N": n, "T": w.T, "thetas": list(w.thetas),
                   "dt": w.dt, "probes": w.n_probe,
                   "decomposition": "eigenvalues and projected weights V^T [F, P] "
                                    "(the eigenvector matrix is not formed)"},
        "cholesky_s": round(chol_s, 4),
        "speedup_modal_vs_cholesky": round(chol_s / modal_s, 3),
        "signal_agreement_modal_vs_cholesky": agree,
        "phases_s": {k: round(v, 4) for k, v in avg.items()},
        "modal_with_eigenvectors_s": round(avg["setup"] + avg["decompose_full"]
                                           + avg["modal_steps"], 4),
        "decomposition_tflops": round(_decomp_flops(n, _band_block(w.R), full=True)
                                      / avg["decompose_full"] / 1e12, 3),
        "roofline": {"bound": "hbm", "kernel": "triangular solve pair (fwd+bwd per step)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }
    return res


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args):
    """The oracle (plain C, one thread) on a bounded sample of the same kind
    of workload: three small plates, each timed for the decomposition
    (Cholesky, standard form, cyclic Jacobi, eigenvectors), the modal steps
    and the direct Cholesky stepper.  Power laws t = a N^b fitted to the three
    sizes (least squares in log-log) extrapolate the decomposition to the
    workload's N and the steps to its N and T; the fitted exponents are
    reported beside the value, which is an extrapolation."""
    import numpy as np
    import oracle
    from paper_2407_11993_amd import inputs
    oracle.build(force=False)
    t_sample = 2000
    if args.workload.endswith("-electrodes"):
        full = _electrode_workload(args.workload, args.T)
        samples = [inputs.electrode_plate(nx, ny, ew, T=t_sample)
                   for nx, ny, ew in ((12, 18, 4), (16, 24, 4), (20, 30, 6))]
        what = "plates of 12x18, 16x24 and 20x30 cells with two electrodes"
    else:
        full = _workload(args.workload, args.T)
        samples = []
        for side in (14, 18, 24):
            c0 = side // 2 - 2
            samples.append(inputs.plate(side, side, seed=0, crack=((c0, c0 + 4), (c0, c0 + 1), 1e3),
                                        T=t_sample, wave="gauss",
                                        coil=((side - 1) / 2, (side - 1) / 2, 2.0)))
        what = "square plates of 14, 18 and 24 cells a side with a crack"
    ns, t_dec, t_mod, t_dir = [], [], [], []
    for w, reps in zip(samples, (3, 2, 1)):  # best of a few at the small sizes
        L = oracle.assemble_L(w.xyz, w.h)
        pb = oracle.Problem(L, w.R.to_dense(), w.M, w.P,
                            E=None if w.E is None else w.E.to_dense())
        i_D = w.i_D if w.m else None
        td = tm = tc = math.inf
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.modal_eigen(pb, want_V=True)
            d = time.perf_counter() - t0
            td = min(td, d)
            t0 = time.perf_counter()
            oracle.theta_modal(pb, 0.5, 1.0, t_sample, w.i_src, i_D)
            tm = min(tm, max(time.perf_counter() - t0 - d, 1e-6))
            t0 = time.perf_counter()
            oracle.theta_direct(pb, 0.5, 1.0, t_sample, w.i_src, i_D)
            tc = min(tc, time.perf_counter() - t0)
        ns.append(w.n)
        t_dec.append(td)
        t_mod.append(tm / t_sample)
        t_dir.append(tc / t_sample)
        print(f"bench: cpu baseline N={w.n}: decomposition {td:.2f} s, modal steps "
              f"{tm:.2f} s, direct {tc:.2f} s", file=sys.stderr, flush=True)

    def fit(t):
        b, a = np.polyfit(np.log(ns), np.log(t), 1)
        return float(b), (lambda n: float(math.exp(a) * n ** b))

    b_dec, f_dec = fit(t_dec)
    b_dir, f_dir = fit(t_dir)
    nth = len(full.thetas)
    n_full = full.n - full.m
    # the modal steps are N scalar recurrences per step: linear in N, the
    # constant taken from the largest sample (a difference of two timings,
    # too noisy at the small sizes for a fit of its own)
    step_modal = t_mod[-1] * n_full / ns[-1]
    modal_est = f_dec(n_full) + step_modal * full.T * nth
    chol_est = f_dir(n_full) * full.T * nth
    # the same from the largest sample by the textbook exponents (N^3 for the
    # decomposition, N^2 per direct step)
    r = n_full / ns[-1]
    modal_text = t_dec[-1] * r ** 3 + step_modal * full.T * nth
    chol_text = t_dir[-1] * r ** 2 * full.T * nth
    return {"value": round(modal_est, 1), "unit": "s", "cores": 1, "kind": "oracle",
            "extrapolated": True,
            "host": {"cpus": os.cpu_count(), "model": _cpu_model()},
            "sample": (f"oracle modal path (Jacobi decomposition + modal theta-steps) and "
                       f"direct Cholesky stepper, one thread, on {what} (N = "
                       f"{', '.join(str(n) for n in ns)}; T = {t_sample}, theta = 0.5): "
                       f"decomposition {', '.join(f'{t:.2f}' for t in t_dec)} s; value "
                       f"extrapolated to N = {n_full}, T = {full.T} x {nth} theta(s) by the "
                       f"fitted power laws"),
            "fitted_exponents": {"decomposition": round(b_dec, 2),
                                 "direct_step": round(b_dir, 2)},
            "cholesky_estimate_s": round(chol_est, 1),
            "textbook_exponents_estimate_s": {"modal": round(modal_text, 1),
                                              "cholesky": round(chol_text, 1)}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1,
                    help="untimed runs first (the electrode plates warm up on a 48x72 plate)")
    ap.add_argument("--workload", default="plate-256x384-electrodes",
                    help="plate-256x384-electrodes (N = 98,304, 1e5 steps: the headline), "
                         "plate-WxH-electrodes, plate-128x128-crack, block-8x8x8, "
                         "batched-coils-128x128, adjoint-128x256, scan-block-8x8x8")
    ap.add_argument("--T", type=int, default=None, help="override the step count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fd-cells", type=int, default=2,
                    help="adjoint workload: cells checked by central differences")
    ap.add_argument("--chol-steps", type=int, default=300,
                    help="electrode plates: Cholesky steps measured (the rest extrapolated)")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="electrode plates: wall-clock seconds from process start within "
                         "which timed runs are added (at least one is always run)")
    ap.add_argument("--no-many-probes", action="store_true",
                    help="electrode plates: skip the run observed at 301 points")
    ap.add_argument("--cpu-reserve-s", type=float, default=60.0,
                    help="electrode plates: seconds of the budget kept for the CPU baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus above 1 is not supported "
              "(the design document describes how the method would shard)", file=sys.stderr)
        sys.exit(2)
    if args.workload.startswith("batched"):
        res = run_batched(args)
    elif args.workload.startswith("adjoint"):
        res = run_adjoint(args)
    elif args.workload.startswith("scan"):
        res = run_scan(args)
    elif args.workload.endswith("-electrodes"):
        res = run_electrodes(args)
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = cpu_baseline(args)
    else:
        res = run_gpu(args)
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
