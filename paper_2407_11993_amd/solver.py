"""Thin Python front end of libmm: device buffers (torch) in, device buffers out.

Every step of the method runs in libmm's HIP kernels; this module only moves
the problem data to the GPU, calls the C ABI and wraps the results.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib


def _dev(a, dtype=torch.float64, device="cuda"):
    if isinstance(a, torch.Tensor):
        return a.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)


def _colmajor(a: np.ndarray, rows: int) -> np.ndarray:
    """(rows x c) numpy array -> column-major flat buffer."""
    a = np.asarray(a, dtype=np.float64).reshape(rows, -1)
    return np.ascontiguousarray(a.T).ravel()


class Solver:
    """One problem (Sec. 3.1) on one GPU: the modal and the Cholesky method.

    ``workload`` is a :class:`paper_2407_11993_amd.inputs.Workload` (or any
    object with the same fields: xyz, h, R (CSR), M, P, E).  An attribute
    ``L`` (an n x n symmetric positive definite matrix, numpy or torch) is
    handed to the library as the inductance matrix itself instead of the
    generator xyz, h; the device copy is kept by the solver, which the
    library borrows.
    """

    def __init__(self, workload, device: str = "cuda"):
        self.lib = _lib.lib()
        w = workload
        self.device = device
        L = getattr(w, "L", None)
        self.n = int(w.xyz.shape[0]) if L is None else int(L.shape[0])
        self.m = 0 if w.E is None else int(w.E.shape[0])
        self.n_src = int(w.M.shape[1])
        self.n_probe = int(w.P.shape[0])
        # device copies of the problem statement (kept alive by self)
        # column-major device copy (the library reads its lower triangle)
        self._L = None if L is None else _dev(
            L.T if isinstance(L, torch.Tensor) else np.asarray(L).T)
        self._xyz = None if L is not None else _dev(w.xyz.reshape(-1))
        self._rp = _dev(w.R.rowptr, torch.int64)
        self._rc = _dev(w.R.col, torch.int32)
        # the resistance values may be given as a device tensor (R_val), e.g.
        # built from a resistivity field by torch
        rv = getattr(w, "R_val", None)
        self._rv = rv if isinstance(rv, torch.Tensor) else _dev(w.R.val)
        self._M = _dev(_colmajor(w.M, self.n)) if self.n_src else None
        self._P = _dev(_colmajor(w.P.T, self.n))
        if self.m:
            self._ep = _dev(w.E.rowptr, torch.int64)
            self._ec = _dev(w.E.col, torch.int32)
            self._ev = _dev(w.E.val)
        pb = _lib.Problem()
        pb.n = self.n
        pb.xyz = _lib.ptr(self._xyz)
        pb.h = float(w.h) if L is None else 0.0
        if L is not None:
            pb.L = _lib.ptr(self._L)
            pb.ldl = self.n
        pb.r_nnz = int(w.R.val.size)
        pb.r_rowptr, pb.r_col, pb.r_val = (_lib.ptr(self._rp), _lib.ptr(self._rc),
                                           _lib.ptr(self._rv))
        pb.n_e = self.m + 1 if self.m else 0
        if self.m:
            pb.e_nnz = int(w.E.val.size)
            pb.e_rowptr, pb.e_col, pb.e_val = (_lib.ptr(self._ep), _lib.ptr(self._ec),
                                               _lib.ptr(self._ev))
        pb.n_src = self.n_src
        pb.M0 = _lib.ptr(self._M)
        pb.n_probe = self.n_probe
        pb.P = _lib.ptr(self._P)
        ctx = ctypes.c_void_p()
        _lib.check(self.lib.mm_setup(ctypes.byref(pb), _lib.stream_handle(), ctypes.byref(ctx)))
        self.ctx = ctx
        info = (ctypes.c_int64 * 3)()
        _lib.check(self.lib.mm_info(self.ctx, info), self.ctx)
        self.n0 = int(info[1])

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.mm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the method -----------------------------------------------------------
    def decompose(self, projected=False):
        """mm_decompose, or with projected=True mm_decompose_projected (the
        eigenvalues and projected weights only, no eigenvector matrix)."""
        fn = self.lib.mm_decompose_projected if projected else self.lib.mm_decompose
        _lib.check(fn(self.ctx), self.ctx)

    def _waves(self, n_steps, i_src, i_D):
        s = None if self.n_src == 0 else _dev(np.asarray(i_src).reshape(n_steps + 1, self.n_src)
                                              if not isinstance(i_src, torch.Tensor) else i_src)
        d = None if self.m == 0 else _dev(np.asarray(i_D).reshape(n_steps + 1, self.m)
                                          if not isinstance(i_D, torch.Tensor) else i_D)
        return s, d

    def step_modal(self, theta, dt, n_steps, i_src, i_D=None, out=None):
        s, d = self._waves(n_steps, i_src, i_D)
        sig = out if out is not None else torch.empty(
            (n_steps, self.n_probe), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_step_modal(self.ctx, float(theta), float(dt), int(n_steps),
                                          _lib.ptr(s), _lib.ptr(d), _lib.ptr(sig)), self.ctx)
        self._keep = (s, d)
        return sig

    def step_modal_exact(self, dt, n_steps, i_src, i_D=None, out=None):
        """Modal stepping with exact per-mode integration (waveforms linear
        between samples); same state and signal as step_modal."""
        s, d = self._waves(n_steps, i_src, i_D)
        sig = out if out is not None else torch.empty(
            (n_steps, self.n_probe), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_step_modal_exact(self.ctx, float(dt), int(n_steps),
                                                _lib.ptr(s), _lib.ptr(d), _lib.ptr(sig)),
                   self.ctx)
        self._keep = (s, d)
        return sig

    def step_modal_scan(self, theta, dt, n_steps, i_src, i_D=None, exact=False, out=None):
        """step_modal (or step_modal_exact with exact=True), parallel in time."""
        s, d = self._waves(n_steps, i_src, i_D)
        sig = out if out is not None else torch.empty(
            (n_steps, self.n_probe), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_step_modal_scan(self.ctx, float(theta), int(bool(exact)),
                                               float(dt), int(n_steps), _lib.ptr(s),
                                               _lib.ptr(d), _lib.ptr(sig)), self.ctx)
        self._keep = (s, d)
        return sig

    def select_modes(self, tol):
        """Keep the modes whose coupling score exceeds tol times the largest
        (mm_select_modes); returns the kept mode indices (int64, on the device,
        ascending).  step_modal_selective then steps only those."""
        nk = ctypes.c_int64(0)
        idx = torch.empty(max(self.n0, 1), dtype=torch.int64, device=self.device)
        _lib.check(self.lib.mm_select_modes(self.ctx, float(tol), ctypes.byref(nk),
                                            _lib.ptr(idx)), self.ctx)
        return idx[:nk.value]

    def step_modal_selective(self, theta, dt, n_steps, i_src, i_D=None, exact=False,
                             scan=False, out=None):
        """step_modal (or step_modal_exact with exact=True) on the kept modes;
        scan=True runs the steps parallel in time."""
        s, d = self._waves(n_steps, i_src, i_D)
        sig = out if out is not None else torch.empty(
            (n_steps, self.n_probe), dtype=torch.float64, device=self.device)
        flags = (_lib.MM_STEP_EXACT if exact else 0) | (_lib.MM_STEP_SCAN if scan else 0)
        _lib.check(self.lib.mm_step_modal_selective(self.ctx, float(theta), flags,
                                                    float(dt), int(n_steps), _lib.ptr(s),
                                                    _lib.ptr(d), _lib.ptr(sig)), self.ctx)
        self._keep = (s, d)
        return sig

    def phasors(self, omegas, amp_src, amp_D=None):
        """Steady-state phasors (n_w x n_probe, complex) of the probe signals
        P dI/dt for sources Re{amp_src[w, c] exp(j omegas[w] t)} and electrode
        currents Re{amp_D[w, a] exp(j omegas[w] t)}."""
        om = _dev(torch.as_tensor(omegas, dtype=torch.float64).reshape(-1))
        nw = om.numel()

        def pairs(a, cols):
            if cols == 0:
                return None
            a = torch.as_tensor(a, dtype=torch.complex128).reshape(nw, cols)
            return _dev(torch.view_as_real(a.contiguous()).contiguous())

        src = pairs(amp_src, self.n_src)
        dd = pairs(amp_D, self.m) if self.m else None
        out = torch.empty((nw, self.n_probe, 2), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_modal_phasors(self.ctx, int(nw), _lib.ptr(om), _lib.ptr(src),
                                             _lib.ptr(dd), _lib.ptr(out)), self.ctx)
        self._keep = (om, src, dd)
        return torch.view_as_complex(out)

    def step_cholesky(self, theta, dt, n_steps, i_src, i_D=None, out=None):
        s, d = self._waves(n_steps, i_src, i_D)
        sig = out if out is not None else torch.empty(
            (n_steps, self.n_probe), dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_step_cholesky(self.ctx, float(theta), float(dt), int(n_steps),
                                             _lib.ptr(s), _lib.ptr(d), _lib.ptr(sig)), self.ctx)
        self._keep = (s, d)
        return sig

    def current(self, which=_lib.MM_MODAL, rows=None):
        if rows is None:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
            _lib.check(self.lib.mm_probe(self.ctx, which, 0, None, _lib.ptr(out)), self.ctx)
            return out
        r = _dev(_colmajor(rows, self.n))
        k = r.numel() // self.n
        out = torch.empty(k, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_probe(self.ctx, which, k, _lib.ptr(r), _lib.ptr(out)), self.ctx)
        return out

    def batch(self, theta, dt, lens, src, probe, waves, tile=-1):
        """Plan of many independent modal runs (one launch, one HIP graph).

        ``lens``, ``src``, ``probe``: per-run steps, source column and probe
        column; ``waves``: the runs' waveforms packed one after the other
        (lens[r] + 1 samples each).  Returns a :class:`Batch`; its
        ``run()`` fills and returns the packed signals (sum(lens) values)."""
        return Batch(self, theta, dt, lens, src, probe, waves, tile)

    def adjoint(self, theta, dt, n_steps, src, probe, i_src, s_obs, ckpt_every=500):
        """J, dJ/dR (at R's stored entries) and dJ/di_src for the misfit of
        runs that share the waveform i_src (mm_adjoint_modal)."""
        src = np.ascontiguousarray(src, dtype=np.int32)
        probe = np.ascontiguousarray(probe, dtype=np.int32)
        wave = _dev(i_src) if not isinstance(i_src, torch.Tensor) else i_src
        obs = _dev(s_obs) if not isinstance(s_obs, torch.Tensor) else s_obs
        assert wave.numel() == n_steps + 1 and obs.numel() == src.size * n_steps
        J = torch.empty(1, dtype=torch.float64, device=self.device)
        gR = torch.empty(self._rv.numel(), dtype=torch.float64, device=self.device)
        gi = torch.empty(n_steps + 1, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_adjoint_modal(
            self.ctx, float(theta), float(dt), int(n_steps), int(src.size),
            src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            probe.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            _lib.ptr(wave.contiguous()), _lib.ptr(obs.contiguous()), int(ckpt_every),
            _lib.ptr(J), _lib.ptr(gR), _lib.ptr(gi)), self.ctx)
        return J[0], gR, gi

    def reset(self):
        _lib.check(self.lib.mm_reset_state(self.ctx), self.ctx)

    def get_state(self, which=_lib.MM_CHOLESKY):
        """The method's stepping state (n doubles: reduced unknowns, then the
        injected currents of its last step), for a later set_state."""
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_get_state(self.ctx, which, _lib.ptr(out)), self.ctx)
        return out

    def set_state(self, state, which=_lib.MM_CHOLESKY):
        st = _dev(state)
        assert st.numel() == self.n, "the state holds n values"
        _lib.check(self.lib.mm_set_state(self.ctx, which, _lib.ptr(st)), self.ctx)
        torch.cuda.current_stream().synchronize()  # st may be released on return

    def eigenvalues(self):
        out = torch.empty(self.n0, dtype=torch.float64, device=self.device)
        _lib.check(self.lib.mm_eigenvalues(self.ctx, _lib.ptr(out)), self.ctx)
        return out


class _Kernels:
    """The dense building blocks (mmk_* entry points) on torch tensors.

    Matrices are passed as torch tensors holding the column-major layout, i.e.
    the transpose view of a row-major (C-order) tensor is used: a tensor ``A``
    of shape (cols, rows) in C order is the column-major (rows x cols) matrix.
    The helpers below take and return ordinary row-major torch matrices and
    do the transposition.
    """

    @staticmethod
    def _cm(A: torch.Tensor) -> torch.Tensor:
        return A.t().contiguous()  # column-major storage of A

    def gemm(self, A, B, trans_a=False, trans_b=False, alpha=1.0, beta=0.0, C=None):
        A = _dev(A)
        B = _dev(B)
        opA = A.t() if trans_a else A
        opB = B.t() if trans_b else B
        m, k = opA.shape
        n = opB.shape[1]
        Ac, Bc = self._cm(A), self._cm(B)
        Cc = self._cm(_dev(C)) if C is not None else torch.zeros(n, m, dtype=torch.float64,
                                                                 device=A.device)
        _lib.check(_lib.lib().mmk_dgemm(int(trans_a), int(trans_b), m, n, k, float(alpha),
                                        _lib.ptr(Ac), A.shape[0], _lib.ptr(Bc), B.shape[0],
                                        float(beta), _lib.ptr(Cc), max(1, m),
                                        _lib.stream_handle()))
        return Cc.t()

    def gemm_tri(self, A, B, trans_a=False, trans_b=False, alpha=1.0, beta=0.0, C=None,
                 flags=0, b_band=-1):
        """gemm with structure flags (MMK_LOWER, MMK_A_LOWER, MMK_A_UPPER, MMK_B_LOWER)
        and a band of op(B); the zero parts must be stored as zeros."""
        A = _dev(A)
        B = _dev(B)
        opA = A.t() if trans_a else A
        opB = B.t() if trans_b else B
        m, k = opA.shape
        n = opB.shape[1]
        Ac, Bc = self._cm(A), self._cm(B)
        Cc = self._cm(_dev(C)) if C is not None else torch.zeros(n, m, dtype=torch.float64,
                                                                 device=A.device)
        _lib.check(_lib.lib().mmk_dgemm_tri(int(trans_a), int(trans_b), m, n, k, float(alpha),
                                            _lib.ptr(Ac), A.shape[0], _lib.ptr(Bc), B.shape[0],
                                            float(beta), _lib.ptr(Cc), max(1, m), int(flags),
                                            int(b_band), _lib.stream_handle()))
        return Cc.t()

    def symm_lower(self, A, B, alpha=1.0, beta=0.0, C=None):
        """alpha A B + beta C with A symmetric; only A's lower triangle is read."""
        A = _dev(A)
        B = _dev(B)
        m, n = B.shape
        Ac, Bc = self._cm(A), self._cm(B)
        Cc = self._cm(_dev(C)) if C is not None else torch.zeros(n, m, dtype=torch.float64,
                                                                 device=A.device)
        _lib.check(_lib.lib().mmk_dsymm_lower(m, n, float(alpha), _lib.ptr(Ac), max(1, m),
                                              _lib.ptr(Bc), max(1, m), float(beta),
                                              _lib.ptr(Cc), max(1, m), _lib.stream_handle()))
        return Cc.t()

    def potrf(self, A):
        Ac = self._cm(_dev(A))
        n = Ac.shape[0]
        info = ctypes.c_int64(0)
        _lib.check(_lib.lib().mmk_dpotrf(n, _lib.ptr(Ac), max(1, n), ctypes.byref(info),
                                         _lib.stream_handle()))
        return Ac.t(), int(info.value)

    def trtri(self, G):
        Gc = self._cm(_dev(G))
        n = Gc.shape[0]
        _lib.check(_lib.lib().mmk_dtrtri(n, _lib.ptr(Gc), max(1, n), _lib.stream_handle()))
        return Gc.t()

    def sy2sb(self, A, nb):
        Ac = self._cm(_dev(A))
        n = Ac.shape[0]
        ldab = 2 * nb + 1
        AB = torch.zeros(n, ldab, dtype=torch.float64, device=Ac.device)
        _lib.check(_lib.lib().mmk_dsy2sb(n, _lib.ptr(Ac), n, nb, _lib.ptr(AB), ldab,
                                         _lib.stream_handle()))
        return AB  # AB[j, d] = B(j + d, j)

    def sb2st(self, AB, nb):
        AB = _dev(AB).clone()
        n, ldab = AB.shape
        d = torch.empty(n, dtype=torch.float64, device=AB.device)
        e = torch.empty(max(1, n - 1), dtype=torch.float64, device=AB.device)
        _lib.check(_lib.lib().mmk_dsb2st(n, nb, _lib.ptr(AB), ldab, _lib.ptr(d), _lib.ptr(e),
                                         _lib.stream_handle()))
        return d, e[:n - 1]

    def stedc(self, d, e):
        d = _dev(d)
        n = d.numel()
        e = _dev(e) if n > 1 else torch.zeros(1, dtype=torch.float64, device=d.device)
        w = torch.empty(n, dtype=torch.float64, device=d.device)
        Z = torch.empty(n, n, dtype=torch.float64, device=d.device)
        _lib.check(_lib.lib().mmk_dstedc(n, _lib.ptr(d), _lib.ptr(e), _lib.ptr(w),
                                         _lib.ptr(Z), _lib.stream_handle()))
        return w, Z.t()

    def syevd(self, A, nb=64):
        Ac = self._cm(_dev(A))
        n = Ac.shape[0]
        w = torch.empty(n, dtype=torch.float64, device=Ac.device)
        Z = torch.empty(n, n, dtype=torch.float64, device=Ac.device)
        _lib.check(_lib.lib().mmk_dsyevd(n, _lib.ptr(Ac), n, int(nb), _lib.ptr(w), _lib.ptr(Z),
                                         _lib.stream_handle()))
        return w, Z.t()


kernels = _Kernels()


class Batch:
    """Batched modal runs over one decomposed :class:`Solver` (mm_batch_*)."""

    def __init__(self, solver, theta, dt, lens, src, probe, waves, tile=-1):
        self.solver = solver
        lib = solver.lib
        self.lens = np.ascontiguousarray(lens, dtype=np.int64)
        src = np.ascontiguousarray(src, dtype=np.int32)
        probe = np.ascontiguousarray(probe, dtype=np.int32)
        n = self.lens.size
        assert src.size == n and probe.size == n
        total = int(self.lens.sum())
        self.waves = _dev(waves) if not isinstance(waves, torch.Tensor) else waves
        assert self.waves.numel() == total + n
        self.signals = torch.empty(max(total, 1), dtype=torch.float64, device=solver.device)
        self.offsets = np.concatenate([[0], np.cumsum(self.lens)])
        h = ctypes.c_void_p()
        _lib.check(lib.mm_batch_create(
            solver.ctx, float(theta), float(dt), n,
            self.lens.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            probe.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
            _lib.ptr(self.waves), _lib.ptr(self.signals), int(tile), ctypes.byref(h)),
            solver.ctx)
        self.h = h
        info = (ctypes.c_int64 * 4)()
        _lib.check(lib.mm_batch_info(self.h, info), solver.ctx)
        self.threads, self.modes, self.groups, self.total = (int(v) for v in info)

    def run(self):
        _lib.check(self.solver.lib.mm_batch_run(self.h), self.solver.ctx)
        return self.signals[:self.total]

    def signal(self, r):
        """Signal of run r (a view into the packed output)."""
        return self.signals[self.offsets[r]:self.offsets[r + 1]]

    def close(self):
        if getattr(self, "h", None):
            self.solver.lib.mm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
