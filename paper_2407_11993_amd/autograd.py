"""torch.autograd.Function around the modal adjoint (mm_adjoint_modal).

J(rho, i_src) = sum over coil runs of the squared probe-signal misfit; the
gradient comes from the library's backward modal recursion (dJ/dR at R's
stored entries, dJ/di_src), and the chain rule through the resistance model
R.val = A rho + c (:func:`inputs.resistance_model`) maps dJ/dR to dJ/drho.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import inputs
from .solver import Solver


@dataclasses.dataclass
class MisfitProblem:
    """Plate geometry, coils (sources = probes), stepping and observations."""
    dims: tuple
    M: np.ndarray          # n x C coil couplings
    obs: torch.Tensor      # C x T observed signals (device)
    theta: float = 0.5
    dt: float = 1.0
    ckpt_every: int = 500
    h: float = inputs.H_KERNEL

    def __post_init__(self):
        self.xyz = inputs.grid(*self.dims)
        n = self.xyz.shape[0]
        rowptr, col, (ent, cel, coef), const = inputs.resistance_model(self.dims)
        dev = self.obs.device
        self.rowptr, self.col = rowptr, col
        self.A = torch.sparse_coo_tensor(
            torch.as_tensor(np.stack([ent, cel])), torch.as_tensor(coef),
            (const.size, n), dtype=torch.float64).coalesce().to(dev)
        self.At = self.A.t().coalesce()
        self.c = torch.as_tensor(const, dtype=torch.float64, device=dev)
        self.T = int(self.obs.shape[1])
        self.runs = np.arange(self.M.shape[1], dtype=np.int32)

    def workload(self, R_val: torch.Tensor):
        n = self.xyz.shape[0]
        R = inputs.CSR((n, n), self.rowptr, self.col, np.zeros(self.col.size))
        w = inputs.Workload("misfit", self.dims, self.xyz, self.h, np.ones(n), R, self.M,
                            self.M.T.copy(), None, (self.theta,), self.dt, self.T,
                            np.zeros((self.T + 1, self.M.shape[1])), np.zeros((self.T + 1, 0)))
        w.R_val = R_val
        return w


class ModalMisfit(torch.autograd.Function):
    """J = ModalMisfit.apply(rho, i_src, problem) with rho (n) and i_src (T+1)
    device tensors; backward returns dJ/drho and dJ/di_src."""

    @staticmethod
    def forward(ctx, rho, i_src, pb: MisfitProblem):
        R_val = (torch.sparse.mm(pb.A, rho.detach().reshape(-1, 1)).reshape(-1) + pb.c)
        s = Solver(pb.workload(R_val.contiguous()))
        s.decompose()
        J, gR, gi = s.adjoint(pb.theta, pb.dt, pb.T, pb.runs, pb.runs,
                              i_src.detach().contiguous(), pb.obs.contiguous(), pb.ckpt_every)
        s.close()
        g_rho = torch.sparse.mm(pb.At, gR.reshape(-1, 1)).reshape(-1)
        ctx.save_for_backward(g_rho, gi)
        return J.clone()

    @staticmethod
    def backward(ctx, gJ):
        g_rho, gi = ctx.saved_tensors
        return gJ * g_rho, gJ * gi, None
