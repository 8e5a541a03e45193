"""Seeded synthetic workloads (problem data only).

This module builds the *problem statement* that both the GPU library and
the CPU oracle are given: cell centres, the resistance matrix R, source
mutual inductances M0, probe rows P, the reduced electrode incidence E and
the source waveforms sampled at t_k = k dt.  It holds none of the method's
arithmetic: the inductance matrix L, every factorisation, the modal
decomposition and the time stepping are computed separately by each side.

The paper's own workload (an Inconel tube meshed with 100,676 edge-element
unknowns, Sec. 4.1 and 4.6) is not available; these plates stand in for it.

Conventions
-----------
* Cells sit on a unit grid with centre (x, y, z), x in [0, nx) etc., and
  index ``x + nx * (y + ny * z)``.
* R is the Galerkin resistance matrix (Sec. 3.1, R_jk) of the stand-in:
  a 6-neighbour graph Laplacian with edge weight (rho_i + rho_j)/2 (two
  half-cells in series) plus a constant 0.05 on the diagonal, so that R is
  SPD as the paper requires (Sec. 3.1, "strictly positive resistivity").
* A point coil at p couples to cell i through M_i = h / sqrt(|x_i-p|^2+h^2),
  the same smooth kernel as the inductance stand-in, so V0 = -M0 di0/dt
  (Sec. 3.1, eq. induced_voltages_0).
* The probe of a coil is the coil itself: the signal is M0^T dI/dt.
* E (electrodes) is the (Ne-1) x N reduced incidence with the last electrode
  excluded (Sec. 3.1, eq. definition_E); for two electrodes of cells S1, S2
  it is the single row 1_{S1} - 1_{S2}.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

H_KERNEL = 0.7
R_SHIFT = 0.05


@dataclasses.dataclass
class CSR:
    shape: tuple
    rowptr: np.ndarray  # int64, rows + 1
    col: np.ndarray     # int32
    val: np.ndarray     # float64

    def to_dense(self) -> np.ndarray:
        out = np.zeros(self.shape)
        for i in range(self.shape[0]):
            lo, hi = self.rowptr[i], self.rowptr[i + 1]
            np.add.at(out[i], self.col[lo:hi], self.val[lo:hi])
        return out


@dataclasses.dataclass
class Workload:
    """One synthetic problem plus the run parameters."""
    name: str
    dims: tuple                 # (nx, ny, nz)
    xyz: np.ndarray             # N x 3
    h: float
    rho: np.ndarray             # N
    R: CSR                      # N x N
    M: np.ndarray               # N x n_src  (coil couplings)
    P: np.ndarray               # n_probe x N
    E: Optional[CSR]            # (Ne-1) x N or None
    thetas: tuple
    dt: float
    T: int
    i_src: np.ndarray           # (T+1) x n_src
    i_D: np.ndarray             # (T+1) x (Ne-1)
    lengths: Optional[np.ndarray] = None   # batched runs: steps per source

    @property
    def n(self) -> int:
        return self.xyz.shape[0]

    @property
    def m(self) -> int:
        return 0 if self.E is None else self.E.shape[0]

    @property
    def n_src(self) -> int:
        return self.M.shape[1]

    @property
    def n_probe(self) -> int:
        return self.P.shape[0]


# ---------------------------------------------------------------------------
# geometry and fields
# ---------------------------------------------------------------------------
def grid(nx: int, ny: int, nz: int) -> np.ndarray:
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                          indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(np.float64)


def cell(dims, x, y, z=0) -> int:
    nx, ny, _ = dims
    return int(x + nx * (y + ny * z))


def rho_loguniform(n: int, seed: int, lo: float = 0.5, hi: float = 2.0):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def paint_box(rho, dims, xr, yr, value, zr=(0, 1)):
    for z in range(*zr):
        for y in range(*yr):
            for x in range(*xr):
                rho[cell(dims, x, y, z)] = value
    return rho


def resistance_csr(dims, rho, shift: float = R_SHIFT) -> CSR:
    """6-neighbour Laplacian, weights (rho_i+rho_j)/2, plus shift*I."""
    nx, ny, nz = dims
    n = nx * ny * nz
    rows = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                i = cell(dims, x, y, z)
                ent = {}
                diag = shift
                for dx, dy, dz in ((-1, 0, 0), (1, 0, 0), (0, -1, 0),
                                   (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                    xx, yy, zz = x + dx, y + dy, z + dz
                    if 0 <= xx < nx and 0 <= yy < ny and 0 <= zz < nz:
                        j = cell(dims, xx, yy, zz)
                        w = 0.5 * (rho[i] + rho[j])
                        ent[j] = -w
                        diag += w
                ent[i] = diag
                rows.append(sorted(ent.items()))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum([len(r) for r in rows])
    col = np.fromiter((c for r in rows for c, _ in r), dtype=np.int32,
                      count=int(rowptr[-1]))
    val = np.fromiter((v for r in rows for _, v in r), dtype=np.float64,
                      count=int(rowptr[-1]))
    return CSR((n, n), rowptr, col, val)


def resistance_csr_fast(dims, rho, shift: float = R_SHIFT) -> CSR:
    """Vectorised twin of :func:`resistance_csr` for large grids."""
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    src, dst = [], []
    for axis in range(3):
        a = np.take(idx, np.arange(idx.shape[axis] - 1), axis=axis).ravel()
        b = np.take(idx, np.arange(1, idx.shape[axis]), axis=axis).ravel()
        src += [a, b]
        dst += [b, a]
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    w = 0.5 * (rho[src] + rho[dst])
    diag = np.full(n, shift)
    np.add.at(diag, src, w)
    r = np.concatenate([src, np.arange(n)])
    c = np.concatenate([dst, np.arange(n)])
    v = np.concatenate([-w, diag])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return CSR((n, n), rowptr, c.astype(np.int32), v.astype(np.float64))


def resistance_model(dims, shift: float = R_SHIFT):
    """The resistance values as a linear function of the cell resistivities,
    R.val = A rho + c, on the pattern (and entry order) of
    :func:`resistance_csr_fast`.  Returns (rowptr, col, A as COO triples
    (entry, cell, coefficient), c)."""
    nx, ny, nz = dims
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    src, dst = [], []
    for axis in range(3):
        a = np.take(idx, np.arange(idx.shape[axis] - 1), axis=axis).ravel()
        b = np.take(idx, np.arange(1, idx.shape[axis]), axis=axis).ravel()
        src += [a, b]
        dst += [b, a]
    src = np.concatenate(src)
    dst = np.concatenate(dst)
    E = src.size
    r = np.concatenate([src, np.arange(n)])
    c = np.concatenate([dst, np.arange(n)])
    order = np.lexsort((c, r))
    pos = np.empty(order.size, dtype=np.int64)
    pos[order] = np.arange(order.size)
    # off-diagonal entry of edge e: -(rho_src + rho_dst) / 2
    # diagonal entry of cell i: shift + sum over its edges (rho_i + rho_j) / 2
    ent = np.concatenate([pos[:E], pos[:E], pos[E + src], pos[E + src]])
    cel = np.concatenate([src, dst, src, dst])
    coef = np.concatenate([np.full(E, -0.5), np.full(E, -0.5), np.full(E, 0.5), np.full(E, 0.5)])
    const = np.zeros(order.size)
    const[pos[E:]] = shift
    rs, cs = r[order], c[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rs + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cs.astype(np.int32), (ent, cel, coef), const


def coil_coupling(xyz, p, h: float = H_KERNEL) -> np.ndarray:
    d2 = ((xyz - np.asarray(p, dtype=np.float64)) ** 2).sum(axis=1)
    return h / np.sqrt(d2 + h * h)


def electrodes_csr(n: int, s1, s2) -> CSR:
    """Single row 1_{S1} - 1_{S2} (two electrodes, the last one excluded)."""
    cols = np.concatenate([np.asarray(s1), np.asarray(s2)])
    vals = np.concatenate([np.ones(len(s1)), -np.ones(len(s2))])
    order = np.argsort(cols)
    return CSR((1, n), np.array([0, len(cols)], dtype=np.int64),
               cols[order].astype(np.int32), vals[order])


def tk(T: int, dt: float) -> np.ndarray:
    return np.arange(T + 1, dtype=np.float64) * dt


# ---------------------------------------------------------------------------
# the five configurations (and small variants used by the tests)
# ---------------------------------------------------------------------------
def block_8x8x8(T: int = 2000) -> Workload:
    """8x8x8 block, rho = 1, one coil below it, sinusoidal drive."""
    dims = (8, 8, 8)
    xyz = grid(*dims)
    rho = np.ones(xyz.shape[0])
    R = resistance_csr(dims, rho)
    M = coil_coupling(xyz, (3.5, 3.5, -2.0))[:, None]
    t = tk(T, 1.0)
    i_src = np.sin(2 * np.pi * t / 200.0)[:, None]
    return Workload("block-8x8x8", dims, xyz, H_KERNEL, rho, R, M, M.T.copy(),
                    None, (0.5,), 1.0, T, i_src, np.zeros((T + 1, 0)))


def plate(nx: int, ny: int, *, seed: Optional[int] = 0, crack=None,
          coil=None, T: int = 10000, wave: str = "gauss",
          thetas=(0.5, 1.0), name: Optional[str] = None) -> Workload:
    """Thin plate with log-uniform resistivity, optional crack and a coil."""
    dims = (nx, ny, 1)
    xyz = grid(*dims)
    n = xyz.shape[0]
    rho = np.ones(n) if seed is None else rho_loguniform(n, seed)
    if crack is not None:
        (x0, x1), (y0, y1), val = crack
        paint_box(rho, dims, (x0, x1), (y0, y1), val)
    R = resistance_csr_fast(dims, rho)
    if coil is None:
        coil = ((nx - 1) / 2.0, (ny - 1) / 2.0, 2.0)
    M = coil_coupling(xyz, coil)[:, None]
    t = tk(T, 1.0)
    if wave == "gauss":
        i_src = np.exp(-((t - 500.0) / 100.0) ** 2)[:, None]
    else:
        i_src = np.sin(2 * np.pi * t / 200.0)[:, None]
    return Workload(name or f"plate-{nx}x{ny}", dims, xyz, H_KERNEL, rho, R,
                    M, M.T.copy(), None, tuple(thetas), 1.0, T, i_src,
                    np.zeros((T + 1, 0)))


def plate_128x128_crack(T: int = 10000) -> Workload:
    """128x128 plate, log-uniform rho in [0.5, 2] (seed 0), 10x3 crack of
    rho = 1e3, coil two cells above the centre, Gaussian pulse."""
    return plate(128, 128, seed=0, crack=((59, 69), (63, 66), 1e3),
                 coil=(63.5, 63.5, 2.0), T=T, wave="gauss",
                 thetas=(0.5, 1.0), name="plate-128x128-crack")


def electrode_plate(nx: int, ny: int, ew: int, *, T: int, tau_D: float = 2000.0,
                    coil_period: float = 500.0, name: Optional[str] = None,
                    seed: Optional[int] = None) -> Workload:
    """Plate with two electrodes of ``ew`` cells centred on the two short
    edges (y = 0 and y = ny-1), injected current iD = 1 - exp(-t/tau_D),
    and a coil above the centre driven by sin(2 pi t / coil_period)."""
    dims = (nx, ny, 1)
    xyz = grid(*dims)
    n = xyz.shape[0]
    rho = np.ones(n) if seed is None else rho_loguniform(n, seed)
    R = resistance_csr_fast(dims, rho)
    x0 = (nx - ew) // 2
    s1 = [cell(dims, x, 0) for x in range(x0, x0 + ew)]
    s2 = [cell(dims, x, ny - 1) for x in range(x0, x0 + ew)]
    E = electrodes_csr(n, s1, s2)
    M = coil_coupling(xyz, ((nx - 1) / 2.0, (ny - 1) / 2.0, 2.0))[:, None]
    t = tk(T, 1.0)
    i_src = np.sin(2 * np.pi * t / coil_period)[:, None]
    i_D = (1.0 - np.exp(-t / tau_D))[:, None]
    return Workload(name or f"electrode-plate-{nx}x{ny}", dims, xyz, H_KERNEL,
                    rho, R, M, M.T.copy(), E, (0.5,), 1.0, T, i_src, i_D)


def adjoint_plate_128x256(nx: int = 128, ny: int = 256, n_i: int = 8, n_j: int = 8, T: int = 10000,
            seed: int = 5):
    """Adjoint workload: background resistivity log-uniform (seed 5), the
    reference field adds defect A (x in [40,52), y in [60,63), rho = 1e3) and
    defect B (x in [80,86), y in [180,186), rho = 5); n_i x n_j coils at
    (16 i + 7.5, 32 j + 15.5, 2) sharing the Gaussian pulse of the 128x128
    plate.  Returns a dict (dims, xyz, rho_bg, rho_ref, M, i_src, T)."""
    dims = (nx, ny, 1)
    xyz = grid(*dims)
    n = xyz.shape[0]
    rho_bg = rho_loguniform(n, seed)
    rho_ref = rho_bg.copy()
    paint_box(rho_ref, dims, (40, 52), (60, 63), 1e3)
    paint_box(rho_ref, dims, (80, 86), (180, 186), 5.0)
    coils = [(16 * i + 7.5, 32 * j + 15.5, 2.0) for j in range(n_j) for i in range(n_i)]
    M = np.stack([coil_coupling(xyz, p) for p in coils], axis=1)
    t = tk(T, 1.0)
    i_src = np.exp(-((t - 500.0) / 100.0) ** 2)
    return dict(name=f"adjoint-{nx}x{ny}-{len(coils)}coils", dims=dims, xyz=xyz,
                rho_bg=rho_bg, rho_ref=rho_ref, M=M, i_src=i_src, T=T)


def adjoint_plate_32x64(T: int = 2000, seed: int = 5):
    """The adjoint workload at a quarter of the size in x and y: 32x64 plate
    (N = 2048), background log-uniform (seed 5), defect A at x in [10,13),
    y in [15,16) (rho = 1e3) and defect B at x in [20,22), y in [45,47)
    (rho = 5) in the reference field, 8 coils at (8 i + 3.5, 32 j + 15.5, 2),
    i < 4, j < 2, sharing the same Gaussian pulse."""
    nx, ny = 32, 64
    dims = (nx, ny, 1)
    xyz = grid(*dims)
    n = xyz.shape[0]
    rho_bg = rho_loguniform(n, seed)
    rho_ref = rho_bg.copy()
    paint_box(rho_ref, dims, (10, 13), (15, 16), 1e3)
    paint_box(rho_ref, dims, (20, 22), (45, 47), 5.0)
    coils = [(8 * i + 3.5, 32 * j + 15.5, 2.0) for j in range(2) for i in range(4)]
    M = np.stack([coil_coupling(xyz, p) for p in coils], axis=1)
    t = tk(T, 1.0)
    i_src = np.exp(-((t - 500.0) / 100.0) ** 2)
    return dict(name=f"adjoint-{nx}x{ny}-{len(coils)}coils", dims=dims, xyz=xyz,
                rho_bg=rho_bg, rho_ref=rho_ref, M=M, i_src=i_src, T=T)


def plate_256x384_electrodes(T: int = 100000) -> Workload:
    """256x384 plate, rho = 1, electrodes of 16 cells on the two short edges,
    iD = 1 - exp(-t/2000), coil at the centre with period 500."""
    return electrode_plate(256, 384, 16, T=T, name="plate-256x384-electrodes")


def batched_coils(nx: int = 128, ny: int = 128, n_side: int = 16,
                  seed: int = 4, t_lo: int = 2000, t_hi: int = 20000,
                  field_seed: int = 0) -> Workload:
    """Config-2 field with n_side^2 coils on a lift-off-2 grid; each coil has
    its own length in [t_lo, t_hi] and a sine (period 100..1000) or a
    Gaussian pulse (t0 = T_c/4, width 50..200), chosen with p = 1/2."""
    base = plate(nx, ny, seed=field_seed, crack=((59, 69), (63, 66), 1e3)
                 if (nx, ny) == (128, 128) else None, T=1)
    rng = np.random.default_rng(seed)
    step = nx / n_side
    coils = [(step * i + step / 2 - 0.5, (ny / n_side) * j + (ny / n_side) / 2 - 0.5, 2.0)
             for j in range(n_side) for i in range(n_side)]
    M = np.stack([coil_coupling(base.xyz, p) for p in coils], axis=1)
    lengths = rng.integers(t_lo, t_hi + 1, size=len(coils))
    T = int(lengths.max())
    t = tk(T, 1.0)
    waves = np.zeros((T + 1, len(coils)))
    for c in range(len(coils)):
        Tc = int(lengths[c])
        if rng.random() < 0.5:
            period = rng.uniform(100.0, 1000.0)
            w = np.sin(2 * np.pi * t / period)
        else:
            width = rng.uniform(50.0, 200.0)
            w = np.exp(-((t - Tc / 4.0) / width) ** 2)
        w[Tc + 1:] = w[Tc]  # held after the run ends (no further increments)
        waves[:, c] = w
    return Workload(f"batched-{nx}x{ny}-{len(coils)}coils", base.dims,
                    base.xyz, H_KERNEL, base.rho, base.R, M, M.T.copy(), None,
                    (0.5,), 1.0, T, waves, np.zeros((T + 1, 0)),
                    lengths=lengths)
