"""Seeded synthetic inputs for the EXX pair kernel.

This module only *generates inputs*: cells, grids, orbital centres, Gaussian
exponents and orbital grid values.  It holds none of the method's arithmetic
and is the one module that both the oracle-based tests and the HIP path's
tests and benchmark draw their inputs from.

The paper's workloads are PBE0 maximally localized Wannier functions of liquid
water and ice (Sec. IV); those are not available, so water-like stand-ins are
built instead: 4 localized orbitals per molecule on a jittered lattice at
liquid-water density, each a normalized Gaussian times (1 + a random linear
polynomial).  The recipe and its readings are stated in the design notes.

Seeds: configuration k uses SeedSequence(2011072090 + k), split into
independent PCG64 streams per purpose.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

BASE_SEED = 2011072090

# stream ids within a configuration's SeedSequence
_S_SITES, _S_ROT, _S_OFFSET, _S_EXPO, _S_POLY, _S_RADII, _S_DISP, _S_CENTRES = range(8)


@dataclasses.dataclass
class Config:
    key: str
    cell: tuple            # orthorhombic edge lengths (bohr)
    grid: tuple            # points along L_1, L_2, L_3
    n_orb: int
    R_pair: float
    R_PE: float
    R_ME: float
    l_max: int
    stencil_n: int
    cg_tol: float = 1e-10
    lattice: Optional[str] = None       # "sc", "bcc", "fcc" for water-like sets; None: uniform centres
    reps: int = 0                       # lattice repeats per edge
    expo: tuple = (0.9, 1.6)            # Gaussian exponent range (bohr^-2)
    poly_std: float = 0.3               # std of the linear-polynomial coefficients
    jitter: float = 0.3                 # molecule-site jitter amplitude (bohr)
    offset: tuple = (0.6, 0.9)          # orbital offset from the site along a tetrahedral direction
    R_PE_classes: Optional[tuple] = None  # (R_min, step, n_classes) for per-orbital radii
    R_orb_range: Optional[tuple] = None   # per-orbital radius range
    orb_dtype: str = "f64"
    seed_index: int = 0
    hmat: Optional[tuple] = None        # general cell: h[a + 3 al] = (L_al)_a (column-major); None: diag(cell)

    @property
    def h(self) -> np.ndarray:
        if self.hmat is not None:
            return np.asarray(self.hmat, dtype=np.float64).reshape(3, 3, order="F")
        return np.diag(np.asarray(self.cell, dtype=np.float64))

    @property
    def general(self) -> bool:
        return self.hmat is not None

    @property
    def n_points(self) -> int:
        return int(np.prod(self.grid))

    @property
    def spacing(self):
        if self.hmat is not None:
            h = self.h
            return tuple(float(np.linalg.norm(h[:, a])) / self.grid[a] for a in range(3))
        return tuple(self.cell[a] / self.grid[a] for a in range(3))

    @property
    def dV(self) -> float:
        return abs(float(np.linalg.det(self.h))) / float(np.prod(self.grid))


def _cell_matrix(a, b, c, alpha, beta, gamma):
    """Column-major h (h[a + 3 al] = (L_al)_a) of a cell with edge lengths a, b,
    c and angles alpha = (L2, L3), beta = (L1, L3), gamma = (L1, L2) in degrees;
    L1 along x, L2 in the xy plane."""
    al, be, ga = (math.radians(x) for x in (alpha, beta, gamma))
    cx = c * math.cos(be)
    cy = c * (math.cos(al) - math.cos(be) * math.cos(ga)) / math.sin(ga)
    cz = math.sqrt(c * c - cx * cx - cy * cy)
    return [a, 0.0, 0.0, b * math.cos(ga), b * math.sin(ga), 0.0, cx, cy, cz]


# The workloads: a tiny cubic cell for oracle-speed parity, and water-like
# sets of 64, 128, 256 and 512 molecules (4 orbitals each).
CONFIGS = {
    "tiny16": Config("tiny16", (12.0, 12.0, 12.0), (60, 60, 60), 16, 8.0, 5.0, 7.0, 6, 1,
                     expo=(0.8, 1.5), seed_index=1),
    "water64": Config("water64", (23.5, 23.5, 23.5), (120, 120, 120), 256, 10.0, 6.0, 9.0, 6, 3,
                      lattice="sc", reps=4, seed_index=2),
    "water128": Config("water128", (29.6, 29.6, 29.6), (150, 150, 150), 512, 10.0, 6.0, 9.0, 6, 3,
                       lattice="bcc", reps=4, seed_index=3),
    "water256": Config("water256", (37.3, 38.4, 36.5), (192, 198, 188), 1024, 10.0, 6.0, 9.0, 6, 3,
                       lattice="fcc", reps=4, R_PE_classes=(5.0, 0.25, 9), R_orb_range=(5.0, 7.0),
                       seed_index=4),
    "water512": Config("water512", (47.0, 47.0, 47.0), (240, 240, 240), 2048, 10.0, 6.0, 9.0, 8, 3,
                       lattice="sc", reps=8, orb_dtype="f32", seed_index=5),
    # water-like 64-molecule sets in non-orthogonal cells of the same volume
    # and grid spacing as water64 (Sec. III B-C): hexagonal (one auxiliary
    # stencil direction) and triclinic (three)
    "hex64": Config("hex64", (24.6, 24.6, 24.6), (126, 126, 126), 256, 10.0, 6.0, 9.0, 6, 3,
                    lattice="sc", reps=4, seed_index=6, hmat=tuple(_cell_matrix(24.6, 24.6, 24.6, 90, 90, 120))),
    "tri64": Config("tri64", (23.8, 23.8, 23.8), (122, 122, 122), 256, 10.0, 6.0, 9.0, 6, 3,
                    lattice="sc", reps=4, seed_index=7, hmat=tuple(_cell_matrix(23.8, 23.8, 23.8, 80, 95, 100))),
}


@dataclasses.dataclass
class OrbitalSet:
    centres: np.ndarray      # [n_orb, 3] Cartesian, inside the cell
    expo: np.ndarray         # [n_orb]
    poly: np.ndarray         # [n_orb, 3]
    R_orb: Optional[np.ndarray] = None  # [n_orb] per-orbital radii, or None


def _streams(cfg: Config, seed: Optional[int] = None):
    ss = np.random.SeedSequence(BASE_SEED + cfg.seed_index if seed is None else seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(8)]


def _rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a normalized 4D Gaussian quaternion (Shoemake)."""
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


_TETRA = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=np.float64) / math.sqrt(3.0)
_BASIS = {
    "sc": np.array([[0.0, 0.0, 0.0]]),
    "bcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]]),
    "fcc": np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]]),
}


def make_orbitals(cfg: Config, seed: Optional[int] = None) -> OrbitalSet:
    st = _streams(cfg, seed)
    L = np.asarray(cfg.cell, dtype=np.float64)
    if cfg.general and cfg.lattice is None:
        # general cell: uniform centres in crystal coordinates
        centres = st[_S_CENTRES].uniform(0.0, 1.0, size=(cfg.n_orb, 3)) @ cfg.h.T
    elif cfg.general:
        # molecule sites on the lattice in crystal coordinates, Cartesian jitter
        # and tetrahedral orbital offsets as for the orthorhombic sets, wrapped
        # back into the cell in crystal coordinates
        h = cfg.h
        basis = _BASIS[cfg.lattice]
        cells = np.stack(np.meshgrid(*[np.arange(cfg.reps)] * 3, indexing="ij"), -1).reshape(-1, 3)
        frac = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) / cfg.reps
        sites = frac @ h.T + st[_S_SITES].uniform(-cfg.jitter, cfg.jitter, size=frac.shape)
        n_mol = sites.shape[0]
        assert 4 * n_mol == cfg.n_orb, (n_mol, cfg.n_orb)
        centres = np.empty((cfg.n_orb, 3))
        for m in range(n_mol):
            R = _rotation(st[_S_ROT])
            dist = st[_S_OFFSET].uniform(cfg.offset[0], cfg.offset[1], size=4)
            centres[4 * m:4 * m + 4] = sites[m] + dist[:, None] * (_TETRA @ R.T)
        centres = np.mod(centres @ np.linalg.inv(h).T, 1.0) @ h.T
    elif cfg.lattice is None:
        centres = st[_S_CENTRES].uniform(0.0, 1.0, size=(cfg.n_orb, 3)) * L
    else:
        basis = _BASIS[cfg.lattice]
        cells = np.stack(np.meshgrid(*[np.arange(cfg.reps)] * 3, indexing="ij"), -1).reshape(-1, 3)
        frac = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) / cfg.reps
        sites = frac * L + st[_S_SITES].uniform(-cfg.jitter, cfg.jitter, size=frac.shape)
        n_mol = sites.shape[0]
        assert 4 * n_mol == cfg.n_orb, (n_mol, cfg.n_orb)
        centres = np.empty((cfg.n_orb, 3))
        for m in range(n_mol):
            R = _rotation(st[_S_ROT])
            dist = st[_S_OFFSET].uniform(cfg.offset[0], cfg.offset[1], size=4)
            centres[4 * m:4 * m + 4] = sites[m] + dist[:, None] * (_TETRA @ R.T)
        centres = np.mod(centres, L)
    expo = st[_S_EXPO].uniform(cfg.expo[0], cfg.expo[1], size=cfg.n_orb)
    poly = st[_S_POLY].normal(0.0, cfg.poly_std, size=(cfg.n_orb, 3))
    R_orb = None
    if cfg.R_orb_range is not None:
        R_orb = st[_S_RADII].uniform(cfg.R_orb_range[0], cfg.R_orb_range[1], size=cfg.n_orb)
    return OrbitalSet(centres=centres, expo=expo, poly=poly, R_orb=R_orb)


def displace(cfg: Config, orbs: OrbitalSet, step: int, amplitude: float = 0.02) -> OrbitalSet:
    """MD-like trajectory: before evaluation `step` (1-based) every centre moves by
    `amplitude` bohr in a uniformly random direction, cumulatively."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED + cfg.seed_index, 99, step])))
    d = rng.normal(size=orbs.centres.shape)
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    if cfg.general:
        h = cfg.h
        s = np.mod((orbs.centres + amplitude * d) @ np.linalg.inv(h).T, 1.0)
        return dataclasses.replace(orbs, centres=s @ h.T)
    L = np.asarray(cfg.cell)
    return dataclasses.replace(orbs, centres=np.mod(orbs.centres + amplitude * d, L))


def _axis_disp(N: int, L: float, c: float) -> np.ndarray:
    d = np.arange(N, dtype=np.float64) * (L / N) - c
    return d - L * np.floor(d / L + 0.5)


def fill_orbital(cfg_cell: Sequence[float], grid: Sequence[int], centre, expo: float, poly, out: Optional[np.ndarray] = None,
                 normalize: bool = True) -> np.ndarray:
    """phi(r) = exp(-a |d|^2) (1 + c . d), d = minimum-image r - C, on the grid
    [N3, N2, N1] (x fastest), normalized to dV sum phi^2 = 1."""
    N1, N2, N3 = grid
    dx = _axis_disp(N1, cfg_cell[0], centre[0])
    dy = _axis_disp(N2, cfg_cell[1], centre[1])
    dz = _axis_disp(N3, cfg_cell[2], centre[2])
    ex, ey, ez = np.exp(-expo * dx * dx), np.exp(-expo * dy * dy), np.exp(-expo * dz * dz)
    if out is None:
        out = np.empty((N3, N2, N1), dtype=np.float64)
    g = (ez[:, None, None] * ey[None, :, None]) * ex[None, None, :]
    lin = 1.0 + poly[2] * dz[:, None, None] + poly[1] * dy[None, :, None] + poly[0] * dx[None, None, :]
    np.multiply(g, lin, out=out)
    if normalize:
        dV = float(np.prod(cfg_cell)) / float(N1 * N2 * N3)
        out *= 1.0 / math.sqrt(dV * float(np.vdot(out, out)))
    return out


def fill_orbital_cell(h, grid: Sequence[int], centre, expo: float, poly, out: Optional[np.ndarray] = None) -> np.ndarray:
    """fill_orbital for a general cell h (columns L_al): grid point n sits at
    r = h (n / N); d = h (s - floor(s + 1/2)) with s = h^-1 (r - C)."""
    h = np.asarray(h, dtype=np.float64)
    hinv = np.linalg.inv(h)
    N1, N2, N3 = grid
    if out is None:
        out = np.empty((N3, N2, N1), dtype=np.float64)
    n1 = np.arange(N1, dtype=np.float64) / N1
    n2 = np.arange(N2, dtype=np.float64) / N2
    c = np.asarray(centre, dtype=np.float64)
    for k in range(N3):
        f = np.stack(np.meshgrid(n1, n2, indexing="xy"), -1).reshape(-1, 2)   # (x fastest within y)
        fr = np.concatenate([f, np.full((f.shape[0], 1), k / N3)], 1)
        s = (fr @ h.T - c) @ hinv.T
        s -= np.floor(s + 0.5)
        d = s @ h.T
        val = np.exp(-expo * np.sum(d * d, 1)) * (1.0 + d @ np.asarray(poly, dtype=np.float64))
        out[k] = val.reshape(N2, N1)
    dV = abs(float(np.linalg.det(h))) / float(N1 * N2 * N3)
    out *= 1.0 / math.sqrt(dV * float(np.vdot(out, out)))
    return out


def fill_orbitals(cfg: Config, orbs: OrbitalSet, dtype=np.float64, subset: Optional[Sequence[int]] = None) -> np.ndarray:
    idx = range(cfg.n_orb) if subset is None else list(subset)
    N1, N2, N3 = cfg.grid
    arr = np.empty((len(idx), N3, N2, N1), dtype=dtype)
    if cfg.general:
        for k, i in enumerate(idx):
            arr[k] = fill_orbital_cell(cfg.h, cfg.grid, orbs.centres[i], orbs.expo[i], orbs.poly[i])
        return arr
    tmp = np.empty((N3, N2, N1), dtype=np.float64) if dtype != np.float64 else None
    for k, i in enumerate(idx):
        if tmp is None:
            fill_orbital(cfg.cell, cfg.grid, orbs.centres[i], orbs.expo[i], orbs.poly[i], out=arr[k])
        else:
            fill_orbital(cfg.cell, cfg.grid, orbs.centres[i], orbs.expo[i], orbs.poly[i], out=tmp)
            arr[k] = tmp
    return arr


def fill_orbitals_device(cfg: Config, orbs: OrbitalSet, device, dtype=None, out=None, subset=None):
    """fill_orbitals on a GPU with torch, for sets too large to build on the host
    and ship (58 GB of FP64 orbitals for the 256-molecule set).  Same formula,
    same order of the elementwise operations, FP64 arithmetic; the norm is a
    device reduction, so values agree with the host generator to rounding.
    Returns a [n, N3, N2, N1] tensor (or fills `out`)."""
    import torch
    if dtype is None:
        dtype = torch.float32 if cfg.orb_dtype == "f32" else torch.float64
    idx = range(cfg.n_orb) if subset is None else list(subset)
    N1, N2, N3 = cfg.grid
    if out is None:
        out = torch.empty((len(idx), N3, N2, N1), dtype=dtype, device=device)
    if cfg.general:
        # general cell: the fill_orbital_cell formula over the whole grid at once
        h = torch.tensor(cfg.h, dtype=torch.float64, device=device)
        hinv = torch.linalg.inv(h)
        dVg = cfg.dV
        g3, g2, g1 = torch.meshgrid(torch.arange(N3, dtype=torch.float64, device=device) / N3,
                                    torch.arange(N2, dtype=torch.float64, device=device) / N2,
                                    torch.arange(N1, dtype=torch.float64, device=device) / N1, indexing="ij")
        r0 = torch.stack([g1, g2, g3], -1).reshape(-1, 3) @ h.T   # grid point positions, x fastest
        del g1, g2, g3
        for k, i in enumerate(idx):
            c = torch.tensor(orbs.centres[i], dtype=torch.float64, device=device)
            pc = torch.tensor(orbs.poly[i], dtype=torch.float64, device=device)
            a = float(orbs.expo[i])
            s = (r0 - c) @ hinv.T
            s -= torch.floor(s + 0.5)
            d = s @ h.T
            phi = (torch.exp(-a * (d * d).sum(1)) * (1.0 + d @ pc)).reshape(N3, N2, N1)
            phi *= 1.0 / math.sqrt(dVg * float(torch.dot(phi.reshape(-1), phi.reshape(-1)).item()))
            out[k].copy_(phi)
        return out
    dV = float(np.prod(cfg.cell)) / float(N1 * N2 * N3)

    def axis(N, L, c):
        d = torch.arange(N, dtype=torch.float64, device=device) * (L / N) - c
        return d - L * torch.floor(d / L + 0.5)

    for k, i in enumerate(idx):
        c, a, pc = orbs.centres[i], float(orbs.expo[i]), orbs.poly[i]
        dx, dy, dz = axis(N1, cfg.cell[0], float(c[0])), axis(N2, cfg.cell[1], float(c[1])), axis(N3, cfg.cell[2],
                                                                                                  float(c[2]))
        ex, ey, ez = torch.exp(-a * dx * dx), torch.exp(-a * dy * dy), torch.exp(-a * dz * dz)
        g = (ez[:, None, None] * ey[None, :, None]) * ex[None, None, :]
        lin = 1.0 + float(pc[2]) * dz[:, None, None] + float(pc[1]) * dy[None, :, None] + float(pc[0]) * dx[None, None, :]
        phi = g * lin
        phi *= 1.0 / math.sqrt(dV * float(torch.dot(phi.reshape(-1), phi.reshape(-1)).item()))
        out[k].copy_(phi)
    return out


def custom(key="custom", cell=(12.0, 12.0, 12.0), grid=(48, 48, 48), n_orb=4, R_pair=8.0, R_PE=4.0, R_ME=5.5,
           l_max=6, stencil_n=3, cg_tol=1e-12, expo=(0.9, 1.6), seed_index=17, **kw) -> Config:
    """A small configuration for tests (uniform random centres)."""
    return Config(key, tuple(cell), tuple(grid), n_orb, R_pair, R_PE, R_ME, l_max, stencil_n, cg_tol,
                  expo=tuple(expo), seed_index=seed_index, **kw)
