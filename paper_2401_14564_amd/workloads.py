"""Seeded synthetic inputs for the probe-particle hot path.

This module only *creates inputs*: atom positions, types, charges, LJ parameters,
grid geometry, probe, FIRE, scan and frequency-shift settings.  It holds none of
the method's arithmetic (no mixing rules, no forces, no interpolation, no
quadrature), so both the HIP path and the FP64 oracle can read it without
sharing any computation.

Workload shapes follow the paper's stated ranges: samples of tens to hundreds
of atoms (Sec. 5.1.1), grids of 0.1-0.2 A spacing over ~20 A cells giving
1-10 M points (Sec. 5.1.1), image stacks of order 200x200x20 (Sec. 4.3) and a
CO-like probe with lateral stiffness 0.24-0.25 N/m (Sec. 2.1).  The paper's own
molecules and DFT data are not available; these seeded molecules stand in for
them.

Units: positions in Angstrom, energies in eV, charges in e, spring constants in
eV/A^2 (converted from N/m below), cantilever stiffness in N/m, f0 in Hz.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Tuple

import numpy as np

SEED_BASE = 240114564

# 1 N/m expressed in eV/A^2 (exact SI: 1 eV/A^2 = 16.02176634 N/m).  Used only to
# state the probe's spring constants, which the paper quotes in N/m, in the
# internal unit system.
N_PER_M = 1.0 / 16.02176634

# Element LJ parameters (R_i [A], e_i [eV]).  C and H are the values the
# workload specification gives; N, O and the substrate "M" are synthetic
# stand-ins (the paper's OPLS table is not reproduced here).
ELEMENTS = {
    "C": (1.90, 0.0027),
    "H": (1.49, 0.00068),
    "N": (1.80, 0.0030),
    "O": (1.75, 0.0040),
    "M": (2.00, 0.0100),
}


@dataclass
class Atoms:
    pos: np.ndarray      # (n, 3) float64, A
    q: np.ndarray        # (n,) float64, e
    R: np.ndarray        # (n,) float64, A   (element LJ radius R_i)
    eps: np.ndarray      # (n,) float64, eV  (element LJ depth e_i)
    types: List[str] = field(default_factory=list)

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def subset(self, idx) -> "Atoms":
        idx = np.asarray(idx)
        return Atoms(self.pos[idx].copy(), self.q[idx].copy(), self.R[idx].copy(),
                     self.eps[idx].copy(), [self.types[i] for i in idx])

    def copy(self) -> "Atoms":
        return Atoms(self.pos.copy(), self.q.copy(), self.R.copy(), self.eps.copy(),
                     list(self.types))


@dataclass
class Grid:
    origin: Tuple[float, float, float]   # position of voxel (0,0,0), A
    step: Tuple[float, float, float]     # voxel spacing, A
    n: Tuple[int, int, int]              # (nx, ny, nz)
    periodic_xy: int = 0                 # 1: minimum image in x,y with L = n*step
    cutoff: float = 0.0                  # A, pair cutoff used when periodic_xy

    @property
    def nvox(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclass
class Probe:
    R_pp: float = 1.66                   # A
    eps_pp: float = 0.0091               # eV
    q_pp: float = -0.05                  # e
    k_lat: Tuple[float, float] = (0.25 * N_PER_M, 0.25 * N_PER_M)   # eV/A^2
    k_rad: float = 20.0 * N_PER_M        # eV/A^2
    d0: Tuple[float, float, float] = (0.0, 0.0, -4.0)               # A
    q_zz: float = 0.0                    # e A^2, quadrupolar (d_z2) probe charge


@dataclass
class Fire:
    dt0: float = 0.1
    dt_max: float = 1.0                  # 10 dt0, the ratio Bitzek et al. recommend
    f_inc: float = 1.1
    f_dec: float = 0.5
    alpha0: float = 0.1
    f_alpha: float = 0.99
    mass: float = 1.0
    f_conv: float = 1e-4                 # eV/A, Euclidean norm of the net force
    n_min: int = 5
    max_iter: int = 1000


@dataclass
class Scan:
    x0: float
    y0: float
    dx: float
    dy: float
    nx: int
    ny: int
    z_top: float                         # anchor height of scan index 0 (highest)
    dz: float                            # anchor height decreases by dz per index
    nz: int

    @property
    def n_eq(self) -> int:
        return self.nx * self.ny * self.nz


@dataclass
class DfParams:
    A: float = 1.0                       # peak-to-peak amplitude, A
    f0: float = 30300.0                  # Hz
    k_cant: float = 1800.0               # N/m


@dataclass
class Workload:
    name: str
    atoms: Atoms
    grid: Grid
    probe: Probe
    fire: Fire
    scan: Scan
    df: DfParams

    def with_fire(self, **kw) -> "Workload":
        return replace(self, fire=replace(self.fire, **kw))


def _rng(offset: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + offset)


def _place_planar(rng: np.random.Generator, n: int, side: float, center, z_sigma: float,
                  min_sep: float = 1.1, max_tries: int = 200000) -> np.ndarray:
    """Random sequential placement of n points in a side x side square patch
    with a minimum pairwise separation (rejection sampling)."""
    pts = np.zeros((n, 3))
    k = 0
    tries = 0
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"could not place {n} atoms in a {side} A patch")
        p = np.array([center[0] + (rng.random() - 0.5) * side,
                      center[1] + (rng.random() - 0.5) * side,
                      center[2] + (rng.normal(0.0, z_sigma) if z_sigma > 0 else 0.0)])
        if k and np.min(np.sum((pts[:k] - p) ** 2, axis=1)) < min_sep * min_sep:
            continue
        pts[k] = p
        k += 1
    return pts


def _type_counts(n: int) -> List[str]:
    """Organic-like composition 50% C, 33% H, remainder split N/O."""
    nc = n // 2
    nh = n // 3
    rest = n - nc - nh
    nn = rest // 2
    no = rest - nn
    return ["C"] * nc + ["H"] * nh + ["N"] * nn + ["O"] * no


def make_molecule(rng: np.random.Generator, types: List[str], side: float, center,
                  z_sigma: float, q_max: float) -> Atoms:
    n = len(types)
    pos = _place_planar(rng, n, side, center, z_sigma)
    perm = rng.permutation(n)
    types = [types[i] for i in perm]
    q = rng.uniform(-q_max, q_max, size=n)
    q = q - q.mean()                      # zero net charge
    R = np.array([ELEMENTS[t][0] for t in types], dtype=np.float64)
    eps = np.array([ELEMENTS[t][1] for t in types], dtype=np.float64)
    return Atoms(pos, q, R, eps, types)


def config0() -> Workload:
    """Plain method, tiny: 12-atom planar molecule, 160x160x200 grid, 64x64x40 scan."""
    rng = _rng(0)
    atoms = make_molecule(rng, ["C"] * 6 + ["H"] * 6, 6.0, (8.0, 8.0, 0.0), 0.0, 0.2)
    grid = Grid((0.0, 0.0, -4.0), (0.1, 0.1, 0.1), (160, 160, 200))
    scan = Scan(4.8, 4.8, 0.1, 0.1, 64, 64, 11.0, 0.1, 40)
    return Workload("C0: 12 atoms, grid 160x160x200, scan 64x64x40", atoms, grid,
                    Probe(), Fire(), scan, DfParams())


def config1() -> Workload:
    """Plain method, paper scale: 60 atoms, 240^3 grid, 240x240x100 scan."""
    rng = _rng(1)
    types = ["C"] * 30 + ["H"] * 20 + ["N"] * 5 + ["O"] * 5
    atoms = make_molecule(rng, types, 12.0, (12.0, 12.0, 0.0), 0.3, 0.3)
    grid = Grid((0.0, 0.0, -4.0), (0.1, 0.1, 0.1), (240, 240, 240))
    scan = Scan(0.0, 0.0, 0.1, 0.1, 240, 240, 16.9, 0.1, 100)
    return Workload("C1: 60 atoms, grid 240^3, scan 240x240x100", atoms, grid,
                    Probe(), Fire(), scan, DfParams())


def config2() -> Workload:
    """Large sample: 400-atom flake on a 1,200-atom two-layer slab, periodic in xy,
    12 A cutoff, grid 400x400x300, scan 400x400x120."""
    rng = _rng(2)
    ax, ay = 2.0, 40.0 / 15.0
    slab = []
    for layer, (z, sx, sy) in enumerate([(0.0, 0.0, 0.0), (-2.0, ax / 2, ay / 6)]):
        for i in range(20):
            for j in range(15):
                for (bx, by) in [(0.0, 0.0), (ax / 2, ay / 2)]:
                    slab.append(((i * ax + bx + sx) % 40.0, (j * ay + by + sy) % 40.0, z))
    slab = np.array(slab)
    ns = slab.shape[0]
    flake = make_molecule(rng, _type_counts(400), 31.0, (20.0, 20.0, 3.0), 0.3, 0.3)
    pos = np.concatenate([slab, flake.pos])
    q = np.concatenate([np.zeros(ns), flake.q])
    R = np.concatenate([np.full(ns, ELEMENTS["M"][0]), flake.R])
    eps = np.concatenate([np.full(ns, ELEMENTS["M"][1]), flake.eps])
    atoms = Atoms(pos, q, R, eps, ["M"] * ns + flake.types)
    grid = Grid((0.0, 0.0, -5.0), (0.1, 0.1, 0.1), (400, 400, 300), 1, 12.0)
    scan = Scan(0.0, 0.0, 0.1, 0.1, 400, 400, 22.0, 0.1, 120)
    return Workload("C2: 1600 atoms periodic, grid 400x400x300, scan 400x400x120",
                    atoms, grid, Probe(), Fire(), scan, DfParams())


C3_K_LAT_N_PER_M = (0.15, 0.25, 0.5)


def config3_molecule(i: int) -> Workload:
    """Molecule i of the batching set: N ~ U{10..120} atoms, cell fitted with a
    5 A margin, 0.1 A grid, 128x128 tips spanning the cell, 20 heights."""
    rng = np.random.default_rng(SEED_BASE + 3000 + i)
    n = int(rng.integers(10, 121))
    side = math.sqrt(2.4 * n)
    atoms = make_molecule(rng, _type_counts(n), side, (0.0, 0.0, 0.0), 0.3, 0.3)
    h = 0.1
    lo = atoms.pos.min(axis=0) - 5.0
    hi = atoms.pos.max(axis=0) + 5.0
    hi[2] = max(hi[2], 4.9 + 2.0)
    # snap the cell origin to the voxel lattice and round the extent up
    origin = np.floor(lo / h) * h
    nvec = np.ceil((hi - origin) / h).astype(int) + 1
    grid = Grid(tuple(float(v) for v in origin), (h, h, h), tuple(int(v) for v in nvec))
    Lx, Ly = nvec[0] * h, nvec[1] * h
    scan = Scan(float(origin[0]), float(origin[1]), Lx / 128, Ly / 128, 128, 128,
                8.9, 0.1, 20)
    return Workload(f"C3[{i}]: {n} atoms", atoms, grid, Probe(), Fire(), scan, DfParams())


def config3(n_mol: int = 256) -> List[Workload]:
    return [config3_molecule(i) for i in range(n_mol)]


def config4() -> Tuple[Workload, Atoms]:
    """Differentiation: the C1 molecule and grid, a centred 128x128 tip window at
    0.1 A over 30 heights (20 frequency-shift outputs), and a target molecule
    whose positions carry N(0, 0.1 A) noise."""
    w1 = config1()
    scan = Scan(12.0 - 6.4, 12.0 - 6.4, 0.1, 0.1, 128, 128, 9.9, 0.1, 30)
    w = replace(w1, name="C4: C1 molecule, scan 128x128x30", scan=scan)
    rng = _rng(4001)
    target = w.atoms.copy()
    target.pos = target.pos + rng.normal(0.0, 0.1, size=target.pos.shape)
    return w, target


# Grid electrostatics (the Hartree-potential route).  The sample potential of
# a DFT calculation is not available; its stand-in is the periodic potential of
# the atoms' partial charges, each smeared by a Gaussian of width HARTREE_SIGMA.
# The probe density is a Gaussian of width TIP_SIGMA carrying the probe's
# point charge and d_z2 quadrupole.
HARTREE_SIGMA = 0.5      # A
TIP_SIGMA = 0.7          # A
KE = 14.3996454784       # eV A / e^2


def hartree_potential(atoms: Atoms, grid: Grid, sigma: float = HARTREE_SIGMA,
                      trunc: float = 8.0) -> np.ndarray:
    """Synthetic sample potential V [nz][ny][nx] (eV/e) on the grid's periodic
    cell: the charges are spread as Gaussians (cut at trunc*sigma, wrapped) and
    the Poisson equation is solved in Fourier space (zero mean)."""
    n = np.asarray(grid.n)
    h = np.asarray(grid.step, dtype=np.float64)
    o = np.asarray(grid.origin, dtype=np.float64)
    rho = np.zeros((n[2], n[1], n[0]))
    rc = trunc * sigma
    norm = (2 * np.pi * sigma ** 2) ** -1.5
    for p, q in zip(np.asarray(atoms.pos, dtype=np.float64).reshape(-1, 3), atoms.q):
        if q == 0.0:
            continue
        ax = []
        for c in range(3):
            u = (p[c] - o[c]) / h[c]
            i = np.arange(int(np.floor(u - rc / h[c])), int(np.ceil(u + rc / h[c])) + 1)
            ax.append((i % n[c], (i - u) * h[c]))
        (ix, dx), (iy, dy), (iz, dz) = ax
        r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        np.add.at(rho, (iz[:, None, None], iy[None, :, None], ix[None, None, :]),
                  q * norm * np.exp(-r2 / (2 * sigma ** 2)))
    k2 = 0.0
    for c, ax_shape in ((0, (1, 1, -1)), (1, (1, -1, 1)), (2, (-1, 1, 1))):
        m = np.arange(n[c])
        m = np.where(2 * m < n[c], m, m - n[c])
        k2 = k2 + ((2 * np.pi * m / (n[c] * h[c])) ** 2).reshape(ax_shape)
    rk = np.fft.fftn(rho)
    with np.errstate(divide="ignore", invalid="ignore"):
        vk = np.where(k2 > 0, 4 * np.pi * KE * rk / np.where(k2 > 0, k2, 1.0), 0.0)
    return np.real(np.fft.ifftn(vk))


def parity_fire(fire: Fire, f_conv: float = 1e-7, max_iter: int = 20000) -> Fire:
    """FIRE settings for parity runs: a tight convergence threshold so that the
    remaining residual maps to position errors far below the tolerance."""
    return replace(fire, f_conv=f_conv, max_iter=max_iter)


def random_atoms(rng: np.random.Generator, n: int, box_lo, box_hi, q_max=0.3,
                 types=None) -> Atoms:
    """Unconstrained random atoms in a box (for small tests)."""
    if types is None:
        types = [list(ELEMENTS)[i % 4] for i in range(n)]
    pos = rng.uniform(box_lo, box_hi, size=(n, 3))
    q = rng.uniform(-q_max, q_max, size=n)
    R = np.array([ELEMENTS[t][0] for t in types])
    eps = np.array([ELEMENTS[t][1] for t in types])
    return Atoms(pos, q, R, eps, list(types))
