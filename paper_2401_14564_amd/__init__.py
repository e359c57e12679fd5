"""MI355X-native probe-particle model hot path (arXiv 2401.14564).

Python surface over libppm (include/ppm.h).  PyTorch provides device memory and
the current HIP stream; every computation runs in the library's HIP kernels.

  build_ff(grid, probe, atoms)                 -> ff  [nz, ny, nx, 4] float32
  relaxed_scan(grid, ff, probe, fire, scan, dfp=None, pp=True, fz=True)
                                               -> dict(fz, pp, df)
  df(fz, dz, dfp)                              -> df  [nz-2m, ny, nx] float32
  relaxed_scan_backward(...)                   -> dict(pos, q, R, eps) float64
  AFMStack.apply(pos, q, R, eps, grid, probe, fire, scan, dfp) -> df  (autograd)
  lateral_stiffness(grid, ff, probe, scan, pp) -> [nz, ny, nx, 2] soft-mode stiffness
  build_energy(grid, probe, atoms)             -> E   [nz, ny, nx] float32
  relaxed_scan_tricubic(grid, E, probe, fire, scan, dfp=None, ...) -> as relaxed_scan
  BatchPipeline(molecules, jobs, probe, fire, dfp)   many molecules x probes in
      one force-field launch and one scan launch, replayable as a HIP graph

Parameter objects are read by attribute (see workloads.py for the dataclasses).
Atoms may be given as a workloads.Atoms or as a tuple of device tensors
(pos [n,3], q [n], R [n], eps [n]) in float64.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _lib

__all__ = ["build_ff", "relaxed_scan", "df", "df_half_width", "relaxed_scan_backward",
           "AFMStack", "atoms_to_device", "BatchPipeline", "lateral_stiffness",
           "build_energy", "relaxed_scan_tricubic", "Tuning", "tune_build_ff",
           "tune_relaxed_scan"]


@dataclasses.dataclass
class Tuning:
    """Launch shapes (include/ppm.h, ppm_tuning): ff_nzb = force-field voxels per
    thread along z (0 = 8, or 6), scan_tile = relaxed-scan work-group (0 =
    automatic, 16 or 8), scan_fz_direct = 1: with 8 x 8 work-groups and an fz
    output, Fz goes straight to fz instead of an LDS stage.  Chosen by
    tune_build_ff / tune_relaxed_scan."""
    ff_nzb: int = 0
    scan_tile: int = 0
    scan_fz_direct: int = 0


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _device():
    if not torch.cuda.is_available():
        raise RuntimeError("libppm needs a HIP device (torch.cuda.is_available() is False)")
    return torch.device("cuda")


def _need(t, shape, name, dtype=torch.float32):
    """Raise before any launch unless t is a contiguous tensor of exactly this
    shape and dtype: the C ABI takes bare pointers and cannot check sizes.  That
    it lives on the device is checked when its pointer is taken (_lib.ptr)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    shape = tuple(int(v) for v in shape)
    if tuple(t.shape) != shape:
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {shape}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return t


def _grid_shape(grid, *tail):
    nx, ny, nz = (int(v) for v in grid.n)
    return (nz, ny, nx) + tuple(tail)


def _scan_shape(scan, *tail):
    return (int(scan.nz), int(scan.ny), int(scan.nx)) + tuple(tail)


def _df_shape(scan, dfp):
    m = df_half_width(dfp.A, scan.dz)
    return (max(int(scan.nz) - 2 * m, 0), int(scan.ny), int(scan.nx))


def _check_scan_out(out, scan, dfp):
    if out.get("fz") is not None:
        _need(out["fz"], _scan_shape(scan), "out['fz']")
    if out.get("pp") is not None:
        _need(out["pp"], _scan_shape(scan, 4), "out['pp']")
    if out.get("df") is not None:
        if dfp is None:
            raise ValueError("out['df'] given without frequency-shift parameters")
        _need(out["df"], _df_shape(scan, dfp), "out['df']")


def atoms_to_device(atoms, device=None):
    """(pos, q, R, eps) as contiguous float64 device tensors."""
    device = device or _device()
    if isinstance(atoms, (tuple, list)):
        pos, q, R, eps = atoms
    else:
        pos, q, R, eps = atoms.pos, atoms.q, atoms.R, atoms.eps

    def t(x):
        return torch.as_tensor(x, dtype=torch.float64, device=device).contiguous()
    pos, q, R, eps = t(pos).reshape(-1, 3), t(q).reshape(-1), t(R).reshape(-1), t(eps).reshape(-1)
    n = int(q.numel())
    if pos.shape[0] != n or R.numel() != n or eps.numel() != n:
        raise ValueError(f"atoms: {pos.shape[0]} positions, {n} charges, {R.numel()} radii, "
                         f"{eps.numel()} depths")
    return pos, q, R, eps


def df_half_width(A: float, dz: float) -> int:
    return int(_lib.lib().ppm_df_half_width(float(A), float(dz)))


def build_ff(grid, probe, atoms, out: torch.Tensor | None = None,
             tuning: Tuning | None = None) -> torch.Tensor:
    """Force-field grid (Fx, Fy, Fz, E) [nz, ny, nx, 4], float32, on the device;
    with the brick depth of `tuning` if given."""
    L = _lib.lib()
    pos, q, R, eps = atoms_to_device(atoms)
    nx, ny, nz = (int(v) for v in grid.n)
    if out is None:
        out = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=pos.device)
    _need(out, (nz, ny, nx, 4), "out")
    t = _lib.tuning_struct(tuning)
    st = L.ppm_build_ff_tuned(_lib.grid_struct(grid), _lib.probe_struct(probe), t,
                              int(q.numel()), _lib.ptr(pos), _lib.ptr(q), _lib.ptr(R),
                              _lib.ptr(eps), _lib.ptr(out), _stream())
    _lib.check(st, "ppm_build_ff_tuned")
    return out


def tune_build_ff(grid, probe, atoms, out: torch.Tensor | None = None,
                  tuning: Tuning | None = None):
    """Autotune the force-field brick depth on these inputs (ppm_tune_build_ff:
    each candidate timed on the stream; blocks).  Returns (Tuning, {depth: ms});
    `out` (or a scratch grid) holds a built force field afterwards."""
    L = _lib.lib()
    pos, q, R, eps = atoms_to_device(atoms)
    nx, ny, nz = (int(v) for v in grid.n)
    if out is None:
        out = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=pos.device)
    _need(out, (nz, ny, nx, 4), "out")
    import ctypes as ct
    t = _lib.tuning_struct(tuning or Tuning())
    ms = (ct.c_float * 2)()
    st = L.ppm_tune_build_ff(_lib.grid_struct(grid), _lib.probe_struct(probe), int(q.numel()),
                             _lib.ptr(pos), _lib.ptr(q), _lib.ptr(R), _lib.ptr(eps),
                             _lib.ptr(out), _stream(), t, ms)
    _lib.check(st, "ppm_tune_build_ff")
    return Tuning(t.ff_nzb, t.scan_tile, t.scan_fz_direct), {8: float(ms[0]), 6: float(ms[1])}


def _scan_outputs(grid, ff, scan, dfp, fz, pp, out):
    _need(ff, _grid_shape(grid, 4), "ff")
    dev = ff.device
    nz, ny, nx = int(scan.nz), int(scan.ny), int(scan.nx)
    out = dict(out or {})
    _check_scan_out(out, scan, dfp)
    if fz and "fz" not in out:
        out["fz"] = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    if pp and "pp" not in out:
        out["pp"] = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=dev)
    if dfp is not None and "df" not in out:
        m = df_half_width(dfp.A, scan.dz)
        out["df"] = torch.empty((max(nz - 2 * m, 0), ny, nx), dtype=torch.float32, device=dev)
    return out


def relaxed_scan(grid, ff, probe, fire, scan, dfp=None, fz: bool = True, pp: bool = True,
                 out: dict | None = None, tuning: Tuning | None = None) -> dict:
    """Relaxed scan.  Returns dict with 'fz' [nz,ny,nx] (tip force, eV/A), 'pp'
    [nz,ny,nx,4] (probe displacement from rest and FIRE steps, negative if not
    converged) and 'df' [nz-2m,ny,nx] (Hz, when dfp is given).  `tuning` picks
    the work-group shape (the outputs are the same bits for every shape)."""
    L = _lib.lib()
    out = _scan_outputs(grid, ff, scan, dfp, fz, pp, out)
    st = L.ppm_relaxed_scan_tuned(_lib.grid_struct(grid), _lib.ptr(ff), _lib.probe_struct(probe),
                                  _lib.fire_struct(fire), _lib.scan_struct(scan),
                                  _lib.tuning_struct(tuning), _lib.ptr(out.get("fz")),
                                  _lib.ptr(out.get("pp")),
                                  None if dfp is None else _lib.df_struct(dfp),
                                  _lib.ptr(out.get("df")), _stream())
    _lib.check(st, "ppm_relaxed_scan_tuned")
    return out


def tune_relaxed_scan(grid, ff, probe, fire, scan, dfp=None, fz: bool = True, pp: bool = True,
                      out: dict | None = None, tuning: Tuning | None = None):
    """Autotune the scan's work-group shape for these outputs (ppm_tune_relaxed_scan;
    blocks).  Returns (Tuning, {candidate: ms}, outputs), candidates "16x16",
    "8x8" and, with fz, "8x8 fz direct"."""
    import ctypes as ct
    L = _lib.lib()
    out = _scan_outputs(grid, ff, scan, dfp, fz, pp, out)
    t = _lib.tuning_struct(tuning or Tuning())
    ms = (ct.c_float * 3)()
    st = L.ppm_tune_relaxed_scan(_lib.grid_struct(grid), _lib.ptr(ff), _lib.probe_struct(probe),
                                 _lib.fire_struct(fire), _lib.scan_struct(scan),
                                 _lib.ptr(out.get("fz")), _lib.ptr(out.get("pp")),
                                 None if dfp is None else _lib.df_struct(dfp),
                                 _lib.ptr(out.get("df")), _stream(), t, ms)
    _lib.check(st, "ppm_tune_relaxed_scan")
    cand = {"16x16": float(ms[0]), "8x8": float(ms[1])}
    if out.get("fz") is not None:
        cand["8x8 fz direct"] = float(ms[2])
    return Tuning(t.ff_nzb, t.scan_tile, t.scan_fz_direct), cand, out


def build_energy(grid, probe, atoms, out: torch.Tensor | None = None) -> torch.Tensor:
    """Energy-only grid [nz, ny, nx], float32 (input of the tricubic scan)."""
    L = _lib.lib()
    pos, q, R, eps = atoms_to_device(atoms)
    nx, ny, nz = (int(v) for v in grid.n)
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=pos.device)
    _need(out, (nz, ny, nx), "out")
    st = L.ppm_build_energy(_lib.grid_struct(grid), _lib.probe_struct(probe), int(q.numel()),
                            _lib.ptr(pos), _lib.ptr(q), _lib.ptr(R), _lib.ptr(eps), _lib.ptr(out),
                            _stream())
    _lib.check(st, "ppm_build_energy")
    return out


def relaxed_scan_tricubic(grid, E, probe, fire, scan, dfp=None, fz: bool = True, pp: bool = True,
                          out: dict | None = None) -> dict:
    """Relaxed scan on the tricubic interpolant of the energy grid E; outputs as
    relaxed_scan."""
    L = _lib.lib()
    _need(E, _grid_shape(grid), "E")
    dev = E.device
    nz, ny, nx = int(scan.nz), int(scan.ny), int(scan.nx)
    out = dict(out or {})
    _check_scan_out(out, scan, dfp)
    if fz and "fz" not in out:
        out["fz"] = torch.empty((nz, ny, nx), dtype=torch.float32, device=dev)
    if pp and "pp" not in out:
        out["pp"] = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=dev)
    if dfp is not None and "df" not in out:
        m = df_half_width(dfp.A, scan.dz)
        out["df"] = torch.empty((max(nz - 2 * m, 0), ny, nx), dtype=torch.float32, device=dev)
    st = L.ppm_relaxed_scan_tricubic(_lib.grid_struct(grid), _lib.ptr(E), _lib.probe_struct(probe),
                                     _lib.fire_struct(fire), _lib.scan_struct(scan),
                                     _lib.ptr(out.get("fz")), _lib.ptr(out.get("pp")),
                                     None if dfp is None else _lib.df_struct(dfp),
                                     _lib.ptr(out.get("df")), _stream())
    _lib.check(st, "ppm_relaxed_scan_tricubic")
    return out


def df(fz: torch.Tensor, dz: float, dfp, out: torch.Tensor | None = None) -> torch.Tensor:
    """Frequency shift of an Fz stack [nz, ny, nx] (scan-index order)."""
    L = _lib.lib()
    if fz.dim() != 3:
        raise ValueError(f"fz: expected [nz, ny, nx], got shape {tuple(fz.shape)}")
    nz, ny, nx = (int(v) for v in fz.shape)
    _need(fz, (nz, ny, nx), "fz")
    m = df_half_width(dfp.A, dz)
    if out is None:
        out = torch.empty((max(nz - 2 * m, 0), ny, nx), dtype=torch.float32, device=fz.device)
    _need(out, (max(nz - 2 * m, 0), ny, nx), "out")
    st = L.ppm_df(_lib.ptr(fz), nz, ny, nx, float(dz), _lib.df_struct(dfp),
                  _lib.ptr(out), _stream())
    _lib.check(st, "ppm_df")
    return out


def relaxed_scan_backward(grid, ff, probe, scan, dfp, atoms, pp, grad_df,
                          workspace: torch.Tensor | None = None) -> dict:
    """Gradient of sum(grad_df * df) w.r.t. atom positions, charges, R and eps
    (float64 device tensors)."""
    L = _lib.lib()
    _need(pp, _scan_shape(scan, 4), "pp")
    _need(ff, _grid_shape(grid, 4), "ff")
    if tuple(grad_df.shape) != _df_shape(scan, dfp):
        raise ValueError(f"grad_df: shape {tuple(grad_df.shape)}, expected {_df_shape(scan, dfp)}")
    pos, q, R, eps = atoms_to_device(atoms)
    n = int(q.numel())
    sc = _lib.scan_struct(scan)
    nbytes = int(L.ppm_backward_workspace_bytes(sc, n))
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=ff.device)
    _need(workspace, (workspace.numel(),), "workspace", torch.uint8)
    g = {k: torch.empty(s, dtype=torch.float64, device=ff.device)
         for k, s in (("pos", (n, 3)), ("q", (n,)), ("R", (n,)), ("eps", (n,)))}
    gdf = _need(grad_df.to(torch.float32).contiguous(), _df_shape(scan, dfp), "grad_df")
    st = L.ppm_relaxed_scan_backward(_lib.grid_struct(grid), _lib.ptr(ff), _lib.probe_struct(probe),
                                     sc, _lib.df_struct(dfp), n, _lib.ptr(pos), _lib.ptr(q),
                                     _lib.ptr(R), _lib.ptr(eps), _lib.ptr(pp), _lib.ptr(gdf),
                                     _lib.ptr(g["pos"]), _lib.ptr(g["q"]), _lib.ptr(g["R"]),
                                     _lib.ptr(g["eps"]), _lib.ptr(workspace), workspace.numel(),
                                     _stream())
    _lib.check(st, "ppm_relaxed_scan_backward")
    return g


def lateral_stiffness(grid, ff, probe, scan, pp, out: torch.Tensor | None = None):
    """Two smallest eigenvalues of the symmetric stiffness matrix -dG/dr at every
    relaxed point (eV/A^2), [nz, ny, nx, 2]; NaN where not converged."""
    L = _lib.lib()
    _need(pp, _scan_shape(scan, 4), "pp")
    _need(ff, _grid_shape(grid, 4), "ff")
    if out is None:
        out = torch.empty((int(scan.nz), int(scan.ny), int(scan.nx), 2), dtype=torch.float32,
                          device=ff.device)
    _need(out, _scan_shape(scan, 2), "out")
    st = L.ppm_lateral_stiffness(_lib.grid_struct(grid), _lib.ptr(ff), _lib.probe_struct(probe),
                                 _lib.scan_struct(scan), _lib.ptr(pp), _lib.ptr(out), _stream())
    _lib.check(st, "ppm_lateral_stiffness")
    return out


def tip_density(grid, q_pp: float, q_zz: float, sigma: float,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """Probe charge density [nz, ny, nx] (float32, e/A^3) on the grid's lattice of
    offsets from the probe centre: Gaussian-smeared point charge + d_z2 quadrupole."""
    L = _lib.lib()
    nx, ny, nz = (int(v) for v in grid.n)
    if out is None:
        out = torch.empty((nz, ny, nx), dtype=torch.float32, device=_device())
    _need(out, (nz, ny, nx), "out")
    st = L.ppm_tip_density(_lib.grid_struct(grid), float(q_pp), float(q_zz), float(sigma),
                           _lib.ptr(out), _stream())
    _lib.check(st, "ppm_tip_density")
    return out


def hartree_workspace(grid, device=None) -> torch.Tensor:
    """Workspace buffer for hartree_ff on this grid."""
    nbytes = int(_lib.lib().ppm_hartree_workspace_bytes(_lib.grid_struct(grid)))
    if nbytes == 0:
        _lib.check(_lib.PPM_EUNSUPPORTED, "ppm_hartree_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device or _device())


def hartree_ff(grid, V: torch.Tensor, rho: torch.Tensor, out: torch.Tensor | None = None,
               accumulate: bool = False, workspace: torch.Tensor | None = None) -> torch.Tensor:
    """Energy and force of the probe density rho in the sample potential V (both
    [nz, ny, nx] float32): (Fx, Fy, Fz, E) [nz, ny, nx, 4], written, or added to
    `out` when accumulate is set."""
    L = _lib.lib()
    nx, ny, nz = (int(v) for v in grid.n)
    _need(V, (nz, ny, nx), "V")
    _need(rho, (nz, ny, nx), "rho")
    if out is None:
        if accumulate:
            raise ValueError("accumulate=True needs an existing out grid")
        out = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=V.device)
    _need(out, (nz, ny, nx, 4), "out")
    if workspace is None:
        workspace = hartree_workspace(grid, V.device)
    _need(workspace, (workspace.numel(),), "workspace", torch.uint8)
    st = L.ppm_hartree_ff(_lib.grid_struct(grid), _lib.ptr(V), _lib.ptr(rho), int(accumulate),
                          _lib.ptr(out), _lib.ptr(workspace), workspace.numel(), _stream())
    _lib.check(st, "ppm_hartree_ff")
    return out


class AFMStack(torch.autograd.Function):
    """df = AFMStack.apply(pos, q, R, eps, grid, probe, fire, scan, dfp)

    Forward: force-field grid -> relaxed scan -> frequency shift (all HIP).
    Backward: implicit adjoint of the relaxed equilibria (ppm_relaxed_scan_backward)."""

    @staticmethod
    def forward(ctx, pos, q, R, eps, grid, probe, fire, scan, dfp):
        atoms = (pos.detach(), q.detach(), R.detach(), eps.detach())
        ff = build_ff(grid, probe, atoms)
        res = relaxed_scan(grid, ff, probe, fire, scan, dfp=dfp, fz=False, pp=True)
        ctx.save_for_backward(pos.detach(), q.detach(), R.detach(), eps.detach(), ff, res["pp"])
        ctx.params = (grid, probe, scan, dfp)
        return res["df"]

    @staticmethod
    def backward(ctx, grad_df):
        pos, q, R, eps, ff, pp = ctx.saved_tensors
        grid, probe, scan, dfp = ctx.params
        g = relaxed_scan_backward(grid, ff, probe, scan, dfp, (pos, q, R, eps), pp, grad_df)
        return (g["pos"].to(pos.dtype), g["q"].to(q.dtype), g["R"].to(R.dtype),
                g["eps"].to(eps.dtype), None, None, None, None, None)


class BatchPipeline:
    """Force fields of many molecules and scans of many (molecule, probe) jobs,
    one launch per stage (ppm_batch_build_ff, ppm_batch_relaxed_scan).

    molecules: list of (atoms, grid); jobs: list of (molecule index, probe, scan).
    The force fields are built with `probe`'s LJ parameters and charge; every
    job's probe must share them (its springs may differ).  ff_nzb: the brick
    depth of every molecule's build (0 = 8, or 6; BatchPipeline.tuned picks it
    with the autotuner); a molecule's grid equals the single build_ff with the
    same depth bit for bit.  Tables, atoms and arenas are allocated once here;
    run() only launches, so it can be captured with capture() and replayed
    with replay()."""

    @classmethod
    def tuned(cls, molecules, jobs, probe, fire, dfp, keep_fz: bool = False, device=None):
        """A pipeline whose force-field brick depth is chosen by the autotuner
        (ppm_tune_build_ff) on the batch's largest molecule with this probe;
        the timings are kept in .tuning_ms."""
        big = max(range(len(molecules)), key=lambda i: int(np.prod(molecules[i][1].n)) *
                  max(int(molecules[i][0].n), 1))
        atoms, grid = molecules[big]
        t, ms = tune_build_ff(grid, probe, atoms)
        bp = cls(molecules, jobs, probe, fire, dfp, keep_fz=keep_fz, device=device,
                 ff_nzb=t.ff_nzb)
        bp.tuning_ms = ms
        return bp

    def __init__(self, molecules, jobs, probe, fire, dfp, keep_fz: bool = False, device=None,
                 ff_nzb: int = 0):
        import ctypes as ct
        L = _lib.lib()
        dev = device or _device()
        self.n_mol, self.n_jobs = len(molecules), len(jobs)
        self.ff_nzb = int(ff_nzb)
        self.mols = (_lib.BatchMol * self.n_mol)()
        begin = 0
        pos, q, R, eps = [], [], [], []
        for i, (atoms, grid) in enumerate(molecules):
            self.mols[i].grid = _lib.grid_struct(grid)
            self.mols[i].atom_begin = begin
            self.mols[i].n_atoms = int(atoms.n)
            self.mols[i].ff_nzb = self.ff_nzb
            begin += int(atoms.n)
            pos.append(torch.as_tensor(atoms.pos, dtype=torch.float64).reshape(-1, 3))
            q.append(torch.as_tensor(atoms.q, dtype=torch.float64))
            R.append(torch.as_tensor(atoms.R, dtype=torch.float64))
            eps.append(torch.as_tensor(atoms.eps, dtype=torch.float64))
        self.jobs = (_lib.BatchScan * self.n_jobs)()
        for j, (mi, pr, sc) in enumerate(jobs):
            mine = (pr.R_pp, pr.eps_pp, pr.q_pp, float(getattr(pr, "q_zz", 0.0)))
            built = (probe.R_pp, probe.eps_pp, probe.q_pp, float(getattr(probe, "q_zz", 0.0)))
            if mine != built:
                raise ValueError(f"job {j}: probe LJ parameters and charges {mine} differ from "
                                 f"those the force fields are built with {built}")
            self.jobs[j].probe = _lib.probe_struct(pr)
            self.jobs[j].scan = _lib.scan_struct(sc)
            self.jobs[j].mol = int(mi)
        self.dfp = None if dfp is None else _lib.df_struct(dfp)
        totals = (ct.c_int64 * 5)()
        _lib.check(L.ppm_batch_plan(self.n_mol, self.mols, self.n_jobs, self.jobs, self.dfp,
                                    totals), "ppm_batch_plan")
        self.totals = [int(v) for v in totals]
        self.mols_dev = torch.frombuffer(bytearray(bytes(self.mols)), dtype=torch.uint8).to(dev)
        self.jobs_dev = (torch.frombuffer(bytearray(bytes(self.jobs)), dtype=torch.uint8).to(dev)
                         if self.n_jobs else torch.empty(0, dtype=torch.uint8, device=dev))
        self.pos = torch.cat(pos).contiguous().to(dev)
        self.q = torch.cat(q).contiguous().to(dev)
        self.R = torch.cat(R).contiguous().to(dev)
        self.eps = torch.cat(eps).contiguous().to(dev)
        self.ff = torch.empty((self.totals[0], 4), dtype=torch.float32, device=dev)
        self.fz = (torch.empty(self.totals[2], dtype=torch.float32, device=dev)
                   if keep_fz or dfp is None else None)
        self.df = (torch.empty(self.totals[3], dtype=torch.float32, device=dev)
                   if dfp is not None else None)
        self.probe = _lib.probe_struct(probe)
        self.fire = _lib.fire_struct(fire)
        self.m = 0 if dfp is None or not jobs else df_half_width(dfp.A, jobs[0][2].dz)
        self.graph = None

    def build_ff(self):
        L = _lib.lib()
        st = L.ppm_batch_build_ff(self.n_mol, self.mols, _lib.ptr(self.mols_dev), self.probe,
                                  _lib.ptr(self.pos), _lib.ptr(self.q), _lib.ptr(self.R),
                                  _lib.ptr(self.eps), _lib.ptr(self.ff), _stream())
        _lib.check(st, "ppm_batch_build_ff")

    def scan(self):
        if self.n_jobs == 0:             # a batch of force fields only
            return
        L = _lib.lib()
        st = L.ppm_batch_relaxed_scan(self.n_mol, self.mols, _lib.ptr(self.mols_dev), self.n_jobs,
                                      self.jobs, _lib.ptr(self.jobs_dev), self.fire, self.dfp,
                                      _lib.ptr(self.ff), _lib.ptr(self.fz), _lib.ptr(self.df),
                                      _stream())
        _lib.check(st, "ppm_batch_relaxed_scan")

    def run(self):
        self.build_ff()
        self.scan()

    def capture(self):
        """Record run() into a HIP graph (torch.cuda.CUDAGraph)."""
        self.run()                       # warm up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        self.graph.replay()

    # views into the arenas ------------------------------------------------
    def ff_grid(self, i):
        M = self.mols[i]
        n = M.grid.n
        v = int(n[0]) * int(n[1]) * int(n[2])
        return self.ff[M.ff_offset:M.ff_offset + v].view(int(n[2]), int(n[1]), int(n[0]), 4)

    def df_stack(self, j):
        J = self.jobs[j]
        nz, ny, nx = J.scan.nz - 2 * self.m, J.scan.ny, J.scan.nx
        return self.df[J.df_offset:J.df_offset + nz * ny * nx].view(nz, ny, nx)

    def fz_stack(self, j):
        J = self.jobs[j]
        nz, ny, nx = J.scan.nz, J.scan.ny, J.scan.nx
        return self.fz[J.fz_offset:J.fz_offset + nz * ny * nx].view(nz, ny, nx)
