"""FP64 CPU oracle of the probe-particle hot path -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The product library never imports it, and it imports
nothing from the product library: parameter objects are read by attribute
(duck typing), so the seeded input generators can feed both sides.

The arithmetic lives in ppm_oracle.c (plain C, FP64, OpenMP); this module only
marshals NumPy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as ct
import os
import threading

import numpy as np

from . import build as _build

_lib = None
_lock = threading.Lock()

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def _vp(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def lib():
    """Load oracle/liboracle.so, compiling it on first use if it is missing."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_build.LIB) or (
                    os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
                _build.build()
            L = ct.CDLL(_build.LIB)
            vp = ct.c_void_p
            i = ct.c_int
            d = ct.c_double
            L.orc_mix.argtypes = [i, vp, vp, vp, vp, vp, vp, vp, vp]
            L.orc_point.argtypes = [vp, i, vp, vp, vp, vp, vp, vp, vp, vp, vp]
            L.orc_build_ff.argtypes = [vp, vp, vp, i, vp, vp, vp, vp, i, i, vp, vp]
            L.orc_ff_voxels.argtypes = [vp, vp, vp, i, vp, vp, vp, vp, i, vp, vp, vp]
            L.orc_interp.argtypes = [vp, vp, vp, vp, vp, vp]
            L.orc_tip_force.argtypes = [vp, vp, vp, vp, vp]
            L.orc_sym3_min_eig.argtypes = [vp]
            L.orc_sym3_min_eig.restype = d
            L.orc_relaxed_scan.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i, vp, d,
                                           vp, vp, vp, vp, vp]
            L.orc_residual.argtypes = [vp, vp, vp, vp, i, vp, vp, vp, vp]
            L.orc_lateral_stiffness.argtypes = [vp, vp, vp, vp, i, vp, vp, vp]
            L.orc_interp_tricubic.argtypes = [vp, vp, vp, vp, vp, vp, vp]
            L.orc_relaxed_scan_tricubic.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i, vp, d,
                                                    vp, vp, vp, vp, vp]
            L.orc_residual_tricubic.argtypes = [vp, vp, vp, vp, i, vp, vp, vp, vp]
            L.orc_df_m.argtypes = [d, d]
            L.orc_df_m.restype = i
            L.orc_df_weights.argtypes = [d, d, vp]
            L.orc_df_prefactor.argtypes = [d, d, d]
            L.orc_df_prefactor.restype = d
            L.orc_df.argtypes = [vp, i, i, d, d, d, d, vp]
            L.orc_scan_backward.argtypes = [vp, vp, vp, vp, vp, vp, i, vp, vp, vp, d, d, d,
                                            i, vp, vp, vp, vp, vp, vp, vp, vp]
            L.orc_num_threads.restype = i
            L.orc_set_num_threads.argtypes = [i]
            L.orc_tip_density.argtypes = [vp, vp, d, d, d, vp]
            L.orc_correlate.argtypes = [vp, vp, vp, vp, i, vp, vp]
            _lib = L
    return _lib


# ---------------------------------------------------------------- packing --
def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid(grid):
    g = _f64([*grid.origin, *grid.step, float(grid.periodic_xy), float(grid.cutoff)])
    n = np.ascontiguousarray(grid.n, dtype=np.int32)
    return g, n


def _probe(probe):
    return _f64([probe.R_pp, probe.eps_pp, probe.q_pp, probe.k_lat[0], probe.k_lat[1],
                 probe.k_rad, *probe.d0, probe.q_zz])


def _fire(fire):
    f = _f64([fire.dt0, fire.dt_max, fire.f_inc, fire.f_dec, fire.alpha0, fire.f_alpha,
              fire.mass, fire.f_conv])
    fi = np.ascontiguousarray([fire.n_min, fire.max_iter], dtype=np.int32)
    return f, fi


def _scan(scan):
    s = _f64([scan.x0, scan.y0, scan.dx, scan.dy, scan.z_top, scan.dz])
    ns = np.ascontiguousarray([scan.nx, scan.ny, scan.nz], dtype=np.int32)
    return s, ns


def _atoms(atoms):
    pos = _f64(atoms.pos).reshape(-1, 3)
    return pos, _f64(atoms.q), _f64(atoms.R), _f64(atoms.eps)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


# ------------------------------------------------------------- force field --
def mix(atoms, probe):
    """Per-atom mixed parameters (R_iP, e_iP, kq_i, kQ_i)."""
    pos, q, R, eps = _atoms(atoms)
    n = len(q)
    RiP, eiP, kqi, kQi = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_mix(n, _vp(R), _vp(eps), _vp(q), _vp(_probe(probe)), _vp(RiP), _vp(eiP), _vp(kqi),
                  _vp(kQi))
    return RiP, eiP, kqi, kQi


def point_ff(points, atoms, probe, grid):
    """(Fx,Fy,Fz,E) and scale (sum|f_i|, sum|E_i|, rho_min, tie) at arbitrary points."""
    pts = _f64(points).reshape(-1, 3)
    pos, q, R, eps = _atoms(atoms)
    RiP, eiP, kqi, kQi = mix(atoms, probe)
    g, n = _grid(grid)
    out = np.zeros((len(pts), 4))
    sc = np.zeros((len(pts), 4))
    L = lib()
    for k in range(len(pts)):
        L.orc_point(_vp(pts[k]), len(q), _vp(pos), _vp(RiP), _vp(eiP), _vp(kqi), _vp(kQi), _vp(g),
                    _vp(n), _vp(out[k]), _vp(sc[k]))
    return out, sc


def build_ff(grid, probe, atoms, iz0=0, iz1=None, with_scale=False):
    """Force-field grid [iz1-iz0][ny][nx][4] (Fx,Fy,Fz,E), FP64."""
    g, n = _grid(grid)
    if iz1 is None:
        iz1 = int(grid.n[2])
    pos, q, R, eps = _atoms(atoms)
    shape = (iz1 - iz0, int(grid.n[1]), int(grid.n[0]), 4)
    ff = np.zeros(shape)
    sc = np.zeros(shape) if with_scale else None
    lib().orc_build_ff(_vp(g), _vp(n), _vp(_probe(probe)), len(q), _vp(pos), _vp(q), _vp(R),
                       _vp(eps), iz0, iz1, _vp(ff), _vp(sc))
    return (ff, sc) if with_scale else ff


def ff_voxels(grid, probe, atoms, idx, with_scale=True):
    """Force field at voxel indices idx[m][3] = (ix, iy, iz)."""
    g, n = _grid(grid)
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 3)
    pos, q, R, eps = _atoms(atoms)
    out = np.zeros((len(idx), 4))
    sc = np.zeros((len(idx), 4)) if with_scale else None
    lib().orc_ff_voxels(_vp(g), _vp(n), _vp(_probe(probe)), len(q), _vp(pos), _vp(q), _vp(R),
                        _vp(eps), len(idx), _vp(idx), _vp(out), _vp(sc))
    return (out, sc) if with_scale else out


def interp(ff, grid, r, with_jac=False):
    """Trilinear interpolation of (Fx,Fy,Fz) at point r (and its in-cell Jacobian)."""
    g, n = _grid(grid)
    ff = _f64(ff)
    F = np.zeros(3)
    J = np.zeros(9) if with_jac else None
    lib().orc_interp(_vp(ff), _vp(g), _vp(n), _vp(_f64(r)), _vp(F), _vp(J))
    return (F, J.reshape(3, 3)) if with_jac else F


def tip_force(r, anchor, probe, with_jac=False):
    F = np.zeros(3)
    J = np.zeros(9) if with_jac else None
    lib().orc_tip_force(_vp(_f64(r)), _vp(_f64(anchor)), _vp(_probe(probe)), _vp(F), _vp(J))
    return (F, J.reshape(3, 3)) if with_jac else F


def sym3_min_eig(S):
    return float(lib().orc_sym3_min_eig(_vp(_f64(S).reshape(9))))


# -------------------------------------------------------------------- scan --
def all_columns(scan):
    iy, ix = np.meshgrid(np.arange(scan.ny), np.arange(scan.nx), indexing="ij")
    return np.stack([ix.ravel(), iy.ravel()], axis=1).astype(np.int32)


def relaxed_scan(grid, ff, probe, fire, scan, cols=None, polish_tol=0.0, with_lambda=False):
    """Relaxed scan over the tip columns `cols` [ncol][2] = (ix, iy) (default:
    all, row-major in y then x).  Returns dict with arrays indexed [col][k]:
    r (…,3), fz, iters, gnorm, lam (if with_lambda)."""
    g, n = _grid(grid)
    f, fi = _fire(fire)
    s, ns = _scan(scan)
    if cols is None:
        cols = all_columns(scan)
    cols = np.ascontiguousarray(cols, dtype=np.int32).reshape(-1, 2)
    nc, nz = len(cols), scan.nz
    ff = _f64(ff)
    assert ff.shape == (grid.n[2], grid.n[1], grid.n[0], 4)
    r = np.zeros((nc, nz, 3))
    fz = np.zeros((nc, nz))
    it = np.zeros((nc, nz), dtype=np.int32)
    gn = np.zeros((nc, nz))
    lam = np.zeros((nc, nz)) if with_lambda else None
    lib().orc_relaxed_scan(_vp(g), _vp(n), _vp(ff), _vp(_probe(probe)), _vp(f), _vp(fi),
                           _vp(s), _vp(ns), nc, _vp(cols), float(polish_tol), _vp(r), _vp(fz),
                           _vp(it), _vp(gn), _vp(lam))
    out = dict(cols=cols, r=r, fz=fz, iters=it, gnorm=gn)
    if with_lambda:
        out["lam"] = lam
    return out


def residual(grid, ff, probe, anchors, rs, with_lambda=True):
    """|G| (and the stability eigenvalue) at given probe positions."""
    g, n = _grid(grid)
    anchors = _f64(anchors).reshape(-1, 3)
    rs = _f64(rs).reshape(-1, 3)
    m = len(rs)
    gn = np.zeros(m)
    lam = np.zeros(m) if with_lambda else None
    lib().orc_residual(_vp(g), _vp(n), _vp(_f64(ff)), _vp(_probe(probe)), m, _vp(anchors),
                       _vp(rs), _vp(gn), _vp(lam))
    return (gn, lam) if with_lambda else gn


def interp_tricubic(En, grid, r, with_hessian=False):
    """Tricubic (Catmull-Rom) interpolated energy, force -grad E and Hessian of
    the energy grid En [nz][ny][nx] at point r."""
    g, n = _grid(grid)
    En = _f64(En)
    E = np.zeros(1)
    F = np.zeros(3)
    H = np.zeros(9) if with_hessian else None
    lib().orc_interp_tricubic(_vp(En), _vp(g), _vp(n), _vp(_f64(r)), _vp(E), _vp(F), _vp(H))
    return (E[0], F, H.reshape(3, 3)) if with_hessian else (E[0], F)


def relaxed_scan_tricubic(grid, En, probe, fire, scan, cols=None, polish_tol=0.0,
                          with_lambda=False):
    """Relaxed scan on the tricubic potential of the energy grid En [nz][ny][nx];
    same outputs as relaxed_scan."""
    g, n = _grid(grid)
    f, fi = _fire(fire)
    s, ns = _scan(scan)
    if cols is None:
        cols = all_columns(scan)
    cols = np.ascontiguousarray(cols, dtype=np.int32).reshape(-1, 2)
    nc, nz = len(cols), scan.nz
    En = _f64(En)
    assert En.shape == (grid.n[2], grid.n[1], grid.n[0])
    r = np.zeros((nc, nz, 3))
    fz = np.zeros((nc, nz))
    it = np.zeros((nc, nz), dtype=np.int32)
    gn = np.zeros((nc, nz))
    lam = np.zeros((nc, nz)) if with_lambda else None
    lib().orc_relaxed_scan_tricubic(_vp(g), _vp(n), _vp(En), _vp(_probe(probe)), _vp(f), _vp(fi),
                                    _vp(s), _vp(ns), nc, _vp(cols), float(polish_tol), _vp(r),
                                    _vp(fz), _vp(it), _vp(gn), _vp(lam))
    out = dict(cols=cols, r=r, fz=fz, iters=it, gnorm=gn)
    if with_lambda:
        out["lam"] = lam
    return out


def residual_tricubic(grid, En, probe, anchors, rs, with_lambda=True):
    g, n = _grid(grid)
    anchors = _f64(anchors).reshape(-1, 3)
    rs = _f64(rs).reshape(-1, 3)
    m = len(rs)
    gn = np.zeros(m)
    lam = np.zeros(m) if with_lambda else None
    lib().orc_residual_tricubic(_vp(g), _vp(n), _vp(_f64(En)), _vp(_probe(probe)), m,
                                _vp(anchors), _vp(rs), _vp(gn), _vp(lam))
    return (gn, lam) if with_lambda else gn


def lateral_stiffness(grid, ff, probe, anchors, rs):
    """Two smallest eigenvalues of sym(-dG/dr) at probe positions rs (soft modes)."""
    g, n = _grid(grid)
    anchors = _f64(anchors).reshape(-1, 3)
    rs = _f64(rs).reshape(-1, 3)
    out = np.zeros((len(rs), 2))
    lib().orc_lateral_stiffness(_vp(g), _vp(n), _vp(_f64(ff)), _vp(_probe(probe)), len(rs),
                                _vp(anchors), _vp(rs), _vp(out))
    return out


# ---------------------------------------------------------- frequency shift --
def df_m(A, dz) -> int:
    return int(lib().orc_df_m(float(A), float(dz)))


def df_weights(A, dz):
    """Weights w_j, j = -m..m, for physical offsets j*dz."""
    m = df_m(A, dz)
    w = np.zeros(2 * m + 1)
    lib().orc_df_weights(float(A), float(dz), _vp(w))
    return w


def df_prefactor(A, f0, k) -> float:
    return float(lib().orc_df_prefactor(float(A), float(f0), float(k)))


def df(fz, dz, dfp):
    """Frequency shift of an Fz stack [nz][...] in scan-index order."""
    fz = _f64(fz)
    nz = fz.shape[0]
    rest = fz.shape[1:]
    ncol = int(np.prod(rest)) if rest else 1
    m = df_m(dfp.A, dz)
    out = np.zeros((max(nz - 2 * m, 0),) + rest)
    if nz - 2 * m > 0:
        lib().orc_df(_vp(fz), nz, ncol, float(dz), float(dfp.A), float(dfp.f0),
                     float(dfp.k_cant), _vp(out))
    return out


# ----------------------------------------------------------------- adjoint --
def scan_backward(grid, ff, probe, scan, cols, rstar, grad_df, dfp, atoms):
    """FP64 implicit-adjoint gradient of sum(grad_df * df) with respect to atom
    positions, charges, R_i and e_i.  rstar [ncol][nz][3] from relaxed_scan
    (polished), grad_df [nz-2m][ncol]."""
    g, n = _grid(grid)
    s, ns = _scan(scan)
    cols = np.ascontiguousarray(cols, dtype=np.int32).reshape(-1, 2)
    pos, q, R, eps = _atoms(atoms)
    na = len(q)
    gp = np.zeros((na, 3))
    gq, gR, ge = np.zeros(na), np.zeros(na), np.zeros(na)
    lib().orc_scan_backward(_vp(g), _vp(n), _vp(_f64(ff)), _vp(_probe(probe)), _vp(s), _vp(ns),
                            len(cols), _vp(cols), _vp(_f64(rstar)), _vp(_f64(grad_df)),
                            float(dfp.A), float(dfp.f0), float(dfp.k_cant), na, _vp(pos),
                            _vp(q), _vp(R), _vp(eps), _vp(gp), _vp(gq), _vp(gR), _vp(ge))
    return dict(pos=gp, q=gq, R=gR, eps=ge)


# ------------------------------------------------- grid electrostatics --
def tip_density(grid, q_pp, q_zz, sigma):
    """Probe charge density [nz][ny][nx] on the grid's lattice of offsets from the
    probe centre (Gaussian-smeared point charge + d_z2 quadrupole)."""
    g, n = _grid(grid)
    rho = np.zeros((n[2], n[1], n[0]))
    lib().orc_tip_density(_vp(g), _vp(n), float(q_pp), float(q_zz), float(sigma), _vp(rho))
    return rho


def correlate(grid, rho, V, idx=None):
    """E[j] = dV sum_i rho[i] V[i + j] (periodic), at voxels idx[m][3] or everywhere."""
    g, n = _grid(grid)
    rho = _f64(rho)
    V = _f64(V)
    assert rho.shape == V.shape == (n[2], n[1], n[0])
    if idx is None:
        E = np.zeros((n[2], n[1], n[0]))
        lib().orc_correlate(_vp(g), _vp(n), _vp(rho), _vp(V), 0, None, _vp(E))
        return E
    idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, 3)
    E = np.zeros(len(idx))
    lib().orc_correlate(_vp(g), _vp(n), _vp(rho), _vp(V), len(idx), _vp(idx), _vp(E))
    return E


def wavenumbers(n, h):
    """Signed angular wavenumbers of a periodic axis of n points and step h (the
    Nyquist term of an even n is set to zero, so that derivatives of real data
    stay real)."""
    m = np.arange(n)
    m = np.where(2 * m < n, m, m - n).astype(np.float64)
    if n % 2 == 0:
        m[n // 2] = 0.0
    return 2.0 * np.pi * m / (n * h)


def _spectral_gradient(a, grid):
    """d a / d x_c (c = x, y, z) of a periodic grid array a [nz][ny][nx], as the
    derivative of its trigonometric interpolant (numpy FFT)."""
    kx = wavenumbers(grid.n[0], grid.step[0])[None, None, :]
    ky = wavenumbers(grid.n[1], grid.step[1])[None, :, None]
    kz = wavenumbers(grid.n[2], grid.step[2])[:, None, None]
    ak = np.fft.fftn(a)
    return [np.real(np.fft.ifftn(1j * k * ak)) for k in (kx, ky, kz)]


def hartree_ff(grid, rho, V, idx=None):
    """Electrostatic energy of the probe and its force, (Fx, Fy, Fz, E), on the
    whole grid ([nz][ny][nx][4]) or at voxels idx[m][3] ([m][4]).
    E is the cross-correlation of rho with V (direct sum).  F = -grad E is
    taken as the derivative of E's trigonometric interpolant; moving the
    derivative onto the density (summation by parts on the periodic grid),
    F_c = correlate(d rho / d x_c, V), with d rho / d x_c the spectral
    derivative of rho."""
    drho = _spectral_gradient(_f64(rho), grid)
    parts = [correlate(grid, d, V, idx) for d in drho] + [correlate(grid, rho, V, idx)]
    return np.stack(parts, axis=-1)
