"""Shared parity machinery for the GPU tests (imported by tests; not collected).

Tolerances (stated for the workloads, checked element by element):
  * force field: per voxel and component |dF_c| <= 1e-5 * S(v), where S(v) is the
    magnitude sum of every term that enters the sum -- the repulsive and the
    attractive LJ part of each pair and its Coulomb part -- i.e. the scale of the
    rounding error of the sum (from the oracle); the same for E; and
    |dF| / |F| <= 1e-5 wherever the sum is well conditioned, |F| >= S/2 (an n-term
    FP32 sum with condition number S/|F| = k carries up to ~n u k relative error,
    u = 6e-8, so a relative bound on |F| itself is only meaningful for small k);
    for 2 < k <= 10 (S/10 <= |F| < S/2) the relative error grows with k and the
    bound is |dF| / |F| <= 5e-5, i.e. 1e-5 at k = 2 scaled by the tier's
    largest k, 10, over 2 (measured worst on the tiny and paper-scale grids and
    20,000 voxels of the large periodic one: 3.8e-6 at k <= 2, 1.1e-5 for
    2 < k <= 10).
    Voxels closer than 0.5 A to an atom
    (energies of 1e5 eV and more, never visited by the probe) and, with a cutoff,
    voxels with a pair within 1e-3 A^2 of the cutoff sphere (each side applies
    rho^2 < rc^2 in its own precision) are excluded and counted.
  * relaxed probe position: |dr| <= 1e-4 A at graded points.
  * frequency shift: |d df| <= 1e-3 Hz at outputs whose whole stencil is graded.
A relaxed point is graded when the oracle's stability eigenvalue (smallest
eigenvalue of sym(-dG/dr)) is >= 1e-2 eV/A^2, so that the force residual maps to
a position error well inside the tolerance.  Where several equilibria exist
(bistable columns) the scan may legitimately settle in another one: such a
column is accepted from the height where it departs only if every GPU position
from there on is certified by the oracle's force balance, |G_FP64(r_gpu)| <=
2 f_conv + 1e-6 (FIRE's own stopping rule, plus the FP32 rounding of the stored
displacement).  Every ungraded point needs the same certificate.
"""
from __future__ import annotations

import numpy as np

from paper_2401_14564_amd import workloads as W

import oracle as orc

FF_RTOL = 1e-5
FF_RTOL_MID = 5e-5   # |dF|/|F| where S/10 <= |F| < S/2 (condition number 2 to 10)
POS_TOL = 1e-4
DF_TOL = 1e-3
LAM_GRADED = 1e-2


def check_ff(gpu_ff: np.ndarray, ref: np.ndarray, scale: np.ndarray, label: str = ""):
    """gpu_ff, ref, scale: [..., 4]; scale from the oracle (S_F, S_E, rho_min, tie)."""
    gpu = gpu_ff.astype(np.float64)
    excl = scale[..., 2] < 0.5
    excl |= scale[..., 3] <= 1e-3
    ok = ~excl
    dF = np.abs(gpu[..., :3] - ref[..., :3])
    bad_c = (dF > FF_RTOL * scale[..., :1]) & ok[..., None]
    dE = np.abs(gpu[..., 3] - ref[..., 3])
    bad_e = (dE > FF_RTOL * scale[..., 1]) & ok
    Fn = np.linalg.norm(ref[..., :3], axis=-1)
    relall = np.linalg.norm(gpu[..., :3] - ref[..., :3], axis=-1) / np.where(Fn > 0, Fn, 1.0)
    strong = ok & (Fn >= 0.5 * scale[..., 0]) & (Fn > 0)
    mid = ok & (Fn >= 0.1 * scale[..., 0]) & ~strong & (Fn > 0)
    rel = np.where(strong, relall, 0.0)
    rel2 = np.where(mid, relall, 0.0)
    bad_r = rel > FF_RTOL
    bad_r2 = rel2 > FF_RTOL_MID
    assert np.all(np.isfinite(gpu[ok])), f"{label}: non-finite values at graded voxels"
    assert not bad_c.any(), (f"{label}: {bad_c.sum()} component errors, worst "
                             f"{np.max(dF[ok] / np.maximum(scale[ok][:, :1], 1e-300)):.3e}")
    assert not bad_e.any(), f"{label}: {bad_e.sum()} energy errors"
    assert not bad_r.any(), f"{label}: {bad_r.sum()} relative errors, worst {rel.max():.3e}"
    assert not bad_r2.any(), (f"{label}: {bad_r2.sum()} relative errors where S/10 <= |F| < "
                              f"S/2, worst {rel2.max():.3e}")
    wc = np.max(dF[ok] / np.maximum(scale[ok][:, :1], 1e-300)) if ok.any() else 0.0
    we = np.max(dE[ok] / np.maximum(scale[ok][:, 1], 1e-300)) if ok.any() else 0.0
    return dict(n=int(ok.sum()), excluded=int(excl.sum()),
                worst_component_over_S=float(wc), worst_energy_over_S=float(we),
                worst_rel=float(rel.max()) if rel.size else 0.0,
                worst_rel_mid=float(rel2.max()) if rel2.size else 0.0,
                n_strong=int(strong.sum()), n_mid=int(mid.sum()))


def anchors_for(scan, cols):
    cols = np.asarray(cols)
    nz = scan.nz
    ax = scan.x0 + cols[:, 0] * scan.dx
    ay = scan.y0 + cols[:, 1] * scan.dy
    az = scan.z_top - np.arange(nz) * scan.dz
    A = np.zeros((len(cols), nz, 3))
    A[:, :, 0] = ax[:, None]
    A[:, :, 1] = ay[:, None]
    A[:, :, 2] = az[None, :]
    return A


def grade_scan(grid, ff64, probe, fire, scan, cols, ores, gpu_pp, gpu_fz, gpu_df=None, dfp=None,
               max_diverged_frac=0.02, label="", residual=None):
    """Compare the GPU scan (arrays [nz, ny, nx(,4)]) with the oracle result for the
    tip columns `cols` (oracle arrays [col, k]).  `residual` evaluates the oracle's
    force balance at given points (default: trilinear forces from ff64).
    Returns class counts."""
    residual = residual or orc.residual
    cols = np.asarray(cols)
    ix, iy = cols[:, 0], cols[:, 1]
    pp = gpu_pp[:, iy, ix, :].transpose(1, 0, 2).astype(np.float64)     # [col, k, 4]
    fz = gpu_fz[:, iy, ix].T.astype(np.float64)                          # [col, k]
    A = anchors_for(scan, cols)
    r_gpu = A + np.asarray(probe.d0) + pp[..., :3]
    assert np.all(pp[..., 3] >= 0), f"{label}: GPU reports non-converged points"
    dr = np.linalg.norm(r_gpu - ores["r"], axis=-1)
    graded = ores["lam"] >= LAM_GRADED
    nc, nz = dr.shape
    valid = np.ones_like(dr, dtype=bool)          # not in a diverged column segment
    diverged_cols = 0
    # certificate for every GPU point: oracle residual and stability at r_gpu
    gres, glam = residual(grid, ff64, probe, A.reshape(-1, 3), r_gpu.reshape(-1, 3))
    gres = gres.reshape(nc, nz)
    glam = glam.reshape(nc, nz)
    cert = gres <= 2 * fire.f_conv + 1e-6
    for c in range(nc):
        far = np.nonzero(dr[c] > POS_TOL)[0]
        if len(far) == 0:
            continue
        k0 = far[0]
        if cert[c, k0:].all():
            valid[c, k0:] = False
            diverged_cols += 1
    g = graded & valid
    assert np.all(dr[g] <= POS_TOL), (f"{label}: {np.sum(dr[g] > POS_TOL)} graded points off, "
                                      f"worst {dr[g].max():.3e} A")
    ungraded = ~g
    assert np.all(cert[ungraded]), (f"{label}: {np.sum(~cert[ungraded])} uncertified points, "
                                    f"worst residual {gres[ungraded].max():.3e}")
    assert diverged_cols <= max_diverged_frac * nc, f"{label}: {diverged_cols} diverged columns"
    out = dict(points=int(dr.size), graded=int(g.sum()), ungraded=int(ungraded.sum()),
               diverged_cols=diverged_cols, unstable_sym=int(np.sum(glam <= 0)),
               worst_dr=float(dr[g].max()) if g.any() else 0.0,
               worst_dfz=float(np.abs(fz - ores["fz"])[g].max()) if g.any() else 0.0)
    if gpu_df is not None:
        m = orc.df_m(dfp.A, scan.dz)
        odf = orc.df(ores["fz"].T, scan.dz, dfp)                          # [nz-2m, col]
        gdf = gpu_df[:, iy, ix].astype(np.float64)                        # [nz-2m, col]
        win = np.ones_like(odf, dtype=bool)
        for o in range(nz - 2 * m):
            win[o] = g[:, o:o + 2 * m + 1].all(axis=1)
        d = np.abs(gdf - odf)
        assert np.all(d[win] <= DF_TOL), (f"{label}: {np.sum(d[win] > DF_TOL)} df outputs off, "
                                          f"worst {d[win].max():.3e} Hz")
        out.update(df_graded=int(win.sum()), df_total=int(win.size),
                   worst_ddf=float(d[win].max()) if win.any() else 0.0)
    return out


def edge_workload(periodic):
    """Tips over and beyond both x and y edges of the cell (columns from 0.63 A
    before the first voxel to past the last one), probe heights 6 to 3.6 A above
    ten atoms spread over the cell.  Open sample: 9.6 x 9.0 A, charged atoms,
    clamped interpolation.  Periodic sample: 15 x 14 A with a 6.5 A minimum-image
    shifted-force cutoff, charged atoms, wrapped interpolation."""
    rng = np.random.default_rng(31 + periodic)
    h = 0.1
    n = (150, 140, 90) if periodic else (96, 90, 90)
    L = np.array(n[:2]) * h
    atoms = W.random_atoms(rng, 10, [0.3, 0.3, -0.3], [L[0] - 0.3, L[1] - 0.3, 0.3])
    grid = W.Grid((0.0, 0.0, -1.0), (h, h, h), n, periodic, 6.5 if periodic else 0.0)
    dx, dy = ((0.31, 0.30) if periodic else (0.2, 0.2))
    scan = W.Scan(-0.63, -0.52, dx, dy, 52, 50, 10.03, 0.1, 25)
    return W.Workload(f"edges periodic={periodic}", atoms, grid, W.Probe(), W.Fire(), scan,
                      W.DfParams())
