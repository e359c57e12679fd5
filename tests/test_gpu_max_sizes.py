"""Maximum sizes.  The largest force-field grid the ABI accepts (just under 2^31
voxels, 34 GB) is built and checked voxel by voxel against the FP64 oracle; the
scans' 64-bit addressing (grids of 4 GiB and more) is checked on an affine sample
force (trilinear) and a quadratic potential (tricubic), which the interpolants
reproduce exactly, so every relaxed position is the root of the analytic force
balance (Eq. 1), found here by an independent Newton iteration; so is the switch
to 64-bit addressing for planes of 2^24 voxels and more."""
import numpy as np
import pytest
import torch

import oracle as orc
import paper_2401_14564_amd as ppm
from paper_2401_14564_amd import workloads as W
from parity import check_ff

pytestmark = pytest.mark.gpu


def test_ff_build_on_the_largest_grid():
    n = (2048, 1024, 1023)                      # 2,145,386,496 voxels < 2^31
    grid = W.Grid((0.0, 0.0, -2.0), (0.1, 0.1, 0.1), n)
    rng = np.random.default_rng(41)
    atoms = W.random_atoms(rng, 3, [20.0, 20.0, 0.0], [180.0, 80.0, 1.0])
    got = ppm.build_ff(grid, W.Probe(), atoms)
    idx = np.stack([rng.integers(0, n[0], 600), rng.integers(0, n[1], 600),
                    rng.integers(0, n[2], 600)], axis=1)
    idx = np.concatenate([idx, [[0, 0, 0], [n[0] - 1, n[1] - 1, n[2] - 1], [n[0] - 1, 0, n[2] - 1],
                                [0, n[1] - 1, 0]]]).astype(np.int32)
    it = torch.as_tensor(idx, device=got.device, dtype=torch.long)
    sel = got[it[:, 2], it[:, 1], it[:, 0]].cpu().numpy()
    del got, it
    torch.cuda.empty_cache()
    ref, sc = orc.ff_voxels(grid, W.Probe(), atoms, idx)
    info = check_ff(sel, ref, sc, "largest grid")
    print("largest grid", info, flush=True)


def _newton(anchor, probe, Amat, b, r0):
    R0 = np.linalg.norm(probe.d0)
    d0 = np.array(probe.d0)
    k = np.array([probe.k_lat[0], probe.k_lat[1], 0.0])
    r = np.array(r0, float)
    for _ in range(60):
        d = r - anchor
        dn = np.linalg.norm(d)
        G = -probe.k_rad * (dn - R0) * d / dn - k * (d - d0) + Amat @ r + b
        Jt = -probe.k_rad * ((1 - R0 / dn) * np.eye(3) + R0 * np.outer(d, d) / dn ** 3) - np.diag(k)
        r = r - np.linalg.solve(Jt + Amat, G)
    return r


def _affine_ff(n, h, centre, seed=42):
    """float4 grid [nz][ny][nx] holding the affine force A r + b (stable, not
    symmetric), zero energy; returns (ff, A, b)."""
    rng = np.random.default_rng(seed)
    M = rng.normal(size=(3, 3)) * 0.004
    Amat = -(M @ M.T) - 0.003 * np.eye(3) + (M - M.T) * 0.5     # stable, not symmetric
    b = np.array([0.004, -0.003, 0.02]) - Amat @ np.asarray(centre)
    dev = torch.device("cuda")
    ff = torch.empty((n[2], n[1], n[0], 4), dtype=torch.float32, device=dev)
    x = torch.arange(n[0], dtype=torch.float64, device=dev) * h
    y = torch.arange(n[1], dtype=torch.float64, device=dev) * h
    z = torch.arange(n[2], dtype=torch.float64, device=dev) * h
    for c in range(3):
        ff[..., c] = (Amat[c, 0] * x[None, None, :] + Amat[c, 1] * y[None, :, None]
                      + Amat[c, 2] * z[:, None, None] + b[c]).float()
    ff[..., 3] = 0.0
    return ff, Amat, b


def _check_affine_scan(scan, probe, Amat, b, pp, fz, label):
    """Every relaxed point against the Newton root of the analytic balance, and
    the Fz read-out there."""
    assert np.all(pp[..., 3] >= 0)
    worst = 0.0
    for iy in range(scan.ny):
        for ix in range(scan.nx):
            for k in range(scan.nz):
                anchor = np.array([scan.x0 + ix * scan.dx, scan.y0 + iy * scan.dy,
                                   scan.z_top - k * scan.dz])
                rN = _newton(anchor, probe, Amat, b, anchor + np.array(probe.d0))
                rg = anchor + np.array(probe.d0) + pp[k, iy, ix, :3]
                worst = max(worst, float(np.linalg.norm(rg - rN)))
                # read-out: the radial spring's z force at the Newton equilibrium
                d = rN - anchor
                dn = np.linalg.norm(d)
                fzN = probe.k_rad * (dn - np.linalg.norm(probe.d0)) * d[2] / dn
                assert abs(fz[k, iy, ix] - fzN) <= 1e-5, (label, ix, iy, k)
    assert worst <= 1e-4, (label, worst)
    print(label, "worst |dr|", worst, flush=True)


def test_scan_on_a_grid_beyond_4_gib():
    n = (1024, 512, 520)                        # 16 B x 272,629,760 voxels = 4.36 GB
    h = 0.1
    grid = W.Grid((0.0, 0.0, 0.0), (h, h, h), n)
    ff, Amat, b = _affine_ff(n, h, (80.0, 40.0, 30.0))
    probe = W.Probe()
    fire = W.parity_fire(W.Fire())
    scan = W.Scan(79.63, 39.71, 0.13, 0.17, 8, 8, 36.4, 0.1, 12)
    res = ppm.relaxed_scan(grid, ff, probe, fire, scan)
    pp = res["pp"].cpu().numpy()
    fz = res["fz"].cpu().numpy()
    del ff, res
    torch.cuda.empty_cache()
    _check_affine_scan(scan, probe, Amat, b, pp, fz, "wide grid scan")


def test_scan_on_a_grid_with_a_plane_of_2_24_voxels():
    """Below 4 GiB the scans form voxel indices with 24-bit multiplies; a grid
    whose xy plane holds 2^24 voxels or more (here 4097 x 4097 x 3, 0.8 GB) takes
    the 64-bit kernels instead.  Columns next to the far corner, both work-group
    shapes and the Fz-direct route."""
    n = (4097, 4097, 3)
    h = 0.1
    grid = W.Grid((0.0, 0.0, 0.0), (h, h, h), n)
    ff, Amat, b = _affine_ff(n, h, (405.0, 405.0, 0.1))
    probe = W.Probe()
    fire = W.parity_fire(W.Fire())
    scan = W.Scan(404.63, 404.71, 0.13, 0.17, 9, 7, 4.15, 0.05, 2)   # probe 0.15, 0.10 A
    outs = []
    for t in (None, ppm.Tuning(scan_tile=16), ppm.Tuning(scan_tile=8),
              ppm.Tuning(scan_tile=8, scan_fz_direct=1)):
        res = ppm.relaxed_scan(grid, ff, probe, fire, scan, tuning=t)
        outs.append({k: v.cpu().numpy() for k, v in res.items()})
    del ff, res
    torch.cuda.empty_cache()
    for o in outs[1:]:
        for k in o:
            assert np.array_equal(o[k], outs[0][k]), k
    _check_affine_scan(scan, probe, Amat, b, outs[0]["pp"], outs[0]["fz"], "2^24-plane scan")


def test_tricubic_scan_on_an_energy_grid_beyond_4_gib():
    """A quadratic potential E = (r-c).S(r-c)/2 + b.(r-c) is reproduced exactly by
    the Catmull-Rom interpolant, so its force -S(r-c) - b is affine and the
    relaxed positions are again the Newton roots; 2^30 voxels or more (4 GiB of
    FP32) take the 64-bit load path."""
    n = (1024, 1024, 1025)                      # 1,074,790,400 voxels > 2^30
    h = 0.1
    grid = W.Grid((0.0, 0.0, 0.0), (h, h, h), n)
    rng = np.random.default_rng(43)
    M = rng.normal(size=(3, 3)) * 0.004
    S = M @ M.T + 0.003 * np.eye(3)                              # symmetric, positive
    c = np.array([60.0, 50.0, 40.0])
    bvec = np.array([-0.004, 0.003, -0.02])
    dev = torch.device("cuda")
    E = torch.empty((n[2], n[1], n[0]), dtype=torch.float32, device=dev)
    dx = torch.arange(n[0], dtype=torch.float64, device=dev) * h - c[0]
    dy = torch.arange(n[1], dtype=torch.float64, device=dev) * h - c[1]
    for iz in range(n[2]):
        dz = iz * h - c[2]
        q = (0.5 * (S[0, 0] * dx[None, :] ** 2 + S[1, 1] * dy[:, None] ** 2 + S[2, 2] * dz * dz)
             + S[0, 1] * dx[None, :] * dy[:, None] + S[0, 2] * dx[None, :] * dz
             + S[1, 2] * dy[:, None] * dz + bvec[0] * dx[None, :] + bvec[1] * dy[:, None]
             + bvec[2] * dz)
        E[iz] = q.float()
    probe = W.Probe()
    fire = W.parity_fire(W.Fire())
    scan = W.Scan(59.63, 49.71, 0.13, 0.17, 8, 8, 46.4, 0.1, 12)
    res = ppm.relaxed_scan_tricubic(grid, E, probe, fire, scan)
    pp = res["pp"].cpu().numpy()
    del E, res
    torch.cuda.empty_cache()
    assert np.all(pp[..., 3] >= 0)
    Amat, b = -S, S @ c - bvec                                   # F = Amat r + b
    worst = 0.0
    for iy in range(scan.ny):
        for ix in range(scan.nx):
            for k in range(scan.nz):
                anchor = np.array([scan.x0 + ix * scan.dx, scan.y0 + iy * scan.dy,
                                   scan.z_top - k * scan.dz])
                rN = _newton(anchor, probe, Amat, b, anchor + np.array(probe.d0))
                rg = anchor + np.array(probe.d0) + pp[k, iy, ix, :3]
                worst = max(worst, float(np.linalg.norm(rg - rN)))
    assert worst <= 1e-4, worst
    print("wide tricubic scan: worst |dr|", worst, flush=True)
