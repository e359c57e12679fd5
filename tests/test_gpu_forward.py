"""GPU parity of the forward path (force-field build, relaxed scan, frequency
shift) against the FP64 oracle, through the C ABI.  Tolerances: see parity.py."""
import numpy as np
import pytest
import torch

import oracle as orc
import paper_2401_14564_amd as ppm
from paper_2401_14564_amd import workloads as W
from parity import DF_TOL, check_ff, edge_workload, grade_scan

pytestmark = pytest.mark.gpu


def _gpu_ff(w):
    ff = ppm.build_ff(w.grid, w.probe, w.atoms)
    torch.cuda.synchronize()
    return ff


@pytest.fixture(scope="module")
def c0():
    w = W.config0()
    ref, sc = orc.build_ff(w.grid, w.probe, w.atoms, with_scale=True)
    return w, ref, sc


# ------------------------------------------------------------------ FF build
@pytest.mark.parametrize("nzb", [0, 6])
def test_ff_c0_full_grid(c0, nzb):
    """Every voxel of the tiny workload, at the default brick depth and at the
    autotuner's other candidate."""
    w, ref, sc = c0
    got = ppm.build_ff(w.grid, w.probe, w.atoms, tuning=ppm.Tuning(ff_nzb=nzb))
    info = check_ff(got.cpu().numpy(), ref, sc, f"C0 depth {nzb}")
    print("C0 ff", nzb, info, flush=True)


def test_ff_c1_full_grid():
    w = W.config1()
    ref, sc = orc.build_ff(w.grid, w.probe, w.atoms, with_scale=True)
    info = check_ff(_gpu_ff(w).cpu().numpy(), ref, sc, "C1")
    print("C1 ff", info, flush=True)


@pytest.mark.parametrize("nzb", [0, 6])
@pytest.mark.parametrize("n,natoms,periodic", [((5, 3, 3), 4, 0), ((67, 9, 13), 300, 0),
                                               ((64, 4, 8), 1, 0), ((2, 2, 2), 3, 0),
                                               ((130, 90, 11), 40, 1), ((130, 90, 17), 300, 1)])
def test_ff_ragged_and_multi_chunk(n, natoms, periodic, nzb):
    """Grids that are not multiples of the brick, more atoms than one LDS chunk,
    a 2x2x2 grid, and periodic cells with a cutoff, at both brick depths."""
    rng = np.random.default_rng(sum(n) + natoms)
    h = 0.1
    L = np.array(n) * h
    atoms = W.random_atoms(rng, natoms, [0, 0, -1.0], [L[0], L[1], 0.0])
    cutoff = 0.5 * min(L[0], L[1]) - 3.5 if periodic else 0.0
    grid = W.Grid((0.0, 0.0, 1.5), (h, h, h), n, periodic, cutoff)
    ref, sc = orc.build_ff(grid, W.Probe(), atoms, with_scale=True)
    got = ppm.build_ff(grid, W.Probe(), atoms, tuning=ppm.Tuning(ff_nzb=nzb)).cpu().numpy()
    check_ff(got, ref, sc, f"grid {n} atoms {natoms} periodic {periodic} depth {nzb}")


def test_ff_zero_atoms_is_zero_field():
    grid = W.Grid((0.0, 0.0, 0.0), (0.1, 0.1, 0.1), (70, 5, 9))
    empty = W.Atoms(np.zeros((0, 3)), np.zeros(0), np.zeros(0), np.zeros(0), [])
    got = ppm.build_ff(grid, W.Probe(), empty).cpu().numpy()
    assert np.all(got == 0.0)


def test_ff_c2_sampled_voxels():
    """Full 400x400x300 periodic grid with 1,600 atoms, checked on 20,000 seeded
    voxels computed one by one by the oracle."""
    w = W.config2()
    got = _gpu_ff(w)
    rng = np.random.default_rng(2002)
    idx = np.stack([rng.integers(0, w.grid.n[0], 20000), rng.integers(0, w.grid.n[1], 20000),
                    rng.integers(0, w.grid.n[2], 20000)], axis=1)
    ref, sc = orc.ff_voxels(w.grid, w.probe, w.atoms, idx)
    it = torch.as_tensor(idx, device=got.device)
    sel = got[it[:, 2], it[:, 1], it[:, 0]].cpu().numpy()
    info = check_ff(sel, ref, sc, "C2 sampled")
    print("C2 ff", info, flush=True)


def test_ff_c2_voxels_next_to_the_slab():
    """2,000 seeded voxels 0.9-1.2 A above the slab's top layer, where one or two
    atoms' repulsion (thousands of eV) meets hundreds of small terms from the
    atoms within the cutoff: the energy's rounding there depends on the order in
    which the kernel adds them."""
    w = W.config2()
    got = _gpu_ff(w)
    rng = np.random.default_rng(2003)
    iz0 = int(round((0.9 - w.grid.origin[2]) / w.grid.step[2]))
    idx = np.stack([rng.integers(0, w.grid.n[0], 2000), rng.integers(0, w.grid.n[1], 2000),
                    rng.integers(iz0, iz0 + 4, 2000)], axis=1)
    ref, sc = orc.ff_voxels(w.grid, w.probe, w.atoms, idx)
    it = torch.as_tensor(idx, device=got.device)
    sel = got[it[:, 2], it[:, 1], it[:, 0]].cpu().numpy()
    info = check_ff(sel, ref, sc, "C2 next to the slab")
    print("C2 ff next to the slab", info, flush=True)


# ------------------------------------------------------------------ relaxed scan
def _scan_both(w, fire, cols=None, dfp=None):
    """Oracle force field rounded to FP32 feeds both sides; the GPU scans every
    column, the oracle the listed ones (polished equilibria)."""
    ref = orc.build_ff(w.grid, w.probe, w.atoms)
    ff32 = ref.astype(np.float32)
    ff64 = ff32.astype(np.float64)
    res = ppm.relaxed_scan(w.grid, torch.as_tensor(ff32, device="cuda"), w.probe, fire, w.scan,
                           dfp=dfp)
    torch.cuda.synchronize()
    ores = orc.relaxed_scan(w.grid, ff64, w.probe, fire, w.scan, cols=cols, polish_tol=1e-12,
                            with_lambda=True)
    g = {k: v.cpu().numpy() for k, v in res.items()}
    return ff64, ores, g


def test_scan_parity_c0_full():
    w = W.config0()
    fire = W.parity_fire(w.fire)
    ff64, ores, g = _scan_both(w, fire, dfp=w.df)
    info = grade_scan(w.grid, ff64, w.probe, fire, w.scan, ores["cols"], ores, g["pp"], g["fz"],
                      g["df"], w.df, label="C0")
    print("C0 scan", info, flush=True)
    assert info["graded"] > 0.95 * info["points"]


def test_scan_parity_c1_sampled_columns():
    """Full 240x240x100 scan on the GPU; 600 seeded columns re-run by the oracle."""
    w = W.config1()
    fire = W.parity_fire(w.fire)
    rng = np.random.default_rng(1001)
    cols = np.stack([rng.integers(0, w.scan.nx, 600), rng.integers(0, w.scan.ny, 600)], axis=1)
    ff64, ores, g = _scan_both(w, fire, cols=cols, dfp=w.df)
    info = grade_scan(w.grid, ff64, w.probe, fire, w.scan, cols, ores, g["pp"], g["fz"], g["df"],
                      w.df, label="C1")
    print("C1 scan", info, flush=True)
    assert info["graded"] > 0.9 * info["points"]


def test_scan_throughput_tolerance_certificates_c0():
    """At the workload's own convergence threshold (1e-4 eV/A) every GPU point must
    satisfy FIRE's stopping rule under the oracle's force balance (certificate)."""
    w = W.config0()
    ref = orc.build_ff(w.grid, w.probe, w.atoms)
    ff32 = ref.astype(np.float32)
    ff64 = ff32.astype(np.float64)
    res = ppm.relaxed_scan(w.grid, torch.as_tensor(ff32, device="cuda"), w.probe, w.fire, w.scan)
    pp = res["pp"].cpu().numpy()
    assert np.all(pp[..., 3] >= 0)
    cols = orc.all_columns(w.scan)
    from parity import anchors_for
    A = anchors_for(w.scan, cols)
    r = A + np.asarray(w.probe.d0) + pp[:, cols[:, 1], cols[:, 0], :3].transpose(1, 0, 2)
    gn, lam = orc.residual(w.grid, ff64, w.probe, A.reshape(-1, 3), r.reshape(-1, 3))
    assert np.all(gn < w.fire.f_conv * 1.001 + 2e-7)
    print("C0 iters mean", float(pp[..., 3].mean()), "sym-unstable points",
          int(np.sum(lam <= 0)), flush=True)


def test_scan_throughput_tolerance_certificates_c1_sampled():
    """The paper-scale scans exactly as the benchmark runs them (threshold 1e-4
    eV/A, FP32 interpolation arithmetic), trilinear and tricubic: 4,000 seeded
    relaxed points each, checked against FIRE's stopping rule under the
    oracle's FP64 force balance on the same FP32 grid.  The margin beyond
    f_conv covers the FP32 arithmetic (below 1e-6 eV/A here)."""
    w = W.config1()
    ff32 = orc.build_ff(w.grid, w.probe, w.atoms).astype(np.float32)
    res = ppm.relaxed_scan(w.grid, torch.as_tensor(ff32, device="cuda"), w.probe, w.fire,
                           w.scan, dfp=w.df)
    pp = res["pp"].cpu().numpy()
    assert np.all(pp[..., 3] >= 0)                   # every point converged
    rng = np.random.default_rng(2024)
    n = 4000
    ix, iy = rng.integers(0, w.scan.nx, n), rng.integers(0, w.scan.ny, n)
    k = rng.integers(0, w.scan.nz, n)
    from parity import anchors_for
    A = anchors_for(w.scan, np.stack([ix, iy], axis=1))        # [n][nz][3]
    A = A[np.arange(n), k]
    r = A + np.asarray(w.probe.d0) + pp[k, iy, ix, :3]
    gn, _ = orc.residual(w.grid, ff32.astype(np.float64), w.probe, A, r)
    excess = float((gn - w.fire.f_conv).max())
    print("C1 certificate: max |G| - f_conv", excess, flush=True)
    assert np.all(gn < w.fire.f_conv + 2e-6)
    # the tricubic scan on the energy channel, FP32 stencil contraction
    E32 = np.ascontiguousarray(ff32[..., 3])
    tri = ppm.relaxed_scan_tricubic(w.grid, torch.as_tensor(E32, device="cuda"), w.probe,
                                    w.fire, w.scan)
    pt = tri["pp"].cpu().numpy()
    assert np.all(pt[..., 3] >= 0)
    rt = A + np.asarray(w.probe.d0) + pt[k, iy, ix, :3]
    gt, _ = orc.residual_tricubic(w.grid, E32.astype(np.float64), w.probe, A, rt)
    excess = float((gt - w.fire.f_conv).max())
    print("C1 tricubic certificate: max |G| - f_conv", excess, flush=True)
    assert np.all(gt < w.fire.f_conv + 2e-6)


def test_scan_zero_field_exact_rest():
    grid = W.Grid((0.0, 0.0, 0.0), (0.1, 0.1, 0.1), (30, 30, 90))
    ff = torch.zeros((90, 30, 30, 4), dtype=torch.float32, device="cuda")
    scan = W.Scan(0.33, 0.41, 0.1, 0.1, 17, 5, 8.0, 0.1, 13)
    res = ppm.relaxed_scan(grid, ff, W.Probe(), W.Fire(), scan, dfp=W.DfParams())
    assert torch.all(res["fz"] == 0) and torch.all(res["pp"] == 0) and torch.all(res["df"] == 0)


@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 5, 12), (3, 40, 2)])
def test_scan_ragged_shapes(shape):
    """Tip lattices that do not fill the 16x16 tile, a single point and a single
    height, compared with the oracle on every column."""
    nx, ny, nz = shape
    w = W.config0()
    scan = W.Scan(7.1, 7.3, 0.13, 0.11, nx, ny, 10.2, 0.1, nz)
    w = W.Workload("ragged", w.atoms, w.grid, w.probe, w.fire, scan, w.df)
    fire = W.parity_fire(w.fire)
    ff64, ores, g = _scan_both(w, fire)
    grade_scan(w.grid, ff64, w.probe, fire, scan, ores["cols"], ores, g["pp"], g["fz"],
               label=f"ragged {shape}")


@pytest.mark.parametrize("nz", [100, 159, 160, 200])
def test_scan_output_routes_agree(nz):
    """The scan stages Fz in LDS (16x16 blocks up to 159 heights beside the
    helper wave's progress array, 8x8 blocks for a frequency shift without fz
    up to 256) or stores it as each height finishes; every route, and the fused
    frequency shift against the standalone one, gives the same bits (159 and
    160 straddle the 16x16 staging limit)."""
    w = W.config0()
    scan = W.Scan(7.1, 7.3, 0.13, 0.11, 19, 6, 10.2, 0.1, nz)
    ff = ppm.build_ff(w.grid, w.probe, ppm.atoms_to_device(w.atoms))
    run = lambda **kw: ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, scan, **kw)
    full = run(dfp=w.df, fz=True, pp=True)
    df_only = run(dfp=w.df, fz=False, pp=False)
    fz_only = run(fz=True, pp=False)
    pp_only = run(fz=False, pp=True)
    assert torch.equal(full["fz"], fz_only["fz"])
    assert torch.equal(full["df"], df_only["df"])
    assert torch.equal(full["pp"], pp_only["pp"])
    assert torch.equal(ppm.df(full["fz"], scan.dz, w.df), full["df"])
    # the work-group shapes the autotuner chooses between (8 x 8 with Fz
    # written straight to the fz output instead of an LDS stage too)
    for tile, direct in ((16, 0), (8, 0), (8, 1)):
        t = ppm.Tuning(scan_tile=tile, scan_fz_direct=direct)
        for kw in (dict(dfp=w.df, fz=True, pp=True), dict(dfp=w.df, fz=False, pp=False),
                   dict(fz=False, pp=True), dict(dfp=w.df, fz=True, pp=False),
                   dict(fz=True, pp=False)):
            if nz > 256 and not kw.get("fz") and "dfp" in kw:
                continue
            r = run(tuning=t, **kw)
            for k in r:
                assert torch.equal(r[k], full[k]), (tile, direct, k, kw)


def test_scan_below_and_above_grid_clamps():
    """Probe heights outside the grid see the field of the nearest z-layer (the
    grid is clamped in z); both sides agree there too."""
    w = W.config0()
    scan = W.Scan(7.0, 7.0, 0.2, 0.2, 4, 4, 16.5, 0.5, 12)   # probe from 12.5 A down to 7 A
    grid = W.Grid((0.0, 0.0, -4.0), (0.1, 0.1, 0.1), (160, 160, 130))   # top at 8.9 A
    w = W.Workload("clamp", w.atoms, grid, w.probe, w.fire, scan, w.df)
    fire = W.parity_fire(w.fire)
    ff64, ores, g = _scan_both(w, fire)
    grade_scan(grid, ff64, w.probe, fire, scan, ores["cols"], ores, g["pp"], g["fz"],
               label="clamp")


@pytest.mark.parametrize("periodic", [0, 1], ids=["open", "periodic"])
def test_scan_across_xy_edges(periodic):
    """Tips over and beyond both x and y edges of a small grid.  An open grid is
    clamped in x and y (the field is continued constantly past its edge
    voxels); a periodic one wraps.  Trilinear and tricubic scans against the
    oracle on every column."""
    w = edge_workload(periodic)
    grid, scan = w.grid, w.scan
    fire = W.parity_fire(w.fire)
    ff64, ores, g = _scan_both(w, fire)
    info = grade_scan(grid, ff64, w.probe, fire, scan, ores["cols"], ores, g["pp"], g["fz"],
                      label=f"edges periodic={periodic}")
    print("edges", periodic, info, flush=True)
    assert info["graded"] > 0.9 * info["points"]
    E32 = ff64[..., 3].astype(np.float32)
    E64 = E32.astype(np.float64)
    res = ppm.relaxed_scan_tricubic(grid, torch.as_tensor(E32, device="cuda"), w.probe, fire, scan)
    gt = {k: v.cpu().numpy() for k, v in res.items()}
    otr = orc.relaxed_scan_tricubic(grid, E64, w.probe, fire, scan, polish_tol=1e-12,
                                    with_lambda=True)
    info = grade_scan(grid, E64, w.probe, fire, scan, otr["cols"], otr, gt["pp"], gt["fz"],
                      label=f"tricubic edges periodic={periodic}", residual=orc.residual_tricubic)
    print("tricubic edges", periodic, info, flush=True)
    assert info["graded"] > 0.9 * info["points"]
    # every launch route of the trilinear scan gives these bits on this grid too
    # (wrapped cells and clamped edges in each), with a fused frequency shift
    ff32 = torch.as_tensor(ff64.astype(np.float32), device="cuda")
    ref = ppm.relaxed_scan(grid, ff32, w.probe, fire, scan, dfp=w.df, fz=True, pp=True)
    for tile, direct in ((16, 0), (8, 0), (8, 1)):
        t = ppm.Tuning(scan_tile=tile, scan_fz_direct=direct)
        r = ppm.relaxed_scan(grid, ff32, w.probe, fire, scan, dfp=w.df, fz=True, pp=True,
                             tuning=t)
        for k in ref:
            assert torch.equal(r[k], ref[k]), (periodic, tile, direct, k)


# ------------------------------------------------------------------ frequency shift
def test_df_fused_standalone_and_oracle_agree():
    w = W.config0()
    ref = orc.build_ff(w.grid, w.probe, w.atoms).astype(np.float32)
    res = ppm.relaxed_scan(w.grid, torch.as_tensor(ref, device="cuda"), w.probe, w.fire, w.scan,
                           dfp=w.df)
    alone = ppm.df(res["fz"], w.scan.dz, w.df)
    assert torch.equal(alone, res["df"])           # same weights, same summation order
    odf = orc.df(res["fz"].cpu().numpy().astype(np.float64), w.scan.dz, w.df)
    assert np.abs(alone.cpu().numpy() - odf).max() <= DF_TOL * 1e-2


@pytest.mark.parametrize("A,dz,nz", [(1.0, 0.1, 11), (0.7, 0.1, 30), (3.0, 0.05, 61),
                                     (1.3, 0.17, 25)])
def test_df_standalone_random_stacks(A, dz, nz):
    """Standalone kernel on random stacks (several half-widths, minimum height
    count) against the oracle's quadrature."""
    rng = np.random.default_rng(int(A * 100 + nz))
    fz = rng.normal(0, 0.05, size=(nz, 7, 33)).astype(np.float32)
    dfp = W.DfParams(A=A)
    got = ppm.df(torch.as_tensor(fz, device="cuda"), dz, dfp).cpu().numpy()
    ref = orc.df(fz.astype(np.float64), dz, dfp)
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, atol=2e-5 * np.abs(ref).max() + 1e-6)


def test_df_standalone_stack_beyond_the_chunk_grid():
    """A stack of more than 65,535 chunks of 16 outputs: the pass caps its grid
    in y and its blocks take a second chunk."""
    dz, dfp = 0.1, W.DfParams(A=1.0)
    m = ppm.df_half_width(dfp.A, dz)
    nz = 65535 * 16 + 2 * m + 37
    rng = np.random.default_rng(65535)
    fz = rng.normal(0, 0.05, size=(nz, 1, 3)).astype(np.float32)
    got = ppm.df(torch.as_tensor(fz, device="cuda"), dz, dfp).cpu().numpy()
    ref = orc.df(fz.astype(np.float64), dz, dfp)
    assert got.shape == ref.shape == (nz - 2 * m, 1, 3)
    np.testing.assert_allclose(got, ref, atol=2e-5 * np.abs(ref).max() + 1e-6)


@pytest.mark.parametrize("nz", [1, 2])
def test_scan_single_column(nz):
    """A lattice of one column: its block has one active lane beside 255 idle
    ones and the helper wave, which must end once that lane is done; one or two
    heights (the shortest warm-start histories).  Trilinear and tricubic scans
    against the polished oracle; every point must agree."""
    w0 = W.config0()
    scan = W.Scan(8.03, 7.96, 0.1, 0.1, 1, 1, 9.0, 0.1, nz)   # probe from 5 A above the plane
    w = W.Workload("one column", w0.atoms, w0.grid, w0.probe, w0.fire, scan, w0.df)
    fire = W.parity_fire(w.fire)
    print(f"single column, {nz} heights", flush=True)
    ff64, ores, g = _scan_both(w, fire)
    info = grade_scan(w.grid, ff64, w.probe, fire, scan, ores["cols"], ores, g["pp"], g["fz"],
                      label=f"one column nz {nz}")
    assert info["graded"] == info["points"], info
    E32 = np.ascontiguousarray(ff64[..., 3]).astype(np.float32)
    E64 = E32.astype(np.float64)
    tri = ppm.relaxed_scan_tricubic(w.grid, torch.as_tensor(E32, device="cuda"), w.probe, fire,
                                    scan)
    gt = {k: v.cpu().numpy() for k, v in tri.items()}
    otr = orc.relaxed_scan_tricubic(w.grid, E64, w.probe, fire, scan, polish_tol=1e-12,
                                    with_lambda=True)
    info = grade_scan(w.grid, E64, w.probe, fire, scan, otr["cols"], otr, gt["pp"], gt["fz"],
                      label=f"one column tricubic nz {nz}", residual=orc.residual_tricubic)
    assert info["graded"] == info["points"], info


def _c2_window():
    """A 100 x 100-column window of the large periodic workload that crosses the
    cell's x edge (tips at x = 36.0 ... 45.9 A, wrapping at 40 A) and the flake's
    edge, all 120 heights; the oracle's force field on the voxels its probes can
    reach (a 2 A lateral margin, z-layers 100 to 239), NaN elsewhere so that any
    read outside shows."""
    w = W.config2()
    scan = W.Scan(36.0, 14.0, 0.1, 0.1, 100, 100, w.scan.z_top, w.scan.dz, w.scan.nz)
    w = W.Workload("C2 window", w.atoms, w.grid, w.probe, w.fire, scan, w.df)
    nx, ny, nz = w.grid.n
    ix = np.arange(340, 481) % nx
    iy = np.arange(120, 261)
    iz = np.arange(100, 240)
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    idx = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.int32)
    vals = orc.ff_voxels(w.grid, w.probe, w.atoms, idx, with_scale=False)
    ff32 = np.full((nz, ny, nx, 4), np.nan, dtype=np.float32)
    ff32[idx[:, 2], idx[:, 1], idx[:, 0]] = vals.astype(np.float32)
    return w, ff32


def test_scan_c2_window_parity_and_certificates():
    """Large periodic sample (shifted-force 12 A cutoff): the GPU scans a
    100 x 100 x 120 window at the parity threshold, graded against the polished
    oracle on 300 seeded columns (positions, Fz and the frequency shift), then at
    the benchmark's threshold (1e-4 eV/A, FP32 interpolation arithmetic), where
    every point must converge and 4,000 seeded points are certified by the
    oracle's FP64 force balance."""
    w, ff32 = _c2_window()
    ffd = torch.as_tensor(ff32, device="cuda")
    fire = W.parity_fire(w.fire)
    res = ppm.relaxed_scan(w.grid, ffd, w.probe, fire, w.scan, dfp=w.df)
    g = {k: v.cpu().numpy() for k, v in res.items()}
    assert np.all(np.isfinite(g["pp"])) and np.all(np.isfinite(g["df"]))
    rng = np.random.default_rng(2202)
    cols = np.stack([rng.integers(0, w.scan.nx, 300), rng.integers(0, w.scan.ny, 300)], axis=1)
    ff64 = ff32.astype(np.float64)
    ores = orc.relaxed_scan(w.grid, ff64, w.probe, fire, w.scan, cols=cols, polish_tol=1e-12,
                            with_lambda=True)
    assert np.all(np.isfinite(ores["r"]))
    info = grade_scan(w.grid, ff64, w.probe, fire, w.scan, cols, ores, g["pp"], g["fz"],
                      g["df"], w.df, label="C2 window")
    print("C2 window scan", info, flush=True)
    assert info["graded"] > 0.9 * info["points"]
    # the benchmark's threshold
    thr = ppm.relaxed_scan(w.grid, ffd, w.probe, w.fire, w.scan, dfp=w.df)
    pp = thr["pp"].cpu().numpy()
    assert np.all(pp[..., 3] >= 0), f"{int(np.sum(pp[..., 3] < 0))} points not converged"
    n = 4000
    ix, iy = rng.integers(0, w.scan.nx, n), rng.integers(0, w.scan.ny, n)
    k = rng.integers(0, w.scan.nz, n)
    from parity import anchors_for
    A = anchors_for(w.scan, np.stack([ix, iy], axis=1))[np.arange(n), k]
    r = A + np.asarray(w.probe.d0) + pp[k, iy, ix, :3]
    gn, _ = orc.residual(w.grid, ff64, w.probe, A, r)
    print("C2 window certificate: max |G| - f_conv", float((gn - w.fire.f_conv).max()),
          "mean FIRE steps", float(pp[..., 3].mean()), flush=True)
    assert np.all(gn < w.fire.f_conv + 2e-6)


def test_scan_c2_full_lattice_converges():
    """The whole large periodic scan as the benchmark runs it (GPU force field,
    400 x 400 tips x 120 heights, 1e-4 eV/A): every point converges."""
    w = W.config2()
    ff = _gpu_ff(w)
    res = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, fz=False, pp=True)
    it = res["pp"][..., 3]
    bad = int((it < 0).sum().item())
    print("C2 full lattice: mean FIRE steps", float(it.abs().mean().item()), "max",
          float(it.abs().max().item()), "not converged", bad, flush=True)
    assert bad == 0


def test_scan_fire_step_counts_match_oracle_c0():
    """FIRE's path, not only its end point: at the parity threshold (FP64
    interpolation arithmetic on the GPU) the number of FIRE steps per relaxed
    point equals the oracle's (no polish, so both warm starts see the same
    previous equilibria) on at least 99% of the tiny workload's points; where
    they differ, by few steps."""
    w = W.config0()
    fire = W.parity_fire(w.fire)
    ff32 = orc.build_ff(w.grid, w.probe, w.atoms).astype(np.float32)
    res = ppm.relaxed_scan(w.grid, torch.as_tensor(ff32, device="cuda"), w.probe, fire, w.scan,
                           fz=False)
    steps = res["pp"][..., 3].cpu().numpy()                  # [nz, ny, nx]
    ores = orc.relaxed_scan(w.grid, ff32.astype(np.float64), w.probe, fire, w.scan)
    cols = ores["cols"]
    gsteps = steps[:, cols[:, 1], cols[:, 0]].T              # [col, k]
    same = gsteps == ores["iters"]
    diff = np.abs(gsteps - ores["iters"])
    print(f"C0 FIRE steps: {same.mean() * 100:.3f}% identical, {int((~same).sum())} differ "
          f"(largest difference {int(diff.max())}), mean {float(np.abs(gsteps).mean()):.2f}",
          flush=True)
    assert same.mean() >= 0.99
    assert np.all(gsteps >= 0) and np.all(ores["iters"] >= 0)


def test_scan_forced_nonconvergence_is_not_an_error():
    """Non-convergence is reported, not raised: with max_iter = 2 the call
    succeeds, points that need more steps carry -2, the others their step count,
    and the lateral stiffness is NaN exactly where the relaxation did not
    converge."""
    w = W.config0()
    scan = W.Scan(6.3, 6.9, 0.2, 0.2, 21, 13, 9.5, 0.1, 17)
    fire = W.Fire(max_iter=2)
    ff = ppm.build_ff(w.grid, w.probe, w.atoms)
    res = ppm.relaxed_scan(w.grid, ff, w.probe, fire, scan, dfp=w.df)
    steps = res["pp"][..., 3].cpu().numpy()
    assert np.all((steps == -2) | ((steps >= 0) & (steps <= 2)))
    assert np.sum(steps < 0) > 0.5 * steps.size
    k = ppm.lateral_stiffness(w.grid, ff, w.probe, scan, res["pp"]).cpu().numpy()
    assert np.array_equal(np.isnan(k).any(axis=-1), steps < 0)
    assert np.all(np.isfinite(k[steps >= 0]))


def test_scan_mirror_and_translation_invariance():
    """The scan commutes with the symmetries of the method (the oracle's force
    field pins the same for the grid): mirroring the force field in x about the
    grid's centre plane (Fx -> -Fx) and the tip lattice with it mirrors every
    relaxed displacement (ux -> -ux) and keeps Fz and the frequency shift; moving
    the grid origin and the tip lattice together by any offset changes nothing.
    At the parity threshold both hold to 1e-5 A, 1e-5 eV/A and 1e-4 Hz (the
    interpolation weights round differently)."""
    w = W.config0()
    fire = W.parity_fire(w.fire)
    g = W.Grid((4.0, 4.0, -2.0), (0.1, 0.1, 0.1), (80, 80, 110))
    scan = W.Scan(6.3, 6.55, 0.13, 0.11, 23, 19, 10.0, 0.1, 24)
    ff32 = orc.build_ff(g, w.probe, w.atoms).astype(np.float32)
    base = ppm.relaxed_scan(g, torch.as_tensor(ff32, device="cuda"), w.probe, fire, scan,
                            dfp=w.df)
    b = {k: v.cpu().numpy() for k, v in base.items()}
    # mirror x about the plane through voxel (nx - 1)/2
    xc = g.origin[0] + 0.5 * (g.n[0] - 1) * g.step[0]
    mf = ff32[:, :, ::-1, :].copy()
    mf[..., 0] *= -1.0
    mscan = W.Scan(2 * xc - (scan.x0 + (scan.nx - 1) * scan.dx), scan.y0, scan.dx, scan.dy,
                   scan.nx, scan.ny, scan.z_top, scan.dz, scan.nz)
    mir = {k: v.cpu().numpy() for k, v in ppm.relaxed_scan(
        g, torch.as_tensor(mf, device="cuda"), w.probe, fire, mscan, dfp=w.df).items()}
    mp = mir["pp"][:, :, ::-1, :]
    np.testing.assert_allclose(mp[..., 0], -b["pp"][..., 0], atol=1e-5)
    np.testing.assert_allclose(mp[..., 1:3], b["pp"][..., 1:3], atol=1e-5)
    np.testing.assert_allclose(mir["fz"][:, :, ::-1], b["fz"], atol=1e-5)
    np.testing.assert_allclose(mir["df"][:, :, ::-1], b["df"], atol=1e-4)
    # translation of grid and tips together
    d = np.array([0.7371, -1.0523, 0.4189])
    tg = W.Grid(tuple(np.array(g.origin) + d), g.step, g.n)
    tscan = W.Scan(scan.x0 + d[0], scan.y0 + d[1], scan.dx, scan.dy, scan.nx, scan.ny,
                   scan.z_top + d[2], scan.dz, scan.nz)
    tr = {k: v.cpu().numpy() for k, v in ppm.relaxed_scan(
        tg, torch.as_tensor(ff32, device="cuda"), w.probe, fire, tscan, dfp=w.df).items()}
    np.testing.assert_allclose(tr["pp"][..., :3], b["pp"][..., :3], atol=1e-5)
    np.testing.assert_allclose(tr["fz"], b["fz"], atol=1e-5)
    np.testing.assert_allclose(tr["df"], b["df"], atol=1e-4)


def test_scan_quarter_turn_invariance():
    """With equal lateral springs (kx = ky) the scan commutes with a quarter turn
    about the vertical axis through the centre of a square grid: turning the force
    field (node (i, j) -> (n-1-j, i), (Fx, Fy) -> (-Fy, Fx)) and the square tip
    lattice with it turns every relaxed displacement ((ux, uy) -> (-uy, ux)) and
    keeps Fz and the frequency shift, to the tolerances of the mirror test."""
    w = W.config0()
    assert w.probe.k_lat[0] == w.probe.k_lat[1]
    fire = W.parity_fire(w.fire)
    g = W.Grid((4.0, 4.0, -2.0), (0.1, 0.1, 0.1), (80, 80, 110))
    scan = W.Scan(6.3, 6.55, 0.12, 0.12, 21, 17, 10.0, 0.1, 24)
    ff32 = orc.build_ff(g, w.probe, w.atoms).astype(np.float32)
    b = {k: v.cpu().numpy() for k, v in ppm.relaxed_scan(
        g, torch.as_tensor(ff32, device="cuda"), w.probe, fire, scan, dfp=w.df).items()}
    n = g.n[0]
    xc = g.origin[0] + 0.5 * (n - 1) * g.step[0]
    yc = g.origin[1] + 0.5 * (n - 1) * g.step[1]
    rf = ff32[:, ::-1, :, :].transpose(0, 2, 1, 3).copy()      # rf[z, a, c] = ff[z, n-1-c, a]
    rf[..., 0], rf[..., 1] = -rf[..., 1].copy(), rf[..., 0].copy()
    d = scan.dx
    rscan = W.Scan(xc - (scan.y0 + (scan.ny - 1) * d - yc), yc + (scan.x0 - xc), d, d,
                   scan.ny, scan.nx, scan.z_top, scan.dz, scan.nz)
    rot = {k: v.cpu().numpy() for k, v in ppm.relaxed_scan(
        g, torch.as_tensor(rf, device="cuda"), w.probe, fire, rscan, dfp=w.df).items()}
    # rotated column (ny-1-iy, ix) holds base column (ix, iy)
    back = {k: v[:, :, ::-1].swapaxes(1, 2) for k, v in rot.items()}
    np.testing.assert_allclose(back["pp"][..., 0], -b["pp"][..., 1], atol=1e-5)
    np.testing.assert_allclose(back["pp"][..., 1], b["pp"][..., 0], atol=1e-5)
    np.testing.assert_allclose(back["pp"][..., 2], b["pp"][..., 2], atol=1e-5)
    np.testing.assert_allclose(back["fz"], b["fz"], atol=1e-5)
    np.testing.assert_allclose(back["df"], b["df"], atol=1e-4)


def test_ff_force_is_negative_energy_gradient_on_fine_grid():
    """F = -grad E on the GPU: 3 x 3 x 3 grids of 1e-3 A spacing at 40 seeded
    places around the paper-scale molecule; the force at the centre voxel against
    the central difference of the stored FP32 energy.  The bound is the FP32
    rounding of E over 2e-3 A (1e-7 of the energy's magnitude sum, divided by
    the step) plus 1e-3 of |F|."""
    w = W.config1()
    rng = np.random.default_rng(404)
    h = 1e-3
    worst = 0.0
    for _ in range(40):
        c = np.array([rng.uniform(7.0, 17.0), rng.uniform(7.0, 17.0), rng.uniform(2.8, 6.0)])
        g = W.Grid(tuple(c - h), (h, h, h), (3, 3, 3))
        f = ppm.build_ff(g, w.probe, w.atoms).cpu().numpy().astype(np.float64)
        _, sc = orc.ff_voxels(g, w.probe, w.atoms, np.array([[1, 1, 1]], dtype=np.int32))
        fd = -np.array([(f[1, 1, 2, 3] - f[1, 1, 0, 3]), (f[1, 2, 1, 3] - f[1, 0, 1, 3]),
                        (f[2, 1, 1, 3] - f[0, 1, 1, 3])]) / (2 * h)
        F = f[1, 1, 1, :3]
        tol = 1e-7 * sc[0, 1] / h + 1e-3 * np.linalg.norm(F) + 1e-6
        err = np.abs(F - fd).max()
        worst = max(worst, err / tol)
        assert err <= tol, (c, F, fd, tol)
    print("F = -grad E: worst error / bound", worst, flush=True)


def test_autotuner_choices_on_the_large_sample():
    """The autotuner times both brick depths on the large periodic build and
    both work-group shapes on its scan (as the benchmark runs it) and returns
    one of its candidates; the tuned outputs are the default ones (scan) or
    within the parity bound of the oracle (build, checked above)."""
    w = W.config2()
    t, ms = ppm.tune_build_ff(w.grid, w.probe, w.atoms)
    assert t.ff_nzb in (6, 8) and all(v > 0 for v in ms.values())
    ff = ppm.build_ff(w.grid, w.probe, w.atoms, tuning=t)
    t2, ms2, out = ppm.tune_relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=True,
                                         pp=False, tuning=t)
    assert (t2.scan_tile, t2.scan_fz_direct) in ((16, 0), (8, 0), (8, 1))
    assert t2.ff_nzb == t.ff_nzb and len(ms2) == 3 and all(v > 0 for v in ms2.values())
    ref = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=True, pp=False)
    assert torch.equal(out["df"], ref["df"]) and torch.equal(out["fz"], ref["fz"])
    print("large sample tuning:", t2, "build ms", ms, "scan ms", ms2, flush=True)
