"""GPU implicit-adjoint gradients against the FP64 oracle's gradient (which is
pinned by central differences and the translation identity in the oracle tests),
through the C ABI and the autograd Function."""
import numpy as np
import pytest
import torch

import oracle as orc
import paper_2401_14564_amd as ppm
from paper_2401_14564_amd import workloads as W

pytestmark = pytest.mark.gpu

GRAD_RTOL = 1e-3


def _gpu_forward(w, fire, atoms):
    ff = ppm.build_ff(w.grid, w.probe, atoms)
    res = ppm.relaxed_scan(w.grid, ff, w.probe, fire, w.scan, dfp=w.df)
    return ff, res


def _oracle_forward(w, fire, atoms):
    ff = orc.build_ff(w.grid, w.probe, atoms)
    res = orc.relaxed_scan(w.grid, ff, w.probe, fire, w.scan, polish_tol=1e-12)
    df = orc.df(res["fz"].T, w.scan.dz, w.df)          # [nz-2m, col]
    return ff, res, df


GRAD_FLOOR = 1e-2     # elements below 1% of their group's largest are held to
                      # GRAD_RTOL of that 1%


def _compare(g, o, label):
    """Element by element: |g - o| <= GRAD_RTOL * max(|o|, GRAD_FLOOR * max|o|)
    for each gradient group (positions, charges, R_i, e_i)."""
    for k in ("pos", "q", "R", "eps"):
        a = g[k].cpu().numpy().reshape(-1)
        b = o[k].reshape(-1)
        scale = np.abs(b).max()
        ref = np.maximum(np.abs(b), GRAD_FLOOR * scale)
        err = np.abs(a - b) / ref
        print(f"{label} {k}: max|g|={scale:.4e} worst element rel err={err.max():.3e} "
              f"(at |g|={np.abs(b)[err.argmax()]:.3e})", flush=True)
        assert err.max() <= GRAD_RTOL, (label, k, err.max(), int(err.argmax()))


@pytest.mark.parametrize("periodic", [False, True], ids=["open", "periodic"])
@pytest.mark.parametrize("probe", [W.Probe(), W.Probe(q_pp=-0.05, q_zz=-0.1)],
                         ids=["monopole", "mixed"])
def test_backward_small_random_cotangent(periodic, probe):
    """Random cotangent on a small open sample, and on a periodic one whose
    atoms sit near the cell edges (minimum images) with a 4.2 A shifted-force
    cutoff that the probe's neighbourhood crosses."""
    rng = np.random.default_rng(77)
    if periodic:
        atoms = W.random_atoms(rng, 7, [0.0, 0.0, -0.2], [12.0, 11.0, 0.2], q_max=0.3)
        grid = W.Grid((0.0, 0.0, -1.0), (0.1, 0.1, 0.1), (120, 110, 70), 1, 4.2)
        scan = W.Scan(11.13, 10.21, 0.37, 0.41, 9, 7, 7.6, 0.1, 16)
    else:
        atoms = W.random_atoms(rng, 7, [0.8, 0.8, -0.2], [2.6, 2.6, 0.2], q_max=0.3)
        grid = W.Grid((0.0, 0.0, -1.0), (0.1, 0.1, 0.1), (36, 36, 70))
        scan = W.Scan(1.13, 1.21, 0.17, 0.19, 9, 7, 8.2, 0.1, 16)
    w = W.Workload("small", atoms, grid, probe, W.Fire(), scan, W.DfParams())
    fire = W.parity_fire(w.fire, f_conv=1e-8)
    m = orc.df_m(w.df.A, scan.dz)
    gdf = np.random.default_rng(5).normal(size=(scan.nz - 2 * m, scan.ny, scan.nx))
    ff, res = _gpu_forward(w, fire, atoms)
    g = ppm.relaxed_scan_backward(grid, ff, w.probe, scan, w.df, atoms, res["pp"],
                                  torch.as_tensor(gdf, dtype=torch.float32, device="cuda"))
    off, ores, _ = _oracle_forward(w, fire, atoms)
    o = orc.scan_backward(grid, off, w.probe, scan, ores["cols"], ores["r"],
                          gdf.reshape(gdf.shape[0], -1), w.df, atoms)
    _compare(g, o, f"small periodic={periodic} q_zz={probe.q_zz}")


def test_backward_deterministic():
    w, _ = W.config4()
    scan = W.Scan(w.scan.x0, w.scan.y0, 0.1, 0.1, 32, 32, w.scan.z_top, 0.1, 15)
    w = W.Workload("det", w.atoms, w.grid, w.probe, w.fire, scan, w.df)
    ff, res = _gpu_forward(w, w.fire, w.atoms)
    gdf = torch.randn(res["df"].shape, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    a = ppm.relaxed_scan_backward(w.grid, ff, w.probe, scan, w.df, w.atoms, res["pp"], gdf)
    b = ppm.relaxed_scan_backward(w.grid, ff, w.probe, scan, w.df, w.atoms, res["pp"], gdf)
    for k in a:
        assert torch.equal(a[k], b[k])


def test_backward_c4_full_against_oracle():
    """The differentiation workload: 60 atoms, 240^3 grid, 128x128x30 scan, loss
    ||df - df_target||^2 with the target from the perturbed molecule."""
    w, target = W.config4()
    fire = W.parity_fire(w.fire)
    # GPU side
    ff, res = _gpu_forward(w, fire, w.atoms)
    _, res_t = _gpu_forward(w, fire, target)
    gdf = 2.0 * (res["df"] - res_t["df"])
    g = ppm.relaxed_scan_backward(w.grid, ff, w.probe, w.scan, w.df, w.atoms, res["pp"], gdf)
    torch.cuda.synchronize()
    # oracle side
    off, ores, odf = _oracle_forward(w, fire, w.atoms)
    _, _, odf_t = _oracle_forward(w, fire, target)
    o = orc.scan_backward(w.grid, off, w.probe, w.scan, ores["cols"], ores["r"],
                          2.0 * (odf - odf_t), w.df, w.atoms)
    _compare(g, o, "C4")


def test_autograd_function_matches_direct_call():
    w, target = W.config4()
    scan = W.Scan(w.scan.x0 + 3.0, w.scan.y0 + 3.0, 0.1, 0.1, 24, 20, w.scan.z_top, 0.1, 14)
    w = W.Workload("ag", w.atoms, w.grid, w.probe, w.fire, scan, w.df)
    pos, q, R, eps = ppm.atoms_to_device(w.atoms)
    pos.requires_grad_(True)
    q.requires_grad_(True)
    R.requires_grad_(True)
    eps.requires_grad_(True)
    df = ppm.AFMStack.apply(pos, q, R, eps, w.grid, w.probe, w.fire, scan, w.df)
    loss = (df ** 2).sum()
    loss.backward()
    ff, res = _gpu_forward(w, w.fire, w.atoms)
    assert torch.equal(res["df"], df.detach())
    g = ppm.relaxed_scan_backward(w.grid, ff, w.probe, scan, w.df, w.atoms, res["pp"],
                                  2.0 * res["df"])
    assert torch.equal(pos.grad, g["pos"]) and torch.equal(q.grad, g["q"])
    assert torch.equal(R.grad, g["R"]) and torch.equal(eps.grad, g["eps"])


def test_backward_gpu_central_differences_five_atoms():
    """GPU gradient against central differences of the GPU forward (h = 1e-4 A on
    positions) for 5 atoms of the differentiation molecule; the FP32 grid limits
    the difference quotient to about 1e-2 relative accuracy."""
    w, _ = W.config4()
    scan = W.Scan(w.scan.x0 + 2.0, w.scan.y0 + 2.0, 0.1, 0.1, 40, 40, w.scan.z_top, 0.1, 20)
    w = W.Workload("fd", w.atoms, w.grid, w.probe, w.fire, scan, w.df)
    fire = W.parity_fire(w.fire, f_conv=1e-9)
    rng = np.random.default_rng(9)
    gdf_np = rng.normal(size=(scan.nz - 10, scan.ny, scan.nx))
    gdf = torch.as_tensor(gdf_np, dtype=torch.float32, device="cuda")

    def loss(atoms):
        ff, res = _gpu_forward(w, fire, atoms)
        return float((res["df"].double() * gdf.double()).sum())

    ff, res = _gpu_forward(w, fire, w.atoms)
    g = ppm.relaxed_scan_backward(w.grid, ff, w.probe, scan, w.df, w.atoms, res["pp"], gdf)
    gp = g["pos"].cpu().numpy()
    # the five atoms nearest the scanned window
    c = np.array([scan.x0 + 2.0, scan.y0 + 2.0])
    near = np.argsort(np.linalg.norm(w.atoms.pos[:, :2] - c, axis=1))[:5]
    h = 1e-4
    for i in near:
        for k in range(3):
            ap, am = w.atoms.copy(), w.atoms.copy()
            ap.pos[i, k] += h
            am.pos[i, k] -= h
            fd = (loss(ap) - loss(am)) / (2 * h)
            assert abs(gp[i, k] - fd) <= 2e-2 * np.abs(gp).max(), (i, k, gp[i, k], fd)
