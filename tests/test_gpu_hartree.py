"""Electrostatics from a grid potential (Sec. 2.2.3, by the convolution theorem
of Sec. 5.1.2) on the GPU against the FP64 oracle's direct cross-correlation,
which is pinned in test_oracle_hartree.py.  Both sides read the same FP32
potential and density, made by the input generator and the oracle."""
import numpy as np
import pytest
import torch

import oracle as orc
import paper_2401_14564_amd as ppm
from paper_2401_14564_amd import workloads as W

pytestmark = pytest.mark.gpu

# FP32 output of an FP64 transform: a few FP32 ulps of each value, plus a
# floor far below it relative to the largest magnitude of the field (the three
# force components come out of the same transforms and share one scale)
REL, FLOOR = 1e-6, 1e-9


def _scales(ref):
    f = np.abs(ref[..., :3]).max()
    return np.array([f, f, f, np.abs(ref[..., 3]).max()])


def _check(got, ref, label):
    sc = _scales(ref)
    for c in range(4):
        d = np.abs(got[..., c].astype(np.float64) - ref[..., c])
        tol = REL * np.abs(ref[..., c]) + FLOOR * sc[c]
        assert np.all(d <= tol), (label, c, float((d / np.maximum(tol, 1e-300)).max()))
    return float(max((np.abs(got[..., c] - ref[..., c]) / sc[c]).max()
                     for c in range(4) if sc[c] > 0))


def _inputs(grid, n_atoms=5, seed=0, q_pp=-0.05, q_zz=-0.05, sigma=W.TIP_SIGMA):
    rng = np.random.default_rng(seed)
    L = np.array(grid.n) * np.array(grid.step)
    atoms = W.random_atoms(rng, n_atoms, np.array(grid.origin) + 0.2 * L,
                           np.array(grid.origin) + 0.8 * L)
    V = W.hartree_potential(atoms, grid).astype(np.float32)
    rho = orc.tip_density(grid, q_pp, q_zz, sigma).astype(np.float32)
    return V, rho


def test_tip_density_matches_oracle():
    g = W.Grid((0.0, 0.0, 0.0), (0.2, 0.21, 0.19), (30, 25, 36))
    for q_pp, q_zz, s in ((-0.05, 0.0, 0.7), (0.0, -0.05, 0.7), (0.2, 0.1, 0.45)):
        got = ppm.tip_density(g, q_pp, q_zz, s).cpu().numpy()
        ref = orc.tip_density(g, q_pp, q_zz, s)
        d = np.abs(got - ref)
        assert np.all(d <= 2.0 ** -23 * np.abs(ref) + 1e-30 * np.abs(ref).max()), (q_pp, q_zz, s)


@pytest.mark.parametrize("n", [(24, 20, 18), (9, 25, 16), (1000, 3, 2), (2, 2, 2), (5, 48, 27),
                               (6, 2, 1000), (3, 9, 5)])
def test_hartree_full_grid_against_oracle(n):
    """Mixed radices (4, 2, 3, 5), 1000-point axes along x and z (three lines per
    block), the smallest grid, odd lengths on every axis, and ny = 2."""
    g = W.Grid((0.3, -0.1, -2.0), (0.31, 0.29, 0.33), n)
    V, rho = _inputs(g, seed=sum(n))
    ref = orc.hartree_ff(g, rho, V)
    got = ppm.hartree_ff(g, torch.as_tensor(V, device="cuda"),
                         torch.as_tensor(rho, device="cuda")).cpu().numpy()
    worst = _check(got, ref, f"grid {n}")
    print("hartree", n, "worst rel to max", worst, flush=True)


def test_hartree_paper_scale_sampled_voxels():
    """The paper-scale molecule and 240^3 grid (0.1 A), a d_z2 probe of -0.05 e A^2
    (Sec. 2.2.5); 48 seeded voxels re-computed by the oracle's direct sum."""
    w = W.config1()
    V = W.hartree_potential(w.atoms, w.grid).astype(np.float32)
    rho = orc.tip_density(w.grid, 0.0, -0.05, W.TIP_SIGMA).astype(np.float32)
    got = ppm.hartree_ff(w.grid, torch.as_tensor(V, device="cuda"),
                         torch.as_tensor(rho, device="cuda")).cpu().numpy()
    rng = np.random.default_rng(9)
    n = np.array(w.grid.n)
    idx = np.stack([rng.integers(0, n[c], 48) for c in range(3)], axis=1).astype(np.int32)
    # half of the samples in the band the probe scans (z between 2 and 9 A)
    idx[:24, 2] = rng.integers(60, 130, 24)
    ref = orc.hartree_ff(w.grid, rho, V, idx)
    g = got[idx[:, 2], idx[:, 1], idx[:, 0]]
    full = _scales(got)
    for c in range(4):
        d = np.abs(g[:, c] - ref[:, c])
        tol = REL * np.abs(ref[:, c]) + FLOOR * full[c]
        assert np.all(d <= tol), (c, float((d / tol).max()))


def test_hartree_accumulates_onto_the_lennard_jones_grid():
    g = W.Grid((0.0, 0.0, -1.0), (0.3, 0.3, 0.3), (20, 24, 30))
    V, rho = _inputs(g, seed=4)
    rng = np.random.default_rng(5)
    atoms = W.random_atoms(rng, 6, [1.0, 1.0, 0.0], [5.0, 6.0, 1.0])
    probe = W.Probe(q_pp=0.0, q_zz=0.0)
    lj = ppm.build_ff(g, probe, atoms)
    Vd, rd = torch.as_tensor(V, device="cuda"), torch.as_tensor(rho, device="cuda")
    el = ppm.hartree_ff(g, Vd, rd)
    tot = lj.clone()
    ppm.hartree_ff(g, Vd, rd, out=tot, accumulate=True)
    assert torch.equal(tot, lj + el)
    # the workspace is reusable and the result does not depend on its contents
    ws = ppm.hartree_workspace(g)
    ws.fill_(255)
    again = ppm.hartree_ff(g, Vd, rd, workspace=ws)
    assert torch.equal(again, el)
