"""Pins of the oracle's implicit adjoint (gradient of the frequency-shift stack
with respect to atom positions, charges, R_i and e_i).

The adjoint is not in the paper; it differentiates the equilibrium condition of
Eq. 1 and the quadrature of Eq. 3.  It is pinned here against central finite
differences of the whole oracle pipeline (force-field grid -> relaxed scan ->
frequency shift) and against the translation identity: moving the sample, the
grid and the tip lattice together changes nothing, so the position gradients
sum to minus the gradient with respect to a common shift of grid and tips.
"""
import numpy as np
import pytest

import oracle as orc
from paper_2401_14564_amd import workloads as W


def _problem(periodic=False):
    rng = np.random.default_rng(77)
    atoms = W.random_atoms(rng, 4, [0.8, 0.8, -0.2], [2.2, 2.2, 0.2], q_max=0.3)
    if periodic:
        # cell of 9 x 8.4 A with a 4.2 A shifted-force cutoff: the probe heights
        # put the cutoff sphere of every atom within reach of the tip columns,
        # and the atoms near x, y = 0 act through their images
        grid = W.Grid((0.0, 0.0, -1.0), (0.1, 0.1, 0.1), (90, 84, 70), 1, 4.2)
        scan = W.Scan(8.73, 0.21, 0.37, 0.41, 3, 3, 7.6, 0.1, 14)
    else:
        grid = W.Grid((0.0, 0.0, -1.0), (0.1, 0.1, 0.1), (30, 30, 70))
        scan = W.Scan(1.23, 1.31, 0.17, 0.19, 3, 3, 8.2, 0.1, 14)
    fire = W.parity_fire(W.Fire(), f_conv=1e-9, max_iter=50000)
    dfp = W.DfParams()
    m = orc.df_m(dfp.A, scan.dz)
    gdf = np.random.default_rng(5).normal(size=(scan.nz - 2 * m, scan.nx * scan.ny))
    return atoms, grid, scan, fire, dfp, gdf


def _loss(atoms, grid, scan, fire, dfp, gdf, probe=W.Probe()):
    ff = orc.build_ff(grid, probe, atoms)
    res = orc.relaxed_scan(grid, ff, probe, fire, scan, polish_tol=1e-13)
    df = orc.df(res["fz"].T, scan.dz, dfp)           # [nz-2m][ncol]
    return float(np.sum(gdf * df)), ff, res


# the monopole probe of the workloads, and the d_z2 quadrupole probe of the
# model comparison (Sec. 2.2.5: -0.05 e A^2, no monopole)
PROBES = [W.Probe(), W.Probe(q_pp=0.0, q_zz=-0.05)]


@pytest.mark.parametrize("periodic", [False, True], ids=["open", "periodic"])
@pytest.mark.parametrize("probe", PROBES, ids=["monopole", "quadrupole"])
def test_adjoint_matches_central_differences(probe, periodic):
    """Also on a periodic sample, where the shifted-force cutoff enters every
    pair derivative."""
    atoms, grid, scan, fire, dfp, gdf = _problem(periodic)
    L0, ff, res = _loss(atoms, grid, scan, fire, dfp, gdf, probe)
    assert np.all(res["gnorm"] < 1e-12)
    g = orc.scan_backward(grid, ff, probe, scan, res["cols"], res["r"], gdf, dfp, atoms)

    def fd(mod, h):
        ap, am = atoms.copy(), atoms.copy()
        mod(ap, +h)
        mod(am, -h)
        Lp = _loss(ap, grid, scan, fire, dfp, gdf, probe)[0]
        Lm = _loss(am, grid, scan, fire, dfp, gdf, probe)[0]
        return (Lp - Lm) / (2 * h)

    scale = max(np.abs(g["pos"]).max(), 1e-12)
    # smaller steps on the periodic sample: a voxel crossing an atom's cutoff
    # sphere is a kink of the field in the atom's parameters, and the relaxed
    # points there sit close to several of them
    hp = 1e-6 if periodic else 1e-4
    for i in range(atoms.n):
        for k in range(3):
            def mod(a, h, i=i, k=k):
                a.pos[i, k] += h
            assert g["pos"][i, k] == pytest.approx(fd(mod, hp), rel=2e-4, abs=2e-5 * scale)
        def modq(a, h, i=i):
            a.q[i] += h
        assert g["q"][i] == pytest.approx(fd(modq, hp), rel=2e-4, abs=1e-6)
        def modR(a, h, i=i):
            a.R[i] += h
        assert g["R"][i] == pytest.approx(fd(modR, hp), rel=2e-4, abs=1e-6)
        he = (1e-5 if periodic else 1e-3) * atoms.eps[i]
        def mode(a, h, i=i):
            a.eps[i] += h
        assert g["eps"][i] == pytest.approx(fd(mode, he), rel=2e-4, abs=1e-3)


@pytest.mark.parametrize("probe", PROBES, ids=["monopole", "quadrupole"])
def test_adjoint_translation_identity(probe):
    """sum_i dL/dr_i = -dL/d(delta) with delta a common shift of the grid origin
    and the tip lattice (the sample-probe system is translation invariant)."""
    atoms, grid, scan, fire, dfp, gdf = _problem()
    L0, ff, res = _loss(atoms, grid, scan, fire, dfp, gdf, probe)
    g = orc.scan_backward(grid, ff, probe, scan, res["cols"], res["r"], gdf, dfp, atoms)
    tot = g["pos"].sum(axis=0)
    # small step: the interpolated field is only continuous across cell faces,
    # and a common shift of all atoms by 1e-4 A already crosses one here
    h = 1e-5
    for k in range(3):
        vals = []
        for sgn in (+1, -1):
            e = np.zeros(3)
            e[k] = sgn * h
            g2 = W.Grid(tuple(np.array(grid.origin) + e), grid.step, grid.n)
            s2 = W.Scan(scan.x0 + e[0], scan.y0 + e[1], scan.dx, scan.dy, scan.nx, scan.ny,
                        scan.z_top + e[2], scan.dz, scan.nz)
            vals.append(_loss(atoms, g2, s2, fire, dfp, gdf, probe)[0])
        dshift = (vals[0] - vals[1]) / (2 * h)
        assert tot[k] == pytest.approx(-dshift, rel=1e-5, abs=1e-7 * np.abs(g["pos"]).max())


@pytest.mark.parametrize("periodic", [False, True], ids=["open", "periodic"])
def test_adjoint_dot_product(periodic):
    """<J u, w> = <u, J^T w> for the Jacobian J of the frequency-shift stack with
    respect to every parameter at once: J u by a central difference along a
    random direction u of (positions, charges, R_i, e_i), J^T w by the adjoint
    with the random cotangent w."""
    atoms, grid, scan, fire, dfp, w = _problem(periodic)
    probe = W.Probe(q_zz=-0.04)
    L0, ff, res = _loss(atoms, grid, scan, fire, dfp, w, probe)
    g = orc.scan_backward(grid, ff, probe, scan, res["cols"], res["r"], w, dfp, atoms)
    rng = np.random.default_rng(123)
    u = dict(pos=rng.normal(size=atoms.pos.shape), q=rng.normal(size=atoms.n),
             R=rng.normal(size=atoms.n), eps=rng.normal(size=atoms.n) * atoms.eps)
    ut_w = sum(float(np.sum(u[k] * g[k])) for k in u)
    h = 1e-6 if periodic else 1e-5

    def moved(s):
        a = atoms.copy()
        a.pos = a.pos + s * h * u["pos"]
        a.q = a.q + s * h * u["q"]
        a.R = a.R + s * h * u["R"]
        a.eps = a.eps + s * h * u["eps"]
        return a
    Ju_w = (_loss(moved(+1), grid, scan, fire, dfp, w, probe)[0] -
            _loss(moved(-1), grid, scan, fire, dfp, w, probe)[0]) / (2 * h)
    assert Ju_w == pytest.approx(ut_w, rel=1e-5)
