"""Pins of the oracle's tricubic potential interpolation (the variant of Sec.
5.1.1 step 2 that stores only the energy): Catmull-Rom cubic convolution per
axis, force = -grad of the interpolant.  Pinned by polynomial reproduction,
node values, finite differences, C1 continuity across cell faces, the order of
convergence on a Lennard-Jones potential, and a Newton solve of the relaxation
on a quadratic potential."""
import numpy as np
import pytest

import oracle as orc
from paper_2401_14564_amd import workloads as W

PROBE = W.Probe()


def _grid(origin, step, n):
    return W.Grid(tuple(origin), tuple(step), tuple(n))


def _sample(g, fn):
    nx, ny, nz = g.n
    z, y, x = np.meshgrid(g.origin[2] + np.arange(nz) * g.step[2],
                          g.origin[1] + np.arange(ny) * g.step[1],
                          g.origin[0] + np.arange(nx) * g.step[0], indexing="ij")
    return fn(np.stack([x, y, z], axis=-1))


def _quadratic(rng):
    A = rng.normal(size=(3, 3))
    b = rng.normal(size=3)
    c = rng.normal()
    return A, b, c, (lambda r: np.einsum("...i,ij,...j->...", r, A, r) + r @ b + c)


def test_reproduces_quadratics_exactly():
    """Keys' cubic convolution with a = -1/2 reproduces polynomials of degree 2
    per axis, so a quadratic potential, its force and Hessian come out exactly."""
    rng = np.random.default_rng(1)
    A, b, c, fn = _quadratic(rng)
    g = _grid((0.2, -0.1, 0.5), (0.1, 0.13, 0.17), (12, 11, 10))
    En = _sample(g, fn)
    S = A + A.T
    for _ in range(40):
        r = np.array(g.origin) + rng.uniform(1.0, np.array(g.n) - 2.0) * np.array(g.step)
        E, F, H = orc.interp_tricubic(En, g, r, with_hessian=True)
        assert E == pytest.approx(fn(r), abs=1e-11)
        np.testing.assert_allclose(F, -(S @ r + b), atol=1e-10)
        np.testing.assert_allclose(H, S, atol=1e-9)


def test_node_values_and_gradient_by_differences():
    rng = np.random.default_rng(2)
    g = _grid((0, 0, 0), (0.1, 0.1, 0.1), (9, 8, 7))
    En = rng.normal(size=(7, 8, 9))
    for (ix, iy, iz) in [(0, 0, 1), (4, 3, 2), (8, 7, 5)]:
        E, _ = orc.interp_tricubic(En, g, [ix * 0.1, iy * 0.1, iz * 0.1])
        assert E == pytest.approx(En[iz, iy, ix], abs=1e-13)
    h = 1e-6
    for _ in range(20):
        r = rng.uniform([0.01, 0.01, 0.15], [0.79, 0.69, 0.5])    # inside the open grid
        _, F = orc.interp_tricubic(En, g, r)
        fd = np.array([-(orc.interp_tricubic(En, g, r + h * e)[0] -
                         orc.interp_tricubic(En, g, r - h * e)[0]) / (2 * h) for e in np.eye(3)])
        np.testing.assert_allclose(F, fd, rtol=1e-6, atol=1e-6)


def test_c1_continuity_across_cell_faces():
    """Catmull-Rom interpolation is C1: energy and force agree on both sides of a
    cell face."""
    rng = np.random.default_rng(3)
    g = _grid((0, 0, 0), (0.1, 0.1, 0.1), (9, 8, 7))
    En = rng.normal(size=(7, 8, 9))
    for axis in range(3):
        r = np.array([0.34, 0.27, 0.31])
        r[axis] = 0.3
        e = np.zeros(3)
        e[axis] = 1e-10
        Em, Fm = orc.interp_tricubic(En, g, r - e)
        Ep, Fp = orc.interp_tricubic(En, g, r + e)
        assert Em == pytest.approx(Ep, abs=1e-8)
        np.testing.assert_allclose(Fm, Fp, atol=1e-7)


def test_force_converges_with_grid_spacing():
    """On a single Lennard-Jones + Coulomb centre the interpolated force
    approaches the analytic one as the grid is refined, at second order or
    better (cubic convolution: O(h^3) values, O(h^2) derivatives)."""
    atom = W.Atoms(np.array([[1.0, 1.0, 0.0]]), np.array([0.2]), np.array([1.9]),
                   np.array([0.0027]), ["C"])
    pts = np.array([[1.13, 0.91, 3.37], [0.77, 1.21, 3.9], [1.4, 1.05, 3.1]])
    errs = []
    for h in (0.2, 0.1, 0.05):
        n = (int(round(2.0 / h)), int(round(2.0 / h)), int(round(3.0 / h)))
        g = _grid((0.0, 0.0, 1.5), (h, h, h), n)
        En = orc.build_ff(g, PROBE, atom)[..., 3]
        exact, _ = orc.point_ff(pts, atom, PROBE, g)
        got = np.array([orc.interp_tricubic(En, g, p)[1] for p in pts])
        errs.append(np.abs(got - exact[:, :3]).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs


def test_relaxation_on_quadratic_potential_matches_newton():
    """A quadratic potential is interpolated exactly, so FIRE on the tricubic
    potential must land on the root of the analytic force balance."""
    rng = np.random.default_rng(9)
    M = rng.normal(size=(3, 3)) * 0.003
    S = (M @ M.T) + 0.002 * np.eye(3)        # potential 1/2 (r-c) S (r-c) + b.r: stable well
    centre = np.array([2.0, 2.0, 3.0])
    b0 = np.array([-0.004, 0.003, -0.02])

    def pot(r):
        d = r - centre
        return 0.5 * np.einsum("...i,ij,...j->...", d, S, d) + d @ b0

    g = _grid((0.0, 0.0, 0.0), (0.1, 0.1, 0.1), (40, 40, 60))
    En = _sample(g, pot)
    fire = W.parity_fire(W.Fire(), f_conv=1e-10)
    scan = W.Scan(1.9, 2.05, 0.1, 0.1, 2, 1, 7.1, 0.1, 5)
    res = orc.relaxed_scan_tricubic(g, En, PROBE, fire, scan, polish_tol=1e-13)
    R0 = 4.0
    for c, (ix, iy) in enumerate(res["cols"]):
        for k in range(5):
            anchor = np.array([1.9 + 0.1 * ix, 2.05 + 0.1 * iy, 7.1 - 0.1 * k])
            r = anchor + np.array(PROBE.d0)
            for _ in range(100):
                d = r - anchor
                dn = np.linalg.norm(d)
                kk = np.array([PROBE.k_lat[0], PROBE.k_lat[1], 0.0])
                G = -PROBE.k_rad * (dn - R0) * d / dn - kk * (d - np.array(PROBE.d0)) \
                    - (S @ (r - centre) + b0)
                Jt = -PROBE.k_rad * ((1 - R0 / dn) * np.eye(3) + R0 * np.outer(d, d) / dn ** 3) \
                    - np.diag(kk)
                r = r - np.linalg.solve(Jt - S, G)
            np.testing.assert_allclose(res["r"][c, k], r, atol=1e-10)


def test_open_grid_continues_the_force_beyond_its_edges():
    """On a grid without periodic images the point is clamped to the grid box in
    x and y (as in z): beyond the first and last voxel the force is the one at
    the clamped point, so it is continuous across the edge, and it does not
    change along the clamped axis (that column of -dF/dr is zero).  On a
    periodic grid the interpolant repeats with period n*step instead."""
    rng = np.random.default_rng(9)
    g = _grid((0.0, 0.0, 0.0), (0.1, 0.12, 0.1), (9, 8, 10))
    En = rng.normal(size=(10, 8, 9))
    for out_pt, edge_pt, axis in (((-0.35, 0.4, 0.5), (0.0, 0.4, 0.5), 0),
                                  ((1.3, 0.4, 0.5), (0.8, 0.4, 0.5), 0),
                                  ((0.41, -0.2, 0.5), (0.41, 0.0, 0.5), 1),
                                  ((0.41, 1.1, 0.5), (0.41, 0.84, 0.5), 1)):
        E, F, H = orc.interp_tricubic(En, g, out_pt, with_hessian=True)
        E0, F0, H0 = orc.interp_tricubic(En, g, edge_pt, with_hessian=True)
        assert E == pytest.approx(E0, abs=1e-13)
        np.testing.assert_allclose(F, F0, atol=1e-12)
        assert np.all(H[:, axis] == 0.0)
        other = [b for b in range(3) if b != axis]
        np.testing.assert_allclose(H[:, other], H0[:, other], atol=1e-10)
        # just inside the edge the force is the same to first order
        inside = np.array(edge_pt, dtype=float)
        inside[axis] += -1e-7 if out_pt[axis] > edge_pt[axis] else 1e-7
        np.testing.assert_allclose(orc.interp_tricubic(En, g, inside)[1], F0, atol=1e-4)
    gp = W.Grid((0.0, 0.0, 0.0), (0.1, 0.12, 0.1), (9, 8, 10), 1, 0.3)
    r = np.array([0.23, 0.31, 0.47])
    a = orc.interp_tricubic(En, gp, r)
    b = orc.interp_tricubic(En, gp, r + np.array([0.9, -0.96, 0.0]))
    assert a[0] == pytest.approx(b[0], abs=1e-12)
    np.testing.assert_allclose(a[1], b[1], atol=1e-11)
