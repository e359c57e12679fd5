"""Pins of the FP64 oracle against what the paper and mathematics fix.

None of these tests compares the oracle with a retyped copy of its own formula:
each checks a closed form, an invariant, a special case that reduces to a
library routine, or a limit.  Each docstring names the passage it rests on.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special

import oracle as orc
from paper_2401_14564_amd import workloads as W

KE = 14.3996454784


def _grid(origin=(0.0, 0.0, 0.0), step=(0.1, 0.1, 0.1), n=(8, 8, 8), periodic=0, cutoff=0.0):
    return W.Grid(tuple(origin), tuple(step), tuple(n), periodic, cutoff)


def _atoms(pos, q=None, R=None, eps=None):
    pos = np.asarray(pos, dtype=float).reshape(-1, 3)
    n = len(pos)
    q = np.zeros(n) if q is None else np.asarray(q, float)
    R = np.full(n, 1.9) if R is None else np.asarray(R, float)
    eps = np.full(n, 0.0027) if eps is None else np.asarray(eps, float)
    return W.Atoms(pos, q, R, eps, ["X"] * n)


PROBE = W.Probe()


# ---------------------------------------------------------------- LJ / Coulomb
def test_lj_minimum_depth_and_zero_crossing():
    """Eq. 5 with the mixing rules of Sec. 2.2.1: a single LJ pair has its
    minimum at rho = R_i + R_PP with energy -sqrt(e_i e_PP) and zero force,
    and crosses zero at rho = 2^(-1/6) (R_i + R_PP)."""
    a = _atoms([[0.0, 0.0, 0.0]], R=[1.9], eps=[0.0027])
    Rm = 1.9 + PROBE.R_pp
    em = math.sqrt(0.0027 * PROBE.eps_pp)
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    out, _ = orc.point_ff([Rm * d, 2 ** (-1 / 6) * Rm * d, 0.9 * Rm * d, 1.2 * Rm * d],
                          a, PROBE, _grid())
    assert out[0, 3] == pytest.approx(-em, rel=1e-13)
    assert np.abs(out[0, :3]).max() < 1e-15
    assert abs(out[1, 3]) < 1e-15
    # repulsive inside the minimum, attractive outside (force along +d / -d)
    assert np.dot(out[2, :3], d) > 0 and np.dot(out[3, :3], d) < 0


def test_coulomb_closed_form():
    """Eq. 6: E = k_e q_i q_PP / rho (LJ switched off with e_i = 0); the force
    is E/rho along r - r_i.  k_e in eV*A/e^2 is CODATA's e^2/(4 pi eps0)."""
    a = _atoms([[1.0, 2.0, 3.0]], q=[0.7], eps=[0.0])
    probe = W.Probe(q_pp=-0.4)
    r = np.array([1.0 + 1.5, 2.0 - 2.0, 3.0 + 0.3])
    rho = np.linalg.norm(r - a.pos[0])
    out, _ = orc.point_ff([r], a, probe, _grid())
    E = KE * 0.7 * -0.4 / rho
    assert out[0, 3] == pytest.approx(E, rel=1e-14)
    np.testing.assert_allclose(out[0, :3], E / rho * (r - a.pos[0]) / rho, rtol=1e-13)
    # two elementary charges 1 A apart: 14.3996 eV (textbook value)
    a1 = _atoms([[0.0, 0.0, 0.0]], q=[1.0], eps=[0.0])
    out1, _ = orc.point_ff([[0.0, 0.0, 1.0]], a1, W.Probe(q_pp=1.0), _grid())
    assert out1[0, 3] == pytest.approx(14.3996454784, rel=1e-12)


def test_force_is_negative_energy_gradient():
    """Sec. 2.2: F = -grad E.  Central differences of the oracle's energy
    (h = 1e-4 A) match its force on a random 6-atom sample."""
    rng = np.random.default_rng(7)
    a = W.random_atoms(rng, 6, [0, 0, -0.5], [6, 6, 0.5])
    pts = rng.uniform([0, 0, 2.5], [6, 6, 5.0], size=(20, 3))
    h = 1e-4
    out, _ = orc.point_ff(pts, a, PROBE, _grid())
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        Ep, _ = orc.point_ff(pts + e, a, PROBE, _grid())
        Em, _ = orc.point_ff(pts - e, a, PROBE, _grid())
        fd = -(Ep[:, 3] - Em[:, 3]) / (2 * h)
        np.testing.assert_allclose(out[:, k], fd, rtol=1e-6, atol=1e-10)


def test_superposition_and_linearity():
    """Eq. 5 and Eq. 6 are sums over atoms: FF(A u B) = FF(A) + FF(B); the
    Coulomb part is linear in the charges."""
    rng = np.random.default_rng(3)
    g = _grid(origin=(0, 0, 2.0), n=(6, 5, 4))
    A = W.random_atoms(rng, 4, [0, 0, -0.5], [1, 1, 0.5])
    B = W.random_atoms(rng, 3, [0, 0, -0.5], [1, 1, 0.5])
    AB = W.Atoms(np.vstack([A.pos, B.pos]), np.r_[A.q, B.q], np.r_[A.R, B.R],
                 np.r_[A.eps, B.eps], A.types + B.types)
    fa, fb, fab = (orc.build_ff(g, PROBE, x) for x in (A, B, AB))
    np.testing.assert_allclose(fab, fa + fb, rtol=1e-12, atol=1e-15)
    A2, A0 = A.copy(), A.copy()
    A2.q = 2 * A.q
    A0.q = 0 * A.q
    f2, f0 = orc.build_ff(g, PROBE, A2), orc.build_ff(g, PROBE, A0)
    np.testing.assert_allclose(f2 - f0, 2 * (fa - f0), rtol=1e-11, atol=1e-14)


def test_translation_invariance():
    """The sample is rigid and the field depends only on r - r_i: shifting atoms
    and grid origin together leaves every voxel unchanged."""
    rng = np.random.default_rng(11)
    A = W.random_atoms(rng, 5, [0, 0, -0.5], [1, 1, 0.5])
    g = _grid(origin=(-0.2, 0.1, 2.0), n=(5, 6, 4))
    shift = np.array([3.3, -1.7, 0.9])
    B = A.copy()
    B.pos = A.pos + shift
    g2 = _grid(origin=tuple(np.array(g.origin) + shift), n=g.n)
    np.testing.assert_allclose(orc.build_ff(g2, PROBE, B), orc.build_ff(g, PROBE, A),
                               rtol=1e-11, atol=1e-14)


def test_mirror_symmetry():
    """Mirroring the sample in x about a grid plane flips Fx and keeps Fy, Fz
    and E (pair potentials are isotropic)."""
    rng = np.random.default_rng(5)
    A = W.random_atoms(rng, 5, [0, 0, -0.5], [1.0, 1.0, 0.5])
    n = (9, 4, 3)
    g = _grid(origin=(0.1, 0.0, 2.0), n=n)
    xc = 0.1 + 4 * 0.1                      # voxel ix = 4 is the mirror plane
    B = A.copy()
    B.pos[:, 0] = 2 * xc - A.pos[:, 0]
    fa = orc.build_ff(g, PROBE, A)
    fb = orc.build_ff(g, PROBE, B)[:, :, ::-1, :]
    np.testing.assert_allclose(fb[..., 0], -fa[..., 0], rtol=1e-11, atol=1e-14)
    np.testing.assert_allclose(fb[..., 1:], fa[..., 1:], rtol=1e-11, atol=1e-14)


def test_minimum_image_and_cutoff():
    """Periodic xy with a cutoff: an atom just across the cell boundary acts
    through its nearest image, and pairs at rho >= r_c are dropped."""
    L = 2.0
    g = _grid(origin=(0, 0, 0), step=(0.1, 0.1, 0.1), n=(20, 20, 10), periodic=1, cutoff=0.9)
    A = _atoms([[1.95, 0.05, 0.0]], q=[0.3], R=[1.5], eps=[0.002])
    Ashift = _atoms([[1.95 - L, 0.05, 0.0]], q=[0.3], R=[1.5], eps=[0.002])
    for probe in (PROBE, W.Probe(q_zz=-0.1)):
        for r in ([0.2, 0.1, 0.5], [0.25, -0.3, 0.35]):
            r = np.array(r)
            out, _ = orc.point_ff([r], A, probe, g)
            # the same atom's image without periodicity, then the shifted-force
            # construction along the ray through r (see the next test)
            d = r - Ashift.pos[0]
            rho = np.linalg.norm(d)
            pc = Ashift.pos[0] + 0.9 * d / rho
            ref, _ = orc.point_ff([r], Ashift, probe, _grid())
            refc, _ = orc.point_ff([pc], Ashift, probe, _grid())
            E = ref[0, 3] - refc[0, 3] + (rho - 0.9) * (refc[0, :3] @ d / rho)
            assert out[0, 3] == pytest.approx(E, rel=1e-12, abs=1e-15)
    far, _ = orc.point_ff([[1.0, 1.0, 0.5]], A, PROBE, g)   # nearest image 1.08 A > r_c
    assert np.all(far == 0.0)


@pytest.mark.parametrize("probe", [W.Probe(), W.Probe(q_pp=0.0, q_zz=-0.05),
                                   W.Probe(q_pp=-0.05, q_zz=-0.1)],
                         ids=["monopole", "quadrupole", "mixed"])
def test_shifted_force_cutoff(probe):
    """The cutoff of a periodic sample is a shifted-force truncation: along every
    ray from an atom, each pair term Y(direction) g(rho) becomes the remainder of
    its first-order Taylor expansion about rho = r_c, so the energy and the
    force both vanish on the cutoff sphere.  Checked against the untruncated sum
    (open sample, pinned by the LJ and Coulomb closed forms above): for the
    energy, E_c(r) = E(r) - E(p) + (rho - r_c) F(p).(r - r_i)/rho with p the
    point of the ray on the sphere; F = -grad E by central differences, also
    just inside the sphere; and E, F -> 0 as rho -> r_c."""
    rc = 3.7
    g = _grid(origin=(0, 0, 0), step=(0.1, 0.1, 0.1), n=(100, 100, 40), periodic=1, cutoff=rc)
    rng = np.random.default_rng(3)
    for _ in range(12):
        a = rng.uniform([2.0, 2.0, -0.5], [8.0, 8.0, 0.5])
        A = _atoms([a], q=[rng.uniform(-0.3, 0.3)], R=[1.8], eps=[0.003])
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        for rho in (rng.uniform(2.4, rc - 0.05), rc - 1e-7):
            r = a + rho * u
            out, _ = orc.point_ff([r], A, probe, g)
            ref, _ = orc.point_ff([r], A, probe, _grid())
            refc, _ = orc.point_ff([a + rc * u], A, probe, _grid())
            E = ref[0, 3] - refc[0, 3] + (rho - rc) * (refc[0, :3] @ u)
            assert out[0, 3] == pytest.approx(E, rel=1e-11, abs=1e-14)
            if rho > rc - 1e-6:
                assert np.all(np.abs(out[0]) < 1e-8)
                continue
            h = 1e-5
            fd = np.zeros(3)
            for k in range(3):
                e = np.zeros(3)
                e[k] = h
                Ep = orc.point_ff([r + e], A, probe, g)[0][0, 3]
                Em = orc.point_ff([r - e], A, probe, g)[0][0, 3]
                fd[k] = -(Ep - Em) / (2 * h)
            assert np.allclose(out[0, :3], fd, rtol=1e-6, atol=1e-9), (rho, out[0, :3], fd)


# ---------------------------------------------------------------- interpolation
def _affine_ff(n, step, origin, Amat, b):
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz) * step[2] + origin[2], np.arange(ny) * step[1] + origin[1],
                          np.arange(nx) * step[0] + origin[0], indexing="ij")
    r = np.stack([x, y, z], axis=-1)
    ff = np.zeros((nz, ny, nx, 4))
    ff[..., :3] = r @ Amat.T + b
    return ff


def test_trilinear_exact_for_affine_fields():
    """Sec. 5.1.1: trilinear interpolation reproduces any affine field exactly,
    and its in-cell Jacobian is the field's gradient."""
    rng = np.random.default_rng(2)
    Amat = rng.normal(size=(3, 3))
    b = rng.normal(size=3)
    n, step, origin = (7, 6, 5), (0.1, 0.13, 0.2), (0.5, -0.3, 1.0)
    g = _grid(origin=origin, step=step, n=n)
    ff = _affine_ff(n, step, origin, Amat, b)
    for _ in range(50):
        r = np.array(origin) + rng.uniform(0, 1, 3) * (np.array(n) - 1.001) * np.array(step)
        F, J = orc.interp(ff, g, r, with_jac=True)
        np.testing.assert_allclose(F, Amat @ r + b, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(J, Amat, rtol=1e-10, atol=1e-10)


def test_interp_wrap_clamp_and_nodes():
    """Interpolation returns voxel values at voxels; on a periodic grid it is
    periodic in x,y with period n*step; on an open grid it is constant in x,y
    beyond the edge voxels; in z it is always constant outside the grid.  A
    clamped axis contributes nothing to the Jacobian."""
    rng = np.random.default_rng(4)
    n = (5, 4, 6)
    ff = rng.normal(size=(6, 4, 5, 4))
    for periodic in (0, 1):
        g = _grid(origin=(0, 0, 0), n=n, periodic=periodic, cutoff=0.1)
        for (ix, iy, iz) in [(0, 0, 0), (4, 3, 5), (2, 1, 3)]:
            F = orc.interp(ff, g, [ix * 0.1, iy * 0.1, iz * 0.1])
            np.testing.assert_allclose(F, ff[iz, iy, ix, :3], rtol=1e-14, atol=1e-14)
        below = orc.interp(ff, g, [0.123, 0.257, -0.7])
        at0 = orc.interp(ff, g, [0.123, 0.257, 0.0])
        np.testing.assert_allclose(below, at0, atol=1e-14)
        _, J = orc.interp(ff, g, [0.123, 0.257, 0.9], with_jac=True)
        assert np.all(J[:, 2] == 0.0)
    g = _grid(origin=(0, 0, 0), n=n, periodic=1, cutoff=0.1)
    r = np.array([0.123, 0.257, 0.31])
    F0 = orc.interp(ff, g, r)
    np.testing.assert_allclose(orc.interp(ff, g, r + [0.5, 0.0, 0.0]), F0, atol=1e-14)
    np.testing.assert_allclose(orc.interp(ff, g, r + [0.0, -0.4, 0.0]), F0, atol=1e-14)
    # the periodic cell between the last and the first voxel interpolates them
    F = orc.interp(ff, g, [0.45, 0.1, 0.2])
    np.testing.assert_allclose(F, 0.5 * (ff[2, 1, 4, :3] + ff[2, 1, 0, :3]), atol=1e-14)
    g = _grid(origin=(0, 0, 0), n=n, periodic=0)      # x in [0, 0.4], y in [0, 0.3]
    for out_pt, edge_pt, axis in (((-0.3, 0.1, 0.2), (0.0, 0.1, 0.2), 0),
                                  ((0.7, 0.1, 0.2), (0.4, 0.1, 0.2), 0),
                                  ((0.2, -0.25, 0.2), (0.2, 0.0, 0.2), 1),
                                  ((0.2, 0.5, 0.2), (0.2, 0.3, 0.2), 1)):
        out, J = orc.interp(ff, g, out_pt, with_jac=True)
        np.testing.assert_allclose(out, orc.interp(ff, g, edge_pt), atol=1e-14)
        assert np.all(J[:, axis] == 0.0)


# ---------------------------------------------------------------- tip springs
def test_tip_force_rest_and_potential():
    """Eq. 2: the tip force vanishes at the rest displacement d0 and is minus the
    gradient of (k_R/2)(|d|-R0)^2 + sum_xy (k/2)(d-d0)^2; its Jacobian matches
    central differences."""
    probe = W.Probe(k_lat=(0.02, 0.03), k_rad=1.3, d0=(0.2, -0.1, -3.9))
    anchor = np.array([1.0, 2.0, 9.0])
    F = orc.tip_force(anchor + np.array(probe.d0), anchor, probe)
    assert np.abs(F).max() < 1e-15
    R0 = np.linalg.norm(probe.d0)

    def U(r):
        d = r - anchor
        dd = d - np.array(probe.d0)
        return 0.5 * probe.k_rad * (np.linalg.norm(d) - R0) ** 2 + \
            0.5 * probe.k_lat[0] * dd[0] ** 2 + 0.5 * probe.k_lat[1] * dd[1] ** 2

    rng = np.random.default_rng(1)
    h = 1e-5
    for _ in range(10):
        r = anchor + np.array(probe.d0) + rng.normal(0, 0.4, 3)
        F, J = orc.tip_force(r, anchor, probe, with_jac=True)
        fd = np.array([-(U(r + h * e) - U(r - h * e)) / (2 * h) for e in np.eye(3)])
        np.testing.assert_allclose(F, fd, rtol=1e-7, atol=1e-9)
        Jfd = np.stack([(orc.tip_force(r + h * e, anchor, probe) -
                         orc.tip_force(r - h * e, anchor, probe)) / (2 * h) for e in np.eye(3)], axis=1)
        np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-8)


# ---------------------------------------------------------------- relaxation
def _scan1(x, y, z_top, nz, dz=0.1):
    return W.Scan(x, y, 0.1, 0.1, 1, 1, z_top, dz, nz)


def test_zero_field_rest_position():
    """With no sample force the probe rests at anchor + d0 (Eq. 2), the tip force
    is zero and so is the frequency shift (Eq. 3)."""
    g = _grid(origin=(0, 0, 0), n=(10, 10, 60))
    ff = np.zeros((60, 10, 10, 4))
    scan = W.Scan(0.2, 0.3, 0.1, 0.1, 3, 2, 9.0, 0.1, 15)
    res = orc.relaxed_scan(g, ff, PROBE, W.Fire(), scan)
    anchors = np.array([[0.2 + ix * 0.1, 0.3 + iy * 0.1] for (ix, iy) in res["cols"]])
    np.testing.assert_array_equal(res["r"][:, :, 0], np.repeat(anchors[:, :1], 15, 1))
    np.testing.assert_allclose(res["r"][:, :, 2],
                               np.broadcast_to(9.0 - 0.1 * np.arange(15) - 4.0, (6, 15)), atol=1e-13)
    assert np.all(res["fz"] == 0.0) and np.all(res["iters"] == 0)
    df = orc.df(res["fz"].T, 0.1, W.DfParams())
    assert np.all(df == 0.0)


def test_constant_vertical_field_closed_form():
    """Constant sample force c along +z on a symmetric tip: the radial spring is
    compressed by c/k_R, the probe stays under the anchor and the read-out tip
    force (text after Eq. 2) equals c."""
    c = 0.037
    g = _grid(origin=(0, 0, 0), n=(10, 10, 80))
    ff = np.zeros((80, 10, 10, 4))
    ff[..., 2] = c
    fire = W.parity_fire(W.Fire(), f_conv=1e-9)
    res = orc.relaxed_scan(g, ff, PROBE, fire, _scan1(0.45, 0.55, 9.0, 5), polish_tol=1e-13)
    dz = c / PROBE.k_rad
    np.testing.assert_allclose(res["r"][0, :, 2], 9.0 - 0.1 * np.arange(5) - 4.0 + dz, atol=1e-12)
    np.testing.assert_allclose(res["r"][0, :, :2], [[0.45, 0.55]] * 5, atol=1e-12)
    np.testing.assert_allclose(res["fz"][0], c, rtol=1e-10)


def _newton_equilibrium(anchor, probe, Amat, b, r0):
    """Independent FP64 Newton solve of F^T(r) + (A r + b) = 0 for this test."""
    R0 = np.linalg.norm(probe.d0)
    d0 = np.array(probe.d0)
    k = np.array([probe.k_lat[0], probe.k_lat[1], 0.0])
    r = np.array(r0, float)
    for _ in range(100):
        d = r - anchor
        dn = np.linalg.norm(d)
        G = -probe.k_rad * (dn - R0) * d / dn - k * (d - d0) + Amat @ r + b
        Jt = -probe.k_rad * ((1 - R0 / dn) * np.eye(3) + R0 * np.outer(d, d) / dn ** 3) - np.diag(k)
        r = r - np.linalg.solve(Jt + Amat, G)
    return r


def test_affine_field_equilibrium_matches_newton():
    """A sample force that is affine in r is interpolated exactly, so the relaxed
    probe position must be the root of the analytic force balance (Eq. 1) found by
    an independent Newton iteration -- a pin of FIRE + interpolation + springs."""
    rng = np.random.default_rng(9)
    M = rng.normal(size=(3, 3)) * 0.004
    Amat = -(M @ M.T) - 0.003 * np.eye(3) + (M - M.T) * 0.5   # stable, non-symmetric
    b0 = np.array([0.004, -0.003, 0.02])
    n, step, origin = (40, 40, 60), (0.1, 0.1, 0.1), (0.0, 0.0, 0.0)
    g = _grid(origin=origin, step=step, n=n)
    centre = np.array([2.0, 2.0, 3.0])
    b = b0 - Amat @ centre
    ff = _affine_ff(n, step, origin, Amat, b)
    fire = W.parity_fire(W.Fire(), f_conv=1e-10)
    scan = W.Scan(1.9, 2.05, 0.1, 0.1, 2, 1, 7.1, 0.1, 6)
    res = orc.relaxed_scan(g, ff, PROBE, fire, scan, polish_tol=1e-13)
    for c, (ix, iy) in enumerate(res["cols"]):
        for k in range(6):
            anchor = np.array([1.9 + 0.1 * ix, 2.05 + 0.1 * iy, 7.1 - 0.1 * k])
            rN = _newton_equilibrium(anchor, PROBE, Amat, b, anchor + np.array(PROBE.d0))
            np.testing.assert_allclose(res["r"][c, k], rN, atol=1e-10)


def test_stiff_tip_limit_gives_unrelaxed_force():
    """Eq. 2 with k_lat, k_R -> infinity pins the probe at anchor + d0, so the
    read-out force tends to the sample force there, with an O(1/k) error."""
    rng = np.random.default_rng(12)
    A = W.random_atoms(rng, 5, [1.0, 1.0, -0.3], [3.0, 3.0, 0.3])
    g = _grid(origin=(0, 0, -2.0), n=(40, 40, 90))
    ff = orc.build_ff(g, PROBE, A)
    scan = _scan1(1.83, 2.17, 8.0, 3)
    unrelaxed = np.array([orc.interp(ff, g, [1.83, 2.17, 8.0 - 0.1 * k - 4.0])[2] for k in range(3)])
    errs = []
    for kk in [1e2, 1e3, 1e4]:
        k = kk / 16.02176634
        probe = W.Probe(k_lat=(k, k), k_rad=k)
        fire = W.Fire(dt0=0.1 / math.sqrt(kk / 20), dt_max=0.5 / math.sqrt(kk / 20),
                      f_conv=1e-11, max_iter=200000)
        res = orc.relaxed_scan(g, ff, probe, fire, scan, polish_tol=1e-13)
        errs.append(np.abs(res["fz"][0] - unrelaxed).max())
    assert errs[2] < 1e-2 * np.abs(unrelaxed).max() + 1e-9
    assert errs[1] / errs[2] > 5 and errs[0] / errs[1] > 5       # ~1/k convergence


def test_on_axis_atom_symmetry():
    """A single atom on the tip's vertical axis exerts no lateral force there, so
    the probe stays exactly under the anchor (Eq. 1, Eq. 2); its height solves the
    1-D balance of the radial spring against the interpolated Fz, found here by
    bisection."""
    A = _atoms([[2.0, 2.0, 0.0]], q=[0.1], R=[1.9], eps=[0.0027])
    g = _grid(origin=(0, 0, -2.0), n=(40, 40, 100))
    ff = orc.build_ff(g, PROBE, A)
    fire = W.parity_fire(W.Fire(), f_conv=1e-10)
    res = orc.relaxed_scan(g, ff, PROBE, fire, _scan1(2.0, 2.0, 8.0, 12), polish_tol=1e-13)
    np.testing.assert_allclose(res["r"][0, :, :2], 2.0, atol=1e-12)
    col = ff[:, 20, 20, 2]
    zs = -2.0 + 0.1 * np.arange(100)
    for k in range(12):
        az = 8.0 - 0.1 * k

        def bal(z):
            fs = np.interp(z, zs, col)
            return -PROBE.k_rad * ((az - z) - 4.0) * (-1.0) + fs   # spring_z + sample_z
        lo, hi = az - 4.5, az - 3.5
        assert bal(lo) * bal(hi) < 0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if bal(lo) * bal(mid) <= 0:
                hi = mid
            else:
                lo = mid
        assert res["r"][0, k, 2] == pytest.approx(0.5 * (lo + hi), abs=1e-10)


def test_relaxed_points_are_stable_equilibria():
    """Every relaxed point of a C0-like scan satisfies the force balance of Eq. 1
    to the requested tolerance and is a local minimum (stable)."""
    w = W.config0()
    g = _grid(origin=(4.0, 4.0, -4.0), n=(80, 80, 120))
    ff = orc.build_ff(g, w.probe, w.atoms)
    scan = W.Scan(6.0, 6.0, 0.3, 0.3, 12, 12, 10.0, 0.1, 25)
    res = orc.relaxed_scan(g, ff, w.probe, W.Fire(), scan, with_lambda=True)
    assert np.all(res["iters"] >= 0)
    assert np.all(res["gnorm"] < 1e-4)
    assert np.all(res["lam"] > 0)


# ---------------------------------------------------------------- frequency shift
def test_df_weights_match_adaptive_quadrature():
    """Eq. 3: the weights integrate each piecewise-linear basis (hat) function
    against z / sqrt(a^2 - z^2) on [-a, a].  Substituting z = a sin(t) removes the
    endpoint singularity; scipy's adaptive quadrature of the hat pieces then
    reproduces the weights, also when a is not a multiple of dz."""
    for A, dz in [(1.0, 0.1), (0.7, 0.1), (1.3, 0.17)]:
        a = A / 2
        w = orc.df_weights(A, dz)
        m = (len(w) - 1) // 2
        for j in range(-m, m + 1):
            def f(t, j=j):
                z = a * math.sin(t)
                return a * math.sin(t) * max(0.0, 1.0 - abs(z / dz - j))
            knots = [-math.pi / 2] + [math.asin(max(-1.0, min(1.0, (j + s) * dz / a)))
                                      for s in (-1, 0, 1)] + [math.pi / 2]
            knots = sorted(set(knots))
            val = sum(integrate.quad(f, lo, hi, epsabs=1e-14, epsrel=1e-13, limit=200)[0]
                      for lo, hi in zip(knots[:-1], knots[1:]))
            assert w[j + m] == pytest.approx(val, abs=1e-12), (A, dz, j)


@pytest.mark.parametrize("A,dz", [(1.0, 0.1), (0.7, 0.1), (1.3, 0.17), (2.0, 0.05)])
def test_df_exact_for_linear_and_quadratic(A, dz):
    """Eq. 3 for Fz = a0 + a1 z + a2 z^2 gives exactly -(f0/2k) a1 (the even parts
    integrate to zero against the odd kernel; int z^2/sqrt(a^2-z^2) = pi a^2/2)."""
    dfp = W.DfParams(A=A)
    m = orc.df_m(A, dz)
    nz = 2 * m + 7
    zs = 10.0 - dz * np.arange(nz)                   # scan index 0 = highest
    a0, a1, a2 = 0.3, -0.05, 0.002
    fz = a0 + a1 * zs + a2 * zs ** 2
    out = orc.df(fz, dz, dfp)
    # the interpolation error of the quadratic is a bump that is even about z_c,
    # so it integrates to zero against the odd kernel: the result is exact
    expect = -(dfp.f0 / (2 * dfp.k_cant)) * 16.02176634 * (a1 + 2 * a2 * zs[m:nz - m])
    np.testing.assert_allclose(out, expect, rtol=1e-9)


def test_df_constant_is_zero_and_sign():
    """A constant force has no gradient, so Eq. 3 gives zero; an attractive force
    that strengthens towards the sample (Fz more negative lower down) gives a
    negative frequency shift."""
    dfp = W.DfParams()
    zs = 10.0 - 0.1 * np.arange(30)
    assert np.abs(orc.df(np.full(30, 0.2), 0.1, dfp)).max() < 1e-12
    attractive = -0.01 * np.exp(-(zs - 5.0) / 0.8)
    assert np.all(orc.df(attractive, 0.1, dfp) < 0)


def test_df_exponential_bessel_closed_form():
    """For Fz = F0 exp(-z/lam), Eq. 3 is (f0/2k)(4/A) F0 exp(-z_c/lam) I1(A/(2 lam))
    (a modified Bessel function); the piecewise-linear quadrature converges to it
    at second order in dz."""
    F0, lam = -0.02, 0.5
    dfp = W.DfParams()
    errs = []
    for dz in [0.1, 0.05, 0.025]:
        m = orc.df_m(dfp.A, dz)
        nz = 2 * m + 1
        zc = 4.0
        zs = zc + m * dz - dz * np.arange(nz)
        out = orc.df(F0 * np.exp(-zs / lam), dz, dfp)[0]
        exact = (dfp.f0 / (2 * dfp.k_cant)) * (4 / dfp.A) * F0 * np.exp(-zc / lam) * \
            special.i1(dfp.A / (2 * lam)) * 16.02176634
        errs.append(abs(out - exact) / abs(exact))
    assert errs[0] < 5e-3
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_df_small_amplitude_limit():
    """As A -> 0, Eq. 3 tends to -(f0/2k) dFz/dz."""
    F0, lam, zc = -0.02, 0.5, 4.0
    deriv = -F0 / lam * np.exp(-zc / lam)
    for A in [0.02, 0.01]:
        dfp = W.DfParams(A=A)
        dz = A / 20
        m = orc.df_m(A, dz)
        zs = zc + m * dz - dz * np.arange(2 * m + 1)
        out = orc.df(F0 * np.exp(-zs / lam), dz, dfp)[0]
        ref = -(dfp.f0 / (2 * dfp.k_cant)) * deriv * 16.02176634
        assert out == pytest.approx(ref, rel=5 * (A / (2 * lam)) ** 2)


# ---------------------------------------------------------------- golden fixture
def test_df_weights_golden():
    """Regression fixture for A = 1 A, dz = 0.1 A written by tests/golden/make_golden.py
    (which calls only the oracle); the values themselves are pinned by the
    quadrature test above."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "df_weights_A1.0_dz0.1.txt")
    ref = np.loadtxt(path)
    np.testing.assert_allclose(orc.df_weights(1.0, 0.1), ref, rtol=0, atol=1e-15)


# ---------------------------------------------------------- lateral stiffness
def test_lateral_stiffness_at_rest_and_in_constant_field():
    """Sec. 3.3 lateral-mode stiffness: with no sample force the soft modes are the
    lateral springs (k_x, k_y) of Eq. 2; under a constant vertical force c the
    compressed radial spring adds k_R (1 - R0/|d|), |d| = R0 - c/k_R, to both."""
    probe = W.Probe(k_lat=(0.02, 0.013), k_rad=1.3)
    g = _grid(origin=(0, 0, 0), n=(10, 10, 80))
    anchor = np.array([0.45, 0.55, 9.0])
    ff = np.zeros((80, 10, 10, 4))
    k = orc.lateral_stiffness(g, ff, probe, [anchor], [anchor + np.array(probe.d0)])[0]
    np.testing.assert_allclose(k, [0.013, 0.02], atol=1e-15)
    c = 0.037
    ff[..., 2] = c
    dn = 4.0 - c / probe.k_rad
    r = anchor + np.array([0.0, 0.0, -dn])
    k = orc.lateral_stiffness(g, ff, probe, [anchor], [r])[0]
    shift = probe.k_rad * (1 - 4.0 / dn)
    np.testing.assert_allclose(k, [0.013 + shift, 0.02 + shift], rtol=1e-12)


def test_lateral_stiffness_affine_field_matches_eigvalsh():
    """For an affine sample force A r + b the stiffness matrix is exact:
    -(spring Jacobian) - A; its symmetric part's two smallest eigenvalues equal
    numpy's symmetric eigensolver at the Newton equilibrium."""
    rng = np.random.default_rng(21)
    M = rng.normal(size=(3, 3)) * 0.004
    Amat = -(M @ M.T) - 0.003 * np.eye(3) + (M - M.T) * 0.5
    n, step, origin = (40, 40, 60), (0.1, 0.1, 0.1), (0.0, 0.0, 0.0)
    g = _grid(origin=origin, step=step, n=n)
    b = np.array([0.004, -0.003, 0.02]) - Amat @ np.array([2.0, 2.0, 3.0])
    ff = _affine_ff(n, step, origin, Amat, b)
    anchor = np.array([1.93, 2.07, 7.05])
    r = _newton_equilibrium(anchor, PROBE, Amat, b, anchor + np.array(PROBE.d0))
    d = r - anchor
    dn = np.linalg.norm(d)
    R0 = np.linalg.norm(PROBE.d0)
    Jt = -PROBE.k_rad * ((1 - R0 / dn) * np.eye(3) + R0 * np.outer(d, d) / dn ** 3) - \
        np.diag([PROBE.k_lat[0], PROBE.k_lat[1], 0.0])
    K = -(Jt + Amat)
    ref = np.linalg.eigvalsh(0.5 * (K + K.T))[:2]
    got = orc.lateral_stiffness(g, ff, PROBE, [anchor], [r])[0]
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-14)


# ------------------------------------------------- grading eigenvalue, FIRE path
def test_sym3_min_eig_matches_eigvalsh():
    """The stability measure that decides which relaxed points are graded is the
    smallest eigenvalue of a symmetric 3x3 matrix.  Against numpy's symmetric
    eigensolver and against the eigenvalue each matrix was built with, on random
    spectra and on the hard cases of an iterative solver: two or three equal
    eigenvalues, clusters 1e-10 apart, diagonal and zero matrices, and spreads of
    12 orders of magnitude."""
    rng = np.random.default_rng(2401)
    cases = []
    for i in range(1200):
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        kind = i % 6
        lam = rng.normal(size=3) * 10.0 ** rng.uniform(-3, 2)
        if kind == 1:
            lam[1] = lam[0]                                  # double eigenvalue
        elif kind == 2:
            lam[:] = lam[0]                                  # multiple of the identity
        elif kind == 3:
            lam[1] = lam[0] * (1 + 1e-10)                    # near-degenerate cluster
            lam[2] = lam[0] * (1 - 1e-10)
        elif kind == 4:
            lam = np.array([1e-6, 1.0, 1e6]) * rng.choice([-1, 1], 3)
        elif kind == 5:
            Q = np.eye(3)[rng.permutation(3)]                # already diagonal
        S = (Q * lam) @ Q.T
        S = 0.5 * (S + S.T)
        cases.append((S, lam.min()))
    cases.append((np.zeros((3, 3)), 0.0))
    for S, lmin in cases:
        got = orc.sym3_min_eig(S)
        scale = np.abs(S).max() + 1e-300
        ref = np.linalg.eigvalsh(S)[0]
        assert abs(got - ref) <= 1e-12 * scale, (S, got, ref)
        assert abs(got - lmin) <= 1e-12 * scale, (S, got, lmin)


def _fire_1d(G, fire, z0, dt0):
    """FIRE on a one-dimensional force G(z), written for this test from Bitzek et
    al. 2006: in one dimension a velocity that is parallel to the force stays
    parallel under the mixing step, so the mixing is the identity and the path is
    semi-implicit Euler under FIRE's time-step/alpha schedule alone.  Returns
    (steps, z, dt, resets, increases) with the stopping rule of Sec. 5.1.1's
    relaxation (|G| below the threshold or max_iter steps)."""
    z, v, dt, alpha, npos, it = z0, 0.0, dt0, fire.alpha0, 0, 0
    resets = increases = 0
    g = G(z)
    while not abs(g) < fire.f_conv and it < fire.max_iter:
        if it > 0:
            if g * v > 0.0:
                npos += 1
                if npos > fire.n_min:
                    dt = min(dt * fire.f_inc, fire.dt_max)
                    alpha *= fire.f_alpha
                    increases += 1
            else:
                v, dt, alpha, npos = 0.0, dt * fire.f_dec, fire.alpha0, 0
                resets += 1
        v += g * dt / fire.mass
        z += v * dt
        g = G(z)
        it += 1
    return it, z, dt, resets, increases


def test_fire_trajectory_on_a_one_dimensional_well():
    """Pins FIRE's step counts, not only its fixed points.  On the tip axis of a
    sample force that depends on z alone the probe feels the radial spring of
    Eq. 2 (k_R along z) and the trilinear interpolant of the sample force, which
    there is the piecewise-linear interpolant of the nodal Fz (numpy's interp), so
    the relaxation is one-dimensional.  Every height's step count must equal that
    of an independent one-dimensional FIRE, including the warm start between
    heights (linear extrapolation of the displacement, time step carried over
    and not below dt0), and the positions must agree to rounding."""
    n, step, origin = (12, 12, 140), (0.1, 0.1, 0.1), (0.0, 0.0, 0.0)
    g = _grid(origin=origin, step=step, n=n)
    zs = origin[2] + step[2] * np.arange(n[2])
    node_fz = 0.6 * np.exp(-(zs - 4.0) / 0.35) - 0.12 * np.exp(-(zs - 4.0) / 0.9)   # eV/A
    ff = np.zeros((n[2], n[1], n[0], 4))
    ff[..., 2] = node_fz[:, None, None]
    x, y, z_top, dz, nz = 0.55, 0.45, 11.3, 0.1, 30
    R0 = -PROBE.d0[2]
    for f_conv, max_iter in ((1e-4, 1000), (1e-9, 5000), (1e-4, 7)):
        fire = W.Fire(f_conv=f_conv, max_iter=max_iter)
        res = orc.relaxed_scan(g, ff, PROBE, fire, _scan1(x, y, z_top, nz, dz))
        u1 = u2 = 0.0
        dt = fire.dt0
        resets = increases = 0
        for k in range(nz):
            az = z_top - k * dz
            if k == 0:
                z0 = az - R0
            elif k == 1:
                z0 = az + u1
            else:
                z0 = az + u1 + (u1 - u2)

            def G(z, az=az):
                return float(np.interp(z, zs, node_fz)) + PROBE.k_rad * ((az - z) - R0)
            it, z, dt, nr, ni = _fire_1d(G, fire, z0, max(dt, fire.dt0))
            resets += nr
            increases += ni
            conv = abs(G(z)) < fire.f_conv
            assert res["iters"][0, k] == (it if conv else -it), (f_conv, k, res["iters"][0, k], it)
            assert res["r"][0, k, 2] == pytest.approx(z, abs=1e-11)
            np.testing.assert_array_equal(res["r"][0, k, :2], [x, y])
            u2, u1 = u1, z - az
        # the path exercises both branches of the power test
        assert resets > 0 and increases > 0
        if max_iter == 7:
            assert np.any(res["iters"][0] < 0)
        else:
            assert np.all(res["iters"][0] >= 0) and np.abs(res["iters"][0]).sum() > 150


def test_scan_mirror_and_translation_invariance():
    """The relaxed scan inherits the symmetries of Eq. 1 and Eq. 2 (d0 has no x
    component): mirroring the sample in x about a grid plane, with the tip
    lattice mirrored, mirrors every relaxed position and keeps Fz; moving atoms,
    grid origin and tip lattice together by whole voxels moves every relaxed
    position by the same vector and keeps Fz."""
    rng = np.random.default_rng(17)
    A = W.random_atoms(rng, 6, [1.2, 1.2, -0.3], [3.2, 3.0, 0.3], q_max=0.25)
    n = (45, 42, 90)
    g = _grid(origin=(0.0, 0.0, -2.0), n=n)
    fire = W.parity_fire(W.Fire(), f_conv=1e-10)
    scan = W.Scan(1.37, 1.21, 0.23, 0.19, 7, 6, 7.4, 0.1, 12)
    base = orc.relaxed_scan(g, orc.build_ff(g, PROBE, A), PROBE, fire, scan, polish_tol=1e-13)
    # mirror about the plane through voxel 22 (x = 2.2)
    xc = 2.2
    B = A.copy()
    B.pos[:, 0] = 2 * xc - A.pos[:, 0]
    mscan = W.Scan(2 * xc - (scan.x0 + 6 * scan.dx), scan.y0, scan.dx, scan.dy, 7, 6,
                   scan.z_top, scan.dz, scan.nz)
    mir = orc.relaxed_scan(g, orc.build_ff(g, PROBE, B), PROBE, fire, mscan, polish_tol=1e-13)
    # column (ix, iy) of the base is column (6 - ix, iy) of the mirror
    for c, (ix, iy) in enumerate(base["cols"]):
        cm = np.nonzero((mir["cols"][:, 0] == 6 - ix) & (mir["cols"][:, 1] == iy))[0][0]
        np.testing.assert_allclose(mir["r"][cm, :, 0], 2 * xc - base["r"][c, :, 0], atol=1e-9)
        np.testing.assert_allclose(mir["r"][cm, :, 1:], base["r"][c, :, 1:], atol=1e-9)
        np.testing.assert_allclose(mir["fz"][cm], base["fz"][c], atol=1e-9)
    # translation by whole voxels
    d = np.array([0.4, -0.7, 0.3])
    T = A.copy()
    T.pos = A.pos + d
    tg = _grid(origin=tuple(np.array(g.origin) + d), n=n)
    tscan = W.Scan(scan.x0 + d[0], scan.y0 + d[1], scan.dx, scan.dy, 7, 6, scan.z_top + d[2],
                   scan.dz, scan.nz)
    tr = orc.relaxed_scan(tg, orc.build_ff(tg, PROBE, T), PROBE, fire, tscan, polish_tol=1e-13)
    np.testing.assert_allclose(tr["r"], base["r"] + d, atol=1e-9)
    np.testing.assert_allclose(tr["fz"], base["fz"], atol=1e-9)


def test_scan_quarter_turn_invariance():
    """With equal lateral springs the relaxed scan commutes with a quarter turn
    about a vertical grid line (Eq. 1 and Eq. 2 are isotropic in x, y then):
    turning atoms and the square tip lattice about the line through the centre
    node of a square grid turns every relaxed position and keeps Fz."""
    rng = np.random.default_rng(29)
    A = W.random_atoms(rng, 6, [1.2, 1.2, -0.3], [3.2, 3.2, 0.3], q_max=0.25)
    assert PROBE.k_lat[0] == PROBE.k_lat[1]
    n = (45, 45, 90)
    g = _grid(origin=(0.0, 0.0, -2.0), n=n)
    fire = W.parity_fire(W.Fire(), f_conv=1e-10)
    d = 0.21
    scan = W.Scan(1.37, 1.21, d, d, 7, 6, 7.4, 0.1, 12)
    base = orc.relaxed_scan(g, orc.build_ff(g, PROBE, A), PROBE, fire, scan, polish_tol=1e-13)
    xc = yc = 2.2                                     # node 22 of 0 .. 44
    B = A.copy()
    B.pos[:, 0] = xc - (A.pos[:, 1] - yc)
    B.pos[:, 1] = yc + (A.pos[:, 0] - xc)
    rscan = W.Scan(xc - (scan.y0 + 5 * d - yc), yc + (scan.x0 - xc), d, d, 6, 7, scan.z_top,
                   scan.dz, scan.nz)
    rot = orc.relaxed_scan(g, orc.build_ff(g, PROBE, B), PROBE, fire, rscan, polish_tol=1e-13)
    # column (ix, iy) of the base is column (5 - iy, ix) of the turned scan
    for c, (ix, iy) in enumerate(base["cols"]):
        cr = np.nonzero((rot["cols"][:, 0] == 5 - iy) & (rot["cols"][:, 1] == ix))[0][0]
        np.testing.assert_allclose(rot["r"][cr, :, 0], xc - (base["r"][c, :, 1] - yc), atol=1e-9)
        np.testing.assert_allclose(rot["r"][cr, :, 1], yc + (base["r"][c, :, 0] - xc), atol=1e-9)
        np.testing.assert_allclose(rot["r"][cr, :, 2], base["r"][c, :, 2], atol=1e-9)
        np.testing.assert_allclose(rot["fz"][cr], base["fz"][c], atol=1e-9)


@pytest.mark.parametrize("periodic", [0, 1], ids=["open", "periodic"])
def test_pair_newton_third_law(periodic):
    """Each pair acts on the atom with the opposite of its force on the probe:
    for every atom alone, minus the derivative of the probe's energy with respect
    to the atom's position (central differences) equals minus the force on the
    probe, for the LJ + Coulomb pair and the d_z2 term, with and without the
    periodic minimum image and shifted-force cutoff."""
    rng = np.random.default_rng(23)
    A = W.random_atoms(rng, 5, [0.5, 0.5, -0.3], [5.5, 5.0, 0.3], q_max=0.3)
    g = _grid(origin=(0, 0, 0), n=(60, 56, 40), periodic=periodic, cutoff=2.6 if periodic else 0.0)
    probe = W.Probe(q_zz=-0.07)
    h = 1e-5
    for i in range(A.n):
        one = A.subset([i])
        for r in rng.uniform([0.0, 0.0, 2.2], [6.0, 5.6, 3.5], size=(4, 3)):
            F = orc.point_ff([r], one, probe, g)[0][0, :3]
            dEda = np.zeros(3)
            for k in range(3):
                ap, am = one.copy(), one.copy()
                ap.pos[0, k] += h
                am.pos[0, k] -= h
                dEda[k] = (orc.point_ff([r], ap, probe, g)[0][0, 3] -
                           orc.point_ff([r], am, probe, g)[0][0, 3]) / (2 * h)
            # force on the atom = -dE/da; it must be -F
            np.testing.assert_allclose(-dEda, -F, rtol=1e-6, atol=1e-10)
