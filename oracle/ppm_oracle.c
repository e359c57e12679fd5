/*
 * ppm_oracle.c -- plain FP64 CPU oracle for the probe-particle hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the probe-particle method computes.  It exists to check
 * the HIP path; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or constant
 * with the HIP library, and the HIP library never calls it.
 *
 * Paper: Oinonen et al., "Advancing Scanning Probe Microscopy Simulations:
 * A Decade of Development in Probe-Particle Models" (arXiv 2401.14564).
 *
 *   - per-atom mixing rules ............ Sec. 2.2.1 (Eq. 5), Sec. 2.2.2 (Eq. 6)
 *   - LJ + point-charge energy/force ... Eq. 5, Eq. 6, with F = -grad E (Sec. 2.2);
 *                                        periodic samples: minimum image and a
 *                                        shifted-force cutoff (orc_pair_shift)
 *   - quadrupolar probe charge ......... Sec. 2.2.3 (d_z2 charge of the CO tip,
 *                                        moment -0.025 to -0.15 e A^2)
 *   - grid projection of the force field Sec. 5.1.1, step 1
 *   - trilinear force interpolation .... Sec. 5.1.1, step 2
 *   - tip springs ...................... Sec. 2.1, Eq. 2
 *   - force balance on the probe ....... Sec. 2.1, Eq. 1
 *   - FIRE relaxation .................. Sec. 5.1.1, step 2 (Bitzek et al. 2006)
 *   - tip force readout ................ Sec. 2.1 (text after Eq. 2)
 *   - frequency shift .................. Sec. 2.1, Eq. 3 (Giessibl)
 *   - grid electrostatics .............. Sec. 2.2.3 (cross-correlation of the
 *                                        probe density with the sample
 *                                        potential), Sec. 5.1.2
 *   - implicit adjoint ................. not in the paper; derived here from
 *                                        the equilibrium condition of Eq. 1
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   units A / eV / e; k_e = 14.3996454784 eV*A/e^2; 1 eV/A^2 = 16.02176634 N/m;
 *   d0 points from the anchor down to the probe (z up); voxel (i,j,k) sits at
 *   origin + (i hx, j hy, k hz); interpolation wraps x,y on a periodic grid
 *   and clamps them to the first/last cell otherwise (a sample built without
 *   images has no field to wrap to), and always clamps z;
 *   FIRE parameters are inputs, the first step from rest skips the power test;
 *   convergence is |G|_2 < f_conv; warm start between heights: with
 *   u(k) = r*(k) - anchor(k) the relaxed displacement, the relaxation at height
 *   k starts from anchor(k) + u(k-1) + (u(k-1) - u(k-2)) (linear extrapolation;
 *   anchor(k) + u(k-1) at k = 1, anchor + d0 at k = 0), with v = 0, alpha =
 *   alpha0, and dt = max(the previous height's final dt, dt0); frequency shift
 *   integrates the piecewise-linear interpolant of the Fz samples exactly
 *   ("valid" outputs only).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so ppm_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_KE 14.3996454784          /* e^2/(4 pi eps0), eV*A */
#define ORC_EVA2_IN_NM 16.02176634    /* 1 eV/A^2 in N/m */
#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Parameter packing (this oracle's own convention)                          */
/*   grid  g[8]  = ox, oy, oz, hx, hy, hz, periodic_xy, cutoff ; n[3]         */
/*   probe p[10] = R_pp, eps_pp, q_pp, kx, ky, kR, d0x, d0y, d0z, q_zz        */
/*   fire  f[8]  = dt0, dt_max, f_inc, f_dec, alpha0, f_alpha, mass, f_conv   */
/*         fi[2] = n_min, max_iter                                             */
/*   scan  s[6]  = x0, y0, dx, dy, z_top, dz ; ns[3] = nx, ny, nz             */
/* ------------------------------------------------------------------------ */

/* Mixing rules of Sec. 2.2.1: R_iP = R_i + R_PP, e_iP = sqrt(e_i e_PP);
 * Coulomb prefactor of Eq. 6: kq_i = k_e q_i q_PP; the same for the probe's
 * quadrupole moment: kQ_i = k_e q_i q_zz (kQi may be NULL). */
void orc_mix(int n, const double *R, const double *eps, const double *q,
             const double *p, double *RiP, double *eiP, double *kqi, double *kQi)
{
    for (int i = 0; i < n; ++i) {
        RiP[i] = R[i] + p[0];
        eiP[i] = sqrt(eps[i] * p[1]);
        kqi[i] = ORC_KE * q[i] * p[2];
        if (kQi) kQi[i] = ORC_KE * q[i] * p[9];
    }
}

/* Displacement d = r - a, with the minimum image in x,y when periodic. */
static void orc_disp(const double *r, const double *a, const double *g,
                     const int *n, double *d)
{
    d[0] = r[0] - a[0];
    d[1] = r[1] - a[1];
    d[2] = r[2] - a[2];
    if (g[6] != 0.0) {
        double Lx = n[0] * g[3], Ly = n[1] * g[4];
        d[0] -= Lx * nearbyint(d[0] / Lx);
        d[1] -= Ly * nearbyint(d[1] / Ly);
    }
}

/*
 * Quadrupolar probe charge (Sec. 2.2.3).  The paper gives the moment of the
 * CO tip's d_z2 charge (in e A^2) but no convention; this oracle reads it as
 * the point density rho_PP = q_zz d^2 delta / dz^2, i.e. the limit h -> 0 of
 * charges (+q, -2q, +q) at z + h, z, z - h with q h^2 = q_zz.  Its energy in
 * the potential V_i = k_e q_i / |r - r_i| of atom i is the cross-correlation
 * of Sec. 2.2.3 with this density:
 *   E_i = q_zz d^2 V_i / dz^2 = kQ_i (3 dz^2 - rho^2) / rho^5,  kQ_i = k_e q_i q_zz,
 * and F_i = -grad E_i = kQ_i / rho^5 [ (15 dz^2 / rho^2 - 3) d - 6 dz e_z ].
 */
static void orc_quad(double kQ, const double *d, double rho2, double *E, double *F,
                     double *sE, double *sF)
{
    double rho = sqrt(rho2);
    double ir5 = 1.0 / (rho2 * rho2 * rho);
    double z = d[2];
    double c = 15.0 * z * z / rho2 - 3.0;
    *E += kQ * (3.0 * z * z - rho2) * ir5;
    F[0] += kQ * ir5 * c * d[0];
    F[1] += kQ * ir5 * c * d[1];
    F[2] += kQ * ir5 * (c * d[2] - 6.0 * z);
    *sE += fabs(kQ) * (3.0 * z * z + rho2) * ir5;
    *sF += fabs(kQ) * ir5 * ((15.0 * z * z / rho2 + 3.0) * rho + 6.0 * fabs(z));
}

/*
 * Shifted-force truncation at the cutoff rc of a periodic sample.  A pair term
 * of the form Y(direction) g(rho) is replaced by Y(direction) g_sf(rho) with
 *   g_sf(rho) = g(rho) - g(rc) - (rho - rc) g'(rc)   for rho < rc, 0 beyond,
 * so that the term and its force both vanish on the cutoff sphere (a plain
 * truncation leaves a force step there on every charged atom's sphere).  For
 * the LJ + Coulomb pair (Y = 1) this adds -U(rc) + (rho - rc) f(rc) to the
 * energy, with f = -dU/drho, and -f(rc) d/rho to the force.  For the d_z2 term
 * (Y = 3 dz^2/rho^2 - 1, g = rho^-3) it adds Y (3 rho rc^-4 - 4 rc^-3) to
 * u = (3 dz^2 - rho^2)/rho^5, whose gradient is written out below.
 */
static void orc_pair_shift(double e, double Rp, double kq, double rc, double rho,
                           const double *d, double *E, double *F, double *sE, double *sF)
{
    double sc = Rp / rc, sc6 = pow(sc, 6.0), sc12 = sc6 * sc6;
    double Uc = e * (sc12 - 2.0 * sc6) + kq / rc;
    double fc = 12.0 * e * (sc12 - sc6) / rc + kq / (rc * rc);
    *E += -Uc + (rho - rc) * fc;
    for (int t = 0; t < 3; ++t) F[t] -= fc * d[t] / rho;
    *sE += fabs(Uc) + fabs(fc) * (rc + rho);
    *sF += fabs(fc);
}

static void orc_quad_shift(double kQ, double rc, const double *d, double rho2, double *E,
                           double *F, double *sE, double *sF)
{
    double rho = sqrt(rho2), z = d[2];
    double Y = 3.0 * z * z / rho2 - 1.0;
    double irc3 = 1.0 / (rc * rc * rc), irc4 = irc3 / rc;
    *E += kQ * Y * (3.0 * rho * irc4 - 4.0 * irc3);
    /* grad of Y (3 rho rc^-4 - 4 rc^-3) = ax d + bx e_z */
    double ax = -9.0 * irc4 * z * z / (rho2 * rho) + 24.0 * irc3 * z * z / (rho2 * rho2)
                - 3.0 * irc4 / rho;
    double bx = 18.0 * irc4 * z / rho - 24.0 * irc3 * z / rho2;
    F[0] -= kQ * ax * d[0];
    F[1] -= kQ * ax * d[1];
    F[2] -= kQ * (ax * d[2] + bx);
    /* magnitude sums of the separate terms (rounding scale) */
    *sE += fabs(kQ) * (9.0 * irc4 * z * z / rho + 12.0 * irc3 * z * z / rho2
                       + 3.0 * irc4 * rho + 4.0 * irc3);
    *sF += fabs(kQ) * ((9.0 * irc4 * z * z / (rho2 * rho) + 24.0 * irc3 * z * z / (rho2 * rho2)
                        + 3.0 * irc4 / rho) * rho
                       + 18.0 * irc4 * fabs(z) / rho + 24.0 * irc3 * fabs(z) / rho2);
}

/*
 * Energy and force on the probe particle at point r from all atoms
 * (Eq. 5 + Eq. 6, F = -grad E):
 *   E   = sum_i e_iP [ (R_iP/rho)^12 - 2 (R_iP/rho)^6 ] + kq_i / rho
 *   F   = sum_i { 12 e_iP [ (R_iP/rho)^12 - (R_iP/rho)^6 ] / rho^2 + kq_i / rho^3 } (r - r_i)
 * plus the quadrupole term of orc_quad when kQi != NULL.
 * out[4] = Fx, Fy, Fz, E.  If scale != NULL it receives the magnitude sums of
 * every term that enters the sums (the scale of their rounding error):
 * scale[0] = sum_i [12 e_iP ((R/rho)^12 + (R/rho)^6)/rho^2 + |kq_i|/rho^3] rho,
 * scale[1] = sum_i e_iP ((R/rho)^12 + 2 (R/rho)^6) + |kq_i|/rho,
 * (each plus the quadrupole's magnitude bound), scale[2] = min rho,
 * scale[3] = min |rho^2 - rc^2|.
 * With periodic_xy only pairs with rho^2 < rc^2 contribute, each shifted so
 * that it and its force vanish at rc (orc_pair_shift, orc_quad_shift).
 */
void orc_point(const double *r, int na, const double *pos, const double *RiP,
               const double *eiP, const double *kqi, const double *kQi, const double *g,
               const int *n, double *out, double *scale)
{
    double E = 0, Fx = 0, Fy = 0, Fz = 0, sF = 0, sE = 0, rmin = 1e300, tie = 1e300;
    int periodic = g[6] != 0.0;
    double rc2 = g[7] * g[7];
    for (int i = 0; i < na; ++i) {
        double d[3];
        orc_disp(r, pos + 3 * i, g, n, d);
        double rho2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (periodic) {
            double t = fabs(rho2 - rc2);
            if (t < tie) tie = t;
            if (!(rho2 < rc2)) continue;
        }
        double rho = sqrt(rho2);
        if (rho < rmin) rmin = rho;
        double s = RiP[i] / rho;
        double s6 = pow(s, 6.0);
        double s12 = s6 * s6;
        double eLJ = eiP[i] * (s12 - 2.0 * s6);
        double eC = kqi[i] / rho;
        double phi = 12.0 * eiP[i] * (s12 - s6) / rho2 + kqi[i] / (rho2 * rho);
        E += eLJ + eC;
        Fx += phi * d[0];
        Fy += phi * d[1];
        Fz += phi * d[2];
        sF += (12.0 * eiP[i] * (s12 + s6) / rho2 + fabs(kqi[i]) / (rho2 * rho)) * rho;
        sE += eiP[i] * (s12 + 2.0 * s6) + fabs(eC);
        if (periodic) {
            double Fs[3] = { 0.0, 0.0, 0.0 };
            orc_pair_shift(eiP[i], RiP[i], kqi[i], g[7], rho, d, &E, Fs, &sE, &sF);
            Fx += Fs[0]; Fy += Fs[1]; Fz += Fs[2];
        }
        if (kQi && kQi[i] != 0.0) {
            double Fq[3] = { 0.0, 0.0, 0.0 };
            orc_quad(kQi[i], d, rho2, &E, Fq, &sE, &sF);
            if (periodic) orc_quad_shift(kQi[i], g[7], d, rho2, &E, Fq, &sE, &sF);
            Fx += Fq[0]; Fy += Fq[1]; Fz += Fq[2];
        }
    }
    out[0] = Fx; out[1] = Fy; out[2] = Fz; out[3] = E;
    if (scale) { scale[0] = sF; scale[1] = sE; scale[2] = rmin; scale[3] = tie; }
}

/*
 * Grid projection (Sec. 5.1.1, step 1): the force field at every voxel of
 * z-slab [iz0, iz1).  ff is [iz1-iz0][ny][nx][4] (Fx,Fy,Fz,E), scale (may be
 * NULL) is [iz1-iz0][ny][nx][4] as in orc_point.
 */
void orc_build_ff(const double *g, const int *n, const double *p, int na,
                  const double *pos, const double *q, const double *R,
                  const double *eps, int iz0, int iz1, double *ff, double *scale)
{
    double *RiP = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *eiP = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *kqi = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *kQi = malloc(sizeof(double) * (na > 0 ? na : 1));
    orc_mix(na, R, eps, q, p, RiP, eiP, kqi, kQi);
    int nx = n[0], ny = n[1];
    #pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int iz = iz0; iz < iz1; ++iz)
        for (int iy = 0; iy < ny; ++iy)
            for (int ix = 0; ix < nx; ++ix) {
                double r[3] = { g[0] + ix * g[3], g[1] + iy * g[4], g[2] + iz * g[5] };
                size_t o = (((size_t)(iz - iz0) * ny + iy) * nx + ix) * 4;
                orc_point(r, na, pos, RiP, eiP, kqi, kQi, g, n, ff + o,
                          scale ? scale + o : NULL);
            }
    free(RiP); free(eiP); free(kqi); free(kQi);
}

/* Same as orc_point for a list of voxel indices idx[m][3] (sampled checks). */
void orc_ff_voxels(const double *g, const int *n, const double *p, int na,
                   const double *pos, const double *q, const double *R,
                   const double *eps, int m, const int *idx, double *out, double *scale)
{
    double *RiP = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *eiP = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *kqi = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *kQi = malloc(sizeof(double) * (na > 0 ? na : 1));
    orc_mix(na, R, eps, q, p, RiP, eiP, kqi, kQi);
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < m; ++k) {
        double r[3] = { g[0] + idx[3 * k] * g[3], g[1] + idx[3 * k + 1] * g[4],
                        g[2] + idx[3 * k + 2] * g[5] };
        orc_point(r, na, pos, RiP, eiP, kqi, kQi, g, n, out + 4 * (size_t)k,
                  scale ? scale + 4 * (size_t)k : NULL);
    }
    free(RiP); free(eiP); free(kqi); free(kQi);
}

/* ------------------------------------------------------------------------ */
/* Trilinear interpolation of the force components (Sec. 5.1.1, step 2)      */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ix[2], iy[2], iz[2];     /* voxel indices of the cell corners */
    double tx, ty, tz;           /* fractional position inside the cell */
    int xin, yin, zin;           /* 0 when the axis was clamped (field constant along it) */
} orc_cell;

static int orc_wrap(long i, int n)
{
    long m = i % n;
    return (int)(m < 0 ? m + n : m);
}

/* Cell of grid coordinate u on an axis of n points clamped to the first/last
 * cell: outside the grid the field is continued constantly. */
static int orc_clamp_cell(double u, int n, double *t, int *in)
{
    double f = floor(u);
    *in = 1;
    if (f < 0) { *t = 0.0; *in = 0; return 0; }
    if (f > n - 2) { *t = 1.0; *in = 0; return n - 2; }
    *t = u - f;
    return (int)f;
}

static void orc_locate(const double *g, const int *n, const double *r, orc_cell *c)
{
    double ux = (r[0] - g[0]) / g[3];
    double uy = (r[1] - g[1]) / g[4];
    double uz = (r[2] - g[2]) / g[5];
    if (g[6] != 0.0) {
        /* periodic in x,y: wrap */
        double fx = floor(ux), fy = floor(uy);
        c->tx = ux - fx;
        c->ty = uy - fy;
        c->ix[0] = orc_wrap((long)fx, n[0]); c->ix[1] = orc_wrap((long)fx + 1, n[0]);
        c->iy[0] = orc_wrap((long)fy, n[1]); c->iy[1] = orc_wrap((long)fy + 1, n[1]);
        c->xin = c->yin = 1;
    } else {
        int i = orc_clamp_cell(ux, n[0], &c->tx, &c->xin);
        int j = orc_clamp_cell(uy, n[1], &c->ty, &c->yin);
        c->ix[0] = i; c->ix[1] = i + 1;
        c->iy[0] = j; c->iy[1] = j + 1;
    }
    int k = orc_clamp_cell(uz, n[2], &c->tz, &c->zin);
    c->iz[0] = k; c->iz[1] = k + 1;
}

static const double *orc_vox(const double *ff, const int *n, int ix, int iy, int iz)
{
    return ff + (((size_t)iz * n[1] + iy) * n[0] + ix) * 4;
}

/* F^S_h(r): trilinear interpolation of (Fx,Fy,Fz).  If jac != NULL also the
 * in-cell derivative jac[a][b] = dF_a/dr_b. */
void orc_interp(const double *ff, const double *g, const int *n, const double *r,
                double *F, double *jac)
{
    orc_cell c;
    orc_locate(g, n, r, &c);
    double wx[2] = { 1.0 - c.tx, c.tx }, wy[2] = { 1.0 - c.ty, c.ty },
           wz[2] = { 1.0 - c.tz, c.tz };
    double dwx[2] = { -1.0 / g[3], 1.0 / g[3] }, dwy[2] = { -1.0 / g[4], 1.0 / g[4] },
           dwz[2] = { -1.0 / g[5], 1.0 / g[5] };
    if (!c.xin) { dwx[0] = 0.0; dwx[1] = 0.0; }
    if (!c.yin) { dwy[0] = 0.0; dwy[1] = 0.0; }
    if (!c.zin) { dwz[0] = 0.0; dwz[1] = 0.0; }
    F[0] = F[1] = F[2] = 0.0;
    if (jac) for (int k = 0; k < 9; ++k) jac[k] = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int cc = 0; cc < 2; ++cc) {
                const double *v = orc_vox(ff, n, c.ix[a], c.iy[b], c.iz[cc]);
                double w = wx[a] * wy[b] * wz[cc];
                double w_x = dwx[a] * wy[b] * wz[cc];
                double w_y = wx[a] * dwy[b] * wz[cc];
                double w_z = wx[a] * wy[b] * dwz[cc];
                for (int k = 0; k < 3; ++k) {
                    F[k] += w * v[k];
                    if (jac) {
                        jac[3 * k + 0] += w_x * v[k];
                        jac[3 * k + 1] += w_y * v[k];
                        jac[3 * k + 2] += w_z * v[k];
                    }
                }
            }
}

/* ------------------------------------------------------------------------ */
/* Tricubic interpolation of the potential (Sec. 5.1.1, step 2: the variant   */
/* the paper is experimenting with -- store only E, interpolate it with a      */
/* cubic in each direction and take the force as minus its gradient).          */
/* Reading: Catmull-Rom cubic convolution (Keys, a = -1/2) on the 4-point      */
/* stencil i-1..i+2 per axis; x,y wrap on a periodic grid; otherwise (and     */
/* always for z) the point is clamped to the grid box: outside [0, n-1] the    */
/* force is continued constantly along that axis, as the trilinear field is   */
/* (the energy reported there is the value at the clamped point).             */
/* ------------------------------------------------------------------------ */

/* Catmull-Rom basis for the stencil offsets -1, 0, 1, 2 at fraction t, with
 * first (dw) and second (d2w) derivatives with respect to t. */
static void orc_cr_weights(double t, double *w, double *dw, double *d2w)
{
    double t2 = t * t, t3 = t2 * t;
    w[0] = 0.5 * (-t3 + 2.0 * t2 - t);
    w[1] = 0.5 * (3.0 * t3 - 5.0 * t2 + 2.0);
    w[2] = 0.5 * (-3.0 * t3 + 4.0 * t2 + t);
    w[3] = 0.5 * (t3 - t2);
    dw[0] = 0.5 * (-3.0 * t2 + 4.0 * t - 1.0);
    dw[1] = 0.5 * (9.0 * t2 - 10.0 * t);
    dw[2] = 0.5 * (-9.0 * t2 + 8.0 * t + 1.0);
    dw[3] = 0.5 * (3.0 * t2 - 2.0 * t);
    d2w[0] = 0.5 * (-6.0 * t + 4.0);
    d2w[1] = 0.5 * (18.0 * t - 10.0);
    d2w[2] = 0.5 * (-18.0 * t + 8.0);
    d2w[3] = 0.5 * (6.0 * t - 2.0);
}

/* Interpolated energy E, force F = -grad E and (if hess != NULL) the Hessian
 * of E at r, from the energy grid En[nz][ny][nx]. */
void orc_interp_tricubic(const double *En, const double *g, const int *n, const double *r,
                         double *E, double *F, double *hess)
{
    double u[3] = { (r[0] - g[0]) / g[3], (r[1] - g[1]) / g[4], (r[2] - g[2]) / g[5] };
    int periodic = g[6] != 0.0;
    int in[3] = { 1, 1, 1 };
    for (int a = 0; a < 3; ++a) {
        if (a < 2 && periodic) continue;
        if (u[a] < 0.0) { u[a] = 0.0; in[a] = 0; }
        if (u[a] > n[a] - 1) { u[a] = n[a] - 1; in[a] = 0; }
    }
    int base[3];
    double t[3], w[3][4], dw[3][4], d2w[3][4];
    for (int a = 0; a < 3; ++a) {
        double f = floor(u[a]);
        if ((a == 2 || !periodic) && f > n[a] - 2) f = n[a] - 2;   /* top node: last cell, t = 1 */
        base[a] = (int)f;
        t[a] = u[a] - f;
        orc_cr_weights(t[a], w[a], dw[a], d2w[a]);
    }
    int ix[4], iy[4], iz[4];
    for (int s = 0; s < 4; ++s) {
        int x = base[0] + s - 1, y = base[1] + s - 1, z = base[2] + s - 1;
        if (periodic) {
            ix[s] = orc_wrap((long)x, n[0]);
            iy[s] = orc_wrap((long)y, n[1]);
        } else {
            ix[s] = x < 0 ? 0 : (x > n[0] - 1 ? n[0] - 1 : x);
            iy[s] = y < 0 ? 0 : (y > n[1] - 1 ? n[1] - 1 : y);
        }
        iz[s] = z < 0 ? 0 : (z > n[2] - 1 ? n[2] - 1 : z);
    }
    double h[3] = { g[3], g[4], g[5] };
    double e = 0, gr[3] = { 0, 0, 0 }, H[9] = { 0 };
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c) {
                double v = En[((size_t)iz[c] * n[1] + iy[b]) * n[0] + ix[a]];
                e += w[0][a] * w[1][b] * w[2][c] * v;
                gr[0] += dw[0][a] * w[1][b] * w[2][c] * v;
                gr[1] += w[0][a] * dw[1][b] * w[2][c] * v;
                gr[2] += w[0][a] * w[1][b] * dw[2][c] * v;
                if (hess) {
                    H[0] += d2w[0][a] * w[1][b] * w[2][c] * v;
                    H[4] += w[0][a] * d2w[1][b] * w[2][c] * v;
                    H[8] += w[0][a] * w[1][b] * d2w[2][c] * v;
                    H[1] += dw[0][a] * dw[1][b] * w[2][c] * v;
                    H[2] += dw[0][a] * w[1][b] * dw[2][c] * v;
                    H[5] += w[0][a] * dw[1][b] * dw[2][c] * v;
                }
            }
    *E = e;
    for (int a = 0; a < 3; ++a) F[a] = -gr[a] / h[a];
    if (hess) {
        /* hess[a][b] = -dF_a/dx_b: the Hessian of the interpolant at the clamped
         * point, with the columns of clamped axes zero (the force does not
         * change along them); not symmetric then */
        H[3] = H[1]; H[6] = H[2]; H[7] = H[5];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                hess[3 * a + b] = in[b] ? H[3 * a + b] / (h[a] * h[b]) : 0.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Tip springs (Sec. 2.1, Eq. 2)                                              */
/*   F^T = -k_R (|d| - R0) d/|d| - k_xy (.) (d - d0),  d = r - r_TIP          */
/* ------------------------------------------------------------------------ */
void orc_tip_force(const double *r, const double *anchor, const double *p,
                   double *F, double *jac)
{
    double d[3] = { r[0] - anchor[0], r[1] - anchor[1], r[2] - anchor[2] };
    double R0 = sqrt(p[6] * p[6] + p[7] * p[7] + p[8] * p[8]);
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double kR = p[5];
    double fr = -kR * (dn - R0) / dn;
    F[0] = fr * d[0] - p[3] * (d[0] - p[6]);
    F[1] = fr * d[1] - p[4] * (d[1] - p[7]);
    F[2] = fr * d[2];
    if (jac) {
        /* d/dd [ (|d|-R0) d/|d| ] = (1 - R0/|d|) I + R0 d d^T / |d|^3 */
        double a = 1.0 - R0 / dn, b = R0 / (dn * dn * dn);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                jac[3 * i + j] = -kR * ((i == j ? a : 0.0) + b * d[i] * d[j]);
        jac[0] -= p[3];
        jac[4] -= p[4];
    }
}

/* Net force on the probe particle (Eq. 1): G = F^T + F^S_h.  Returns |G|. */
static double orc_net(const double *ff, const double *g, const int *n, const double *p,
                      const double *anchor, const double *r, double *G, double *J)
{
    double Ft[3], Fs[3], Jt[9], Js[9];
    orc_tip_force(r, anchor, p, Ft, J ? Jt : NULL);
    orc_interp(ff, g, n, r, Fs, J ? Js : NULL);
    for (int k = 0; k < 3; ++k) G[k] = Ft[k] + Fs[k];
    if (J) for (int k = 0; k < 9; ++k) J[k] = Jt[k] + Js[k];
    return sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
}

/* Net force with the tricubic potential (ff holds the energy grid). */
static double orc_net_tc(const double *En, const double *g, const int *n, const double *p,
                         const double *anchor, const double *r, double *G, double *J)
{
    double Ft[3], Fs[3], Jt[9], Hs[9], E;
    orc_tip_force(r, anchor, p, Ft, J ? Jt : NULL);
    orc_interp_tricubic(En, g, n, r, &E, Fs, J ? Hs : NULL);
    for (int k = 0; k < 3; ++k) G[k] = Ft[k] + Fs[k];
    if (J) for (int k = 0; k < 9; ++k) J[k] = Jt[k] - Hs[k];   /* dF^S/dr = -Hessian */
    return sqrt(G[0] * G[0] + G[1] * G[1] + G[2] * G[2]);
}

/* Interpolation mode of the relaxation: 0 trilinear forces, 1 tricubic potential. */
static double orc_net_mode(int mode, const double *ff, const double *g, const int *n,
                           const double *p, const double *anchor, const double *r, double *G,
                           double *J)
{
    return mode ? orc_net_tc(ff, g, n, p, anchor, r, G, J)
                : orc_net(ff, g, n, p, anchor, r, G, J);
}

/* Solve the 3x3 system A x = b by Cramer's rule; returns 0 if singular. */
static int orc_solve3(const double *A, const double *b, double *x)
{
    double c00 = A[4] * A[8] - A[5] * A[7];
    double c01 = A[5] * A[6] - A[3] * A[8];
    double c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    if (!(fabs(det) > 1e-300)) return 0;
    double inv[9];
    inv[0] = c00 / det;
    inv[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    inv[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    inv[3] = c01 / det;
    inv[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    inv[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    inv[6] = c02 / det;
    inv[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    inv[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    for (int i = 0; i < 3; ++i)
        x[i] = inv[3 * i] * b[0] + inv[3 * i + 1] * b[1] + inv[3 * i + 2] * b[2];
    return 1;
}

/* Smallest eigenvalue of a symmetric 3x3 matrix (cyclic Jacobi rotations). */
double orc_sym3_min_eig(const double *S_in)
{
    double a[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a[i][j] = S_in[3 * i + j];
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        if (off < 1e-300) break;
        for (int pp = 0; pp < 2; ++pp)
            for (int qq = pp + 1; qq < 3; ++qq) {
                if (a[pp][qq] == 0.0) continue;
                double theta = (a[qq][qq] - a[pp][pp]) / (2.0 * a[pp][qq]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {   /* columns */
                    double akp = a[k][pp], akq = a[k][qq];
                    a[k][pp] = cs * akp - sn * akq;
                    a[k][qq] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {   /* rows */
                    double apk = a[pp][k], aqk = a[qq][k];
                    a[pp][k] = cs * apk - sn * aqk;
                    a[qq][k] = sn * apk + cs * aqk;
                }
            }
    }
    double m = a[0][0];
    if (a[1][1] < m) m = a[1][1];
    if (a[2][2] < m) m = a[2][2];
    return m;
}

/*
 * FIRE relaxation of the probe particle (Bitzek et al. 2006), as the paper's
 * relaxation step uses it.  State r, v; one step:
 *   (from the second step on) P = G.v ;
 *       P > 0 : v <- (1-alpha) v + alpha |v| G/|G| ; after more than n_min
 *               consecutive such steps dt <- min(dt f_inc, dt_max), alpha <- alpha f_alpha
 *       P <= 0: v <- 0, dt <- dt f_dec, alpha <- alpha0
 *   semi-implicit Euler: v += G dt/m ; r += v dt ; re-evaluate G.
 * Stops when |G| < f_conv or after max_iter steps.  Returns the number of
 * steps taken, negated if not converged.  dt_io: the initial time step on
 * entry, the final one on return.
 */
static int orc_fire(int mode, const double *ff, const double *g, const int *n,
                    const double *p, const double *f, const int *fi, const double *anchor,
                    double *r, double *gnorm, double *dt_io)
{
    double v[3] = { 0, 0, 0 }, G[3];
    double dt = *dt_io, alpha = f[4];
    int npos = 0;
    double gn = orc_net_mode(mode, ff, g, n, p, anchor, r, G, NULL);
    int it = 0;
    while (!(gn < f[7]) && it < fi[1]) {
        if (it > 0) {
            double P = G[0] * v[0] + G[1] * v[1] + G[2] * v[2];
            if (P > 0.0) {
                double vn = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                for (int k = 0; k < 3; ++k)
                    v[k] = (1.0 - alpha) * v[k] + alpha * vn * G[k] / gn;
                ++npos;
                if (npos > fi[0]) {
                    dt = fmin(dt * f[2], f[1]);
                    alpha *= f[5];
                }
            } else {
                v[0] = v[1] = v[2] = 0.0;
                dt *= f[3];
                alpha = f[4];
                npos = 0;
            }
        }
        for (int k = 0; k < 3; ++k) {
            v[k] += G[k] * dt / f[6];
            r[k] += v[k] * dt;
        }
        gn = orc_net_mode(mode, ff, g, n, p, anchor, r, G, NULL);
        ++it;
    }
    *gnorm = gn;
    *dt_io = dt;
    return gn < f[7] ? it : -it;
}

/* Newton refinement of an equilibrium with the exact piecewise Jacobian and a
 * backtracking line search on |G|; used only to make the oracle's equilibria
 * exact to ~1e-12 eV/A so that they serve as the expected value. */
static double orc_polish(int mode, const double *ff, const double *g, const int *n,
                         const double *p, const double *anchor, double *r, double tol)
{
    double G[3], J[9];
    double gn = orc_net_mode(mode, ff, g, n, p, anchor, r, G, J);
    for (int iter = 0; iter < 60 && gn >= tol; ++iter) {
        double mg[3] = { -G[0], -G[1], -G[2] }, dlt[3];
        if (!orc_solve3(J, mg, dlt)) break;
        double s = 1.0;
        int ok = 0;
        double rt[3], Gt[3], Jt[9], gt = 0;
        for (int b = 0; b < 40; ++b) {
            for (int k = 0; k < 3; ++k) rt[k] = r[k] + s * dlt[k];
            gt = orc_net_mode(mode, ff, g, n, p, anchor, rt, Gt, Jt);
            if (gt < gn) { ok = 1; break; }
            s *= 0.5;
        }
        if (!ok) break;
        memcpy(r, rt, sizeof rt);
        memcpy(G, Gt, sizeof Gt);
        memcpy(J, Jt, sizeof Jt);
        gn = gt;
    }
    return gn;
}

/* Stability measure at r: smallest eigenvalue of sym(-dG/dr). */
static double orc_lambda_min(int mode, const double *ff, const double *g, const int *n,
                             const double *p, const double *anchor, const double *r)
{
    double G[3], J[9], S[9];
    orc_net_mode(mode, ff, g, n, p, anchor, r, G, J);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S[3 * i + j] = -0.5 * (J[3 * i + j] + J[3 * j + i]);
    return orc_sym3_min_eig(S);
}

/*
 * Relaxed scan (Sec. 2.1 and Sec. 5.1.1): every tip column descends in z
 * independently.  Column c = cols[c] (ix, iy) of the tip lattice, anchor
 * (x0 + ix dx, y0 + iy dy, z_top - k dz) for k = 0 .. nz-1.  With the
 * displacement u(k) = r*(k) - anchor(k), the probe starts at anchor + d0 at
 * k = 0, at anchor(1) + u(0) at k = 1 and at anchor(k) + u(k-1) + (u(k-1) -
 * u(k-2)) from k = 2 on (linear extrapolation), always from rest; the FIRE time
 * step carries over from the previous height, not below dt0.
 * FIRE relaxes G = F^T + F^S_h to |G| < f_conv; with polish_tol > 0 the result
 * is then Newton-refined to |G| < polish_tol.
 * Readout (text after Eq. 2): Fz_tip = -F^T_z at the relaxed position.
 * Outputs per (column, k) (index (c * nz + k)):
 *   r_out[3], fz_out, iters_out (negative = not converged), gnorm_out,
 *   lam_out (smallest eigenvalue of sym(-dG/dr); NULL to skip).
 */
static void orc_relaxed_scan_mode(int mode, const double *g, const int *n, const double *ff,
                                  const double *p, const double *f, const int *fi,
                                  const double *s, const int *ns, int ncols, const int *cols,
                                  double polish_tol, double *r_out, double *fz_out,
                                  int *iters_out, double *gnorm_out, double *lam_out)
{
    int nz = ns[2];
    #pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < ncols; ++c) {
        int ix = cols[2 * c], iy = cols[2 * c + 1];
        double anchor[3] = { s[0] + ix * s[2], s[1] + iy * s[3], s[4] };
        double r[3] = { anchor[0] + p[6], anchor[1] + p[7], anchor[2] + p[8] };
        double u1[3] = { 0, 0, 0 }, u2[3] = { 0, 0, 0 };   /* u(k-1), u(k-2) */
        double dt = f[0];
        for (int k = 0; k < nz; ++k) {
            double az = s[4] - k * s[5];
            anchor[2] = az;
            if (k == 1)
                for (int q = 0; q < 3; ++q) r[q] = anchor[q] + u1[q];
            else if (k >= 2)
                for (int q = 0; q < 3; ++q) r[q] = anchor[q] + u1[q] + (u1[q] - u2[q]);
            dt = fmax(dt, f[0]);
            double gn;
            int it = orc_fire(mode, ff, g, n, p, f, fi, anchor, r, &gn, &dt);
            if (polish_tol > 0.0) gn = orc_polish(mode, ff, g, n, p, anchor, r, polish_tol);
            double Ft[3];
            orc_tip_force(r, anchor, p, Ft, NULL);
            size_t o = (size_t)c * nz + k;
            r_out[3 * o] = r[0]; r_out[3 * o + 1] = r[1]; r_out[3 * o + 2] = r[2];
            fz_out[o] = -Ft[2];
            iters_out[o] = it;
            gnorm_out[o] = gn;
            if (lam_out) lam_out[o] = orc_lambda_min(mode, ff, g, n, p, anchor, r);
            for (int q = 0; q < 3; ++q) { u2[q] = u1[q]; u1[q] = r[q] - anchor[q]; }
        }
    }
}

/* All three eigenvalues of a symmetric 3x3 matrix, ascending (cyclic Jacobi). */
static void orc_sym3_eigs(const double *S_in, double *ev)
{
    double a[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) a[i][j] = S_in[3 * i + j];
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = fabs(a[0][1]) + fabs(a[0][2]) + fabs(a[1][2]);
        if (off < 1e-300) break;
        for (int pp = 0; pp < 2; ++pp)
            for (int qq = pp + 1; qq < 3; ++qq) {
                if (a[pp][qq] == 0.0) continue;
                double theta = (a[qq][qq] - a[pp][pp]) / (2.0 * a[pp][qq]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < 3; ++k) {
                    double akp = a[k][pp], akq = a[k][qq];
                    a[k][pp] = cs * akp - sn * akq;
                    a[k][qq] = sn * akp + cs * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = a[pp][k], aqk = a[qq][k];
                    a[pp][k] = cs * apk - sn * aqk;
                    a[qq][k] = sn * apk + cs * aqk;
                }
            }
    }
    ev[0] = a[0][0]; ev[1] = a[1][1]; ev[2] = a[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2 - i; ++j)
            if (ev[j] > ev[j + 1]) { double t = ev[j]; ev[j] = ev[j + 1]; ev[j + 1] = t; }
}

/*
 * Lateral vibration stiffness of the probe at relaxed points (Sec. 3.3: the
 * stiffness of the probe's lateral modes is changed by the curvature of the
 * tip-sample interaction).  The stiffness matrix is K = -dG/dr (springs of
 * Eq. 2 plus the interpolated sample force); its symmetric part has one stiff
 * radial mode and two soft (lateral) modes.  out[2k], out[2k+1] = the two
 * smallest eigenvalues of sym(K), ascending (eV/A^2).
 */
void orc_lateral_stiffness(const double *g, const int *n, const double *ff, const double *p,
                           int m, const double *anchors, const double *rs, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < m; ++k) {
        double G[3], J[9], S[9], ev[3];
        orc_net(ff, g, n, p, anchors + 3 * k, rs + 3 * k, G, J);
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) S[3 * i + j] = -0.5 * (J[3 * i + j] + J[3 * j + i]);
        orc_sym3_eigs(S, ev);
        out[2 * k] = ev[0];
        out[2 * k + 1] = ev[1];
    }
}

void orc_relaxed_scan(const double *g, const int *n, const double *ff, const double *p,
                      const double *f, const int *fi, const double *s, const int *ns,
                      int ncols, const int *cols, double polish_tol,
                      double *r_out, double *fz_out, int *iters_out, double *gnorm_out,
                      double *lam_out)
{
    orc_relaxed_scan_mode(0, g, n, ff, p, f, fi, s, ns, ncols, cols, polish_tol, r_out, fz_out,
                          iters_out, gnorm_out, lam_out);
}

/* Relaxed scan on the tricubic potential: En is the energy grid [nz][ny][nx]. */
void orc_relaxed_scan_tricubic(const double *g, const int *n, const double *En, const double *p,
                               const double *f, const int *fi, const double *s, const int *ns,
                               int ncols, const int *cols, double polish_tol,
                               double *r_out, double *fz_out, int *iters_out,
                               double *gnorm_out, double *lam_out)
{
    orc_relaxed_scan_mode(1, g, n, En, p, f, fi, s, ns, ncols, cols, polish_tol, r_out, fz_out,
                          iters_out, gnorm_out, lam_out);
}

/* Net force and stability at given points (used for certificates). */
void orc_residual(const double *g, const int *n, const double *ff, const double *p,
                  int m, const double *anchors, const double *rs, double *gnorm,
                  double *lam)
{
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < m; ++k) {
        double G[3];
        gnorm[k] = orc_net(ff, g, n, p, anchors + 3 * k, rs + 3 * k, G, NULL);
        if (lam) lam[k] = orc_lambda_min(0, ff, g, n, p, anchors + 3 * k, rs + 3 * k);
    }
}

/* Same on the tricubic potential (En = energy grid). */
void orc_residual_tricubic(const double *g, const int *n, const double *En, const double *p,
                           int m, const double *anchors, const double *rs, double *gnorm,
                           double *lam)
{
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < m; ++k) {
        double G[3];
        gnorm[k] = orc_net_tc(En, g, n, p, anchors + 3 * k, rs + 3 * k, G, NULL);
        if (lam) lam[k] = orc_lambda_min(1, En, g, n, p, anchors + 3 * k, rs + 3 * k);
    }
}

/* ------------------------------------------------------------------------ */
/* Frequency shift (Sec. 2.1, Eq. 3)                                          */
/* ------------------------------------------------------------------------ */

/* Number of samples on each side of the centre: m = ceil(A/(2 dz) - 1e-9). */
int orc_df_m(double A, double dz)
{
    return (int)ceil(A / (2.0 * dz) - 1e-9);
}

/*
 * Quadrature weights w[j], j = -m..m (stored at w[j+m]) such that
 *   I(z_c) = int_{-a}^{a} z Fz(z_c + z) / sqrt(a^2 - z^2) dz = sum_j w_j Fz(z_c + j dz)
 * exactly when Fz is the piecewise-linear interpolant of its samples, a = A/2.
 * On a segment [z0, z1] the interpolant is (Fz0 (z1 - z) + Fz1 (z - z0)) / dz,
 * and int z/sqrt(a^2-z^2) = -sqrt(a^2-z^2),
 *     int z^2/sqrt(a^2-z^2) = (a^2/2) asin(z/a) - (z/2) sqrt(a^2-z^2).
 */
void orc_df_weights(double A, double dz, double *w)
{
    int m = orc_df_m(A, dz);
    double a = 0.5 * A;
    for (int j = 0; j <= 2 * m; ++j) w[j] = 0.0;
    for (int j = -m; j < m; ++j) {
        double z0 = j * dz, z1 = (j + 1) * dz;
        double lo = z0 > -a ? z0 : -a, hi = z1 < a ? z1 : a;
        if (!(lo < hi)) continue;
        double sl = sqrt(fmax(a * a - lo * lo, 0.0)), sh = sqrt(fmax(a * a - hi * hi, 0.0));
        double ul = lo / a, uh = hi / a;
        if (ul < -1) ul = -1;
        if (uh > 1) uh = 1;
        double K1 = -sh + sl;
        double K2 = (0.5 * a * a * asin(uh) - 0.5 * hi * sh) - (0.5 * a * a * asin(ul) - 0.5 * lo * sl);
        w[j + m] += (z1 * K1 - K2) / dz;
        w[j + 1 + m] += (K2 - z0 * K1) / dz;
    }
}

/* Prefactor C such that df = C * I:  C = -(f0 / 2k) (8 / (pi A^2)) * 16.02176634
 * (I in eV, A in A, k in N/m, result in Hz). */
double orc_df_prefactor(double A, double f0, double k)
{
    return -(f0 / (2.0 * k)) * (8.0 / (ORC_PI * A * A)) * ORC_EVA2_IN_NM;
}

/*
 * Frequency-shift stack from an Fz stack [nz][ncol] indexed by scan index
 * (index 0 = highest anchor, heights decrease by dz).  Output [nz-2m][ncol]:
 * output c is centred at scan index c + m; a physical offset +j dz is scan
 * index c + m - j.
 */
void orc_df(const double *fz, int nz, int ncol, double dz, double A, double f0,
            double k, double *df)
{
    int m = orc_df_m(A, dz);
    double *w = malloc(sizeof(double) * (2 * m + 1));
    orc_df_weights(A, dz, w);
    double C = orc_df_prefactor(A, f0, k);
    for (int c = 0; c + 2 * m < nz; ++c)
        for (int col = 0; col < ncol; ++col) {
            double I = 0.0;
            for (int j = -m; j <= m; ++j)
                I += w[j + m] * fz[(size_t)(c + m - j) * ncol + col];
            df[(size_t)c * ncol + col] = C * I;
        }
    free(w);
}

/* ------------------------------------------------------------------------ */
/* Implicit adjoint of the relaxed scan + frequency shift                    */
/* ------------------------------------------------------------------------ */

/*
 * Gradient of L with respect to atom positions, charges, R_i and e_i, given
 * dL/d(df) for every output of the stack and the (exact) equilibria r* of the
 * scan.  At an equilibrium G(r*, theta) = 0 (Eq. 1), so
 *   d r_star / d theta = -J^{-1} dG/dtheta,  J = dG/dr,
 * and Fz_tip = -F^T_z(r*) depends on theta only through r*.  With
 *   gbar_k = dL/dFz_k (transposed frequency-shift weights) and
 *   mu = -J^{-T} (gbar_k grad_r Fz_tip),
 * dL/dtheta = sum_k mu . dF^S_h/dtheta, and dF^S_h/dtheta is the trilinear
 * combination of d f_i(v)/dtheta over the eight cell corners v.
 *   f_i(v) = phi(rho) d, d = v - a_i,
 *   phi = 12 e (R^12 rho^-14 - R^6 rho^-8) + kq rho^-3  (e = e_iP, R = R_iP),
 * plus, for a quadrupolar probe, f_i = -kQ_i grad u with u = (3 dz^2 - rho^2)/rho^5
 * (orc_quad); grad u = a d + b e_z, a = 3 rho^-5 - 15 dz^2 rho^-7, b = 6 dz rho^-5,
 * so d f_i / d a_i = kQ_i hess u and d f_i / d q_i = -k_e q_zz grad u.  On a
 * periodic sample both terms carry the shifted-force truncation of orc_point
 * (phi gains -f(rc)/rho, u gains Y (3 rho rc^-4 - 4 rc^-3)) and pairs beyond rc
 * are skipped.
 * rstar [ncol][nz][3] in the order of cols; grad_df [nz-2m][ncol].
 */
void orc_scan_backward(const double *g, const int *n, const double *ff, const double *p,
                       const double *s, const int *ns, int ncols, const int *cols,
                       const double *rstar, const double *grad_df,
                       double A, double f0, double kc,
                       int na, const double *pos, const double *q, const double *R,
                       const double *eps,
                       double *g_pos, double *g_q, double *g_R, double *g_eps)
{
    int nz = ns[2];
    int m = orc_df_m(A, s[5]);
    int nc = nz - 2 * m;
    double *w = malloc(sizeof(double) * (2 * m + 1));
    orc_df_weights(A, s[5], w);
    double C = orc_df_prefactor(A, f0, kc);
    double *RiP = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *eiP = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *kqi = malloc(sizeof(double) * (na > 0 ? na : 1));
    double *kQi = malloc(sizeof(double) * (na > 0 ? na : 1));
    orc_mix(na, R, eps, q, p, RiP, eiP, kqi, kQi);
    for (int i = 0; i < na; ++i) {
        g_pos[3 * i] = g_pos[3 * i + 1] = g_pos[3 * i + 2] = 0.0;
        g_q[i] = g_R[i] = g_eps[i] = 0.0;
    }
    double rc2 = g[7] * g[7];
    int periodic = g[6] != 0.0;
    #pragma omp parallel
    {
        double *lp = calloc((size_t)6 * (na > 0 ? na : 1), sizeof(double));
        #pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < ncols; ++c) {
            int ix = cols[2 * c], iy = cols[2 * c + 1];
            for (int k = 0; k < nz; ++k) {
                /* gbar_k = sum_out grad_df[out] * C * w_j with out = k - m + j */
                double gbar = 0.0;
                for (int j = -m; j <= m; ++j) {
                    int out = k - m + j;
                    if (out < 0 || out >= nc) continue;
                    gbar += grad_df[(size_t)out * ncols + c] * C * w[j + m];
                }
                if (gbar == 0.0) continue;
                double anchor[3] = { s[0] + ix * s[2], s[1] + iy * s[3], s[4] - k * s[5] };
                const double *r = rstar + 3 * ((size_t)c * nz + k);
                double G[3], J[9], Jt[9], Ft[3];
                orc_net(ff, g, n, p, anchor, r, G, J);
                orc_tip_force(r, anchor, p, Ft, Jt);
                /* grad_r Fz_tip = -(row z of dF^T/dr) */
                double b[3] = { gbar * Jt[6], gbar * Jt[7], gbar * Jt[8] };
                /* solve J^T mu = b  (mu = -J^{-T} (gbar grad Fz) = J^{-T}(gbar * Jt_z)) */
                double JT[9] = { J[0], J[3], J[6], J[1], J[4], J[7], J[2], J[5], J[8] };
                double mu[3];
                if (!orc_solve3(JT, b, mu)) continue;
                orc_cell cl;
                orc_locate(g, n, r, &cl);
                double wx[2] = { 1.0 - cl.tx, cl.tx }, wy[2] = { 1.0 - cl.ty, cl.ty },
                       wz[2] = { 1.0 - cl.tz, cl.tz };
                for (int aa = 0; aa < 2; ++aa)
                    for (int bb = 0; bb < 2; ++bb)
                        for (int cc = 0; cc < 2; ++cc) {
                            double wc = wx[aa] * wy[bb] * wz[cc];
                            if (wc == 0.0) continue;
                            double v[3] = { g[0] + cl.ix[aa] * g[3], g[1] + cl.iy[bb] * g[4],
                                            g[2] + cl.iz[cc] * g[5] };
                            double mw[3] = { wc * mu[0], wc * mu[1], wc * mu[2] };
                            for (int i = 0; i < na; ++i) {
                                double d[3];
                                orc_disp(v, pos + 3 * i, g, n, d);
                                double rho2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                                if (periodic && !(rho2 < rc2)) continue;
                                double rho = sqrt(rho2);
                                double e = eiP[i], Rp = RiP[i];
                                double sr = Rp / rho;
                                double s6 = pow(sr, 6.0), s12 = s6 * s6;
                                double ir2 = 1.0 / rho2, ir3 = ir2 / rho;
                                double phi = 12.0 * e * (s12 - s6) * ir2 + kqi[i] * ir3;
                                /* phi'(rho)/rho */
                                double dphi = 12.0 * e * (-14.0 * s12 + 8.0 * s6) * ir2 * ir2
                                              - 3.0 * kqi[i] * ir3 * ir2;
                                /* per-rho factors of d phi / d(q_i, R_iP, e_iP) */
                                double phq = ir3;
                                double phR = 12.0 * e * (12.0 * s12 - 6.0 * s6) / Rp * ir2;
                                double phe = 12.0 * (s12 - s6) * ir2;
                                if (periodic) {
                                    /* shifted force (orc_pair_shift): phi -= f(rc)/rho with
                                       f(rc) = 12 e (sc^12 - sc^6)/rc + kq/rc^2 */
                                    double rc = g[7], sc = Rp / rc;
                                    double sc6 = pow(sc, 6.0), sc12 = sc6 * sc6;
                                    double fc = 12.0 * e * (sc12 - sc6) / rc + kqi[i] / (rc * rc);
                                    phi -= fc / rho;
                                    dphi += fc * ir3;
                                    phq -= 1.0 / (rc * rc * rho);
                                    phR -= 12.0 * e * (12.0 * sc12 - 6.0 * sc6) / (Rp * rc * rho);
                                    phe -= 12.0 * (sc12 - sc6) / (rc * rho);
                                }
                                double md = mw[0] * d[0] + mw[1] * d[1] + mw[2] * d[2];
                                /* d f / d a_i = -(phi I + (phi'/rho) d d^T) */
                                for (int t = 0; t < 3; ++t)
                                    lp[6 * i + t] -= phi * mw[t] + dphi * md * d[t];
                                /* d f / d q_i = k_e q_PP (d phi / d kq_i) d */
                                lp[6 * i + 3] += ORC_KE * p[2] * phq * md;
                                /* d f / d R_iP = (d phi / d R_iP) d; without a cutoff
                                   12 e (12 s^12 - 6 s^6) / (R rho^2) d */
                                lp[6 * i + 4] += phR * md;
                                /* d f / d e_i = (d e_iP / d e_i)(d phi / d e_iP) d, with
                                   d e_iP / d e_i = e_PP / (2 e_iP) */
                                if (e > 0.0)
                                    lp[6 * i + 5] += (p[1] / (2.0 * e)) * phe * md;
                                if (p[9] != 0.0) {
                                    double z = d[2];
                                    double ir5 = ir3 * ir2, ir7 = ir5 * ir2, ir9 = ir7 * ir2;
                                    double ua = 3.0 * ir5 - 15.0 * z * z * ir7;
                                    double ub = 6.0 * z * ir5;
                                    /* grad a . mw and grad b . mw */
                                    double ga = (-15.0 * ir7 + 105.0 * z * z * ir9) * md
                                                - 30.0 * z * ir7 * mw[2];
                                    double gb = 6.0 * ir5 * mw[2] - 30.0 * z * ir7 * md;
                                    if (periodic) {
                                        /* shifted d_z2 term (orc_quad_shift): grad u gains
                                           ax d + bx e_z; add them and their gradients . mw */
                                        double rc = g[7];
                                        double irc3 = 1.0 / (rc * rc * rc), irc4 = irc3 / rc;
                                        double ir1 = 1.0 / rho, ir4 = ir2 * ir2, ir6 = ir4 * ir2;
                                        ua += -9.0 * irc4 * z * z * ir3 + 24.0 * irc3 * z * z * ir4
                                              - 3.0 * irc4 * ir1;
                                        ub += 18.0 * irc4 * z * ir1 - 24.0 * irc3 * z * ir2;
                                        ga += -9.0 * irc4 * (2.0 * z * ir3 * mw[2] - 3.0 * z * z * ir5 * md)
                                              + 24.0 * irc3 * (2.0 * z * ir4 * mw[2] - 4.0 * z * z * ir6 * md)
                                              + 3.0 * irc4 * ir3 * md;
                                        gb += 18.0 * irc4 * (ir1 * mw[2] - z * ir3 * md)
                                              - 24.0 * irc3 * (ir2 * mw[2] - 2.0 * z * ir4 * md);
                                    }
                                    double Hm[3] = { ua * mw[0] + d[0] * ga,
                                                     ua * mw[1] + d[1] * ga,
                                                     ua * mw[2] + d[2] * ga + gb };
                                    for (int t = 0; t < 3; ++t)
                                        lp[6 * i + t] += kQi[i] * Hm[t];
                                    lp[6 * i + 3] -= ORC_KE * p[9] * (ua * md + ub * mw[2]);
                                }
                            }
                        }
            }
        }
        #pragma omp critical
        for (int i = 0; i < na; ++i) {
            g_pos[3 * i] += lp[6 * i];
            g_pos[3 * i + 1] += lp[6 * i + 1];
            g_pos[3 * i + 2] += lp[6 * i + 2];
            g_q[i] += lp[6 * i + 3];
            g_R[i] += lp[6 * i + 4];
            g_eps[i] += lp[6 * i + 5];
        }
        free(lp);
    }
    free(w); free(RiP); free(eiP); free(kqi); free(kQi);
}

/* ------------------------------------------------------------------------ */
/* Electrostatics from a grid potential (Sec. 2.2.3, Eq. of the cross-       */
/* correlation; Sec. 5.1.2)                                                  */
/* ------------------------------------------------------------------------ */

/* Signed offset of index i on a periodic axis of n points: i for i < n/2,
 * i - n above (for even n the index n/2 is taken as -n/2). */
static int orc_wrap_offset(int i, int n)
{
    return (2 * i < n) ? i : i - n;
}

/*
 * Charge density of the probe particle sampled on the grid's periodic lattice
 * of offsets from the probe centre (index 0 = the centre, negative offsets
 * wrapped to the far end):
 *   rho(r) = q_pp G(r) + q_zz d^2 G / dz^2,
 *   G(r)   = (2 pi sigma^2)^(-3/2) exp(-r^2 / (2 sigma^2)),
 * i.e. the point charge and the d_z2 quadrupole of the probe smeared by a
 * Gaussian of width sigma (as sigma -> 0 the quadrupole part is the point
 * density q_zz d^2 delta/dz^2).  rho is [nz][ny][nx], e/A^3.
 */
void orc_tip_density(const double *g, const int *n, double q_pp, double q_zz, double sigma,
                     double *rho)
{
    double s2 = sigma * sigma;
    double norm = 1.0 / pow(2.0 * ORC_PI * s2, 1.5);
    for (int iz = 0; iz < n[2]; ++iz)
        for (int iy = 0; iy < n[1]; ++iy)
            for (int ix = 0; ix < n[0]; ++ix) {
                double x = orc_wrap_offset(ix, n[0]) * g[3];
                double y = orc_wrap_offset(iy, n[1]) * g[4];
                double z = orc_wrap_offset(iz, n[2]) * g[5];
                double G = norm * exp(-(x * x + y * y + z * z) / (2.0 * s2));
                double d2G = G * (z * z / (s2 * s2) - 1.0 / s2);
                rho[((size_t)iz * n[1] + iy) * n[0] + ix] = q_pp * G + q_zz * d2G;
            }
}

/*
 * Cross-correlation of the probe density with the sample potential (the
 * electrostatic energy of the probe, Sec. 2.2.3), as the plain sum over the
 * periodic grid that the integral becomes:
 *   E[j] = dV sum_i rho[i] V[(i + j) mod n],   dV = hx hy hz,
 * with rho from orc_tip_density (offsets from the probe centre) and V the
 * sample potential on the grid (eV/e).  E is evaluated at the m voxels
 * idx[m][3] = (ix, iy, iz), or at every voxel ([nz][ny][nx]) if idx is NULL.
 */
void orc_correlate(const double *g, const int *n, const double *rho, const double *V, int m,
                   const int *idx, double *E)
{
    int nx = n[0], ny = n[1], nz = n[2];
    size_t N = (size_t)nx * ny * nz;
    double dV = g[3] * g[4] * g[5];
    long long cnt = idx ? m : (long long)N;
    #pragma omp parallel for schedule(dynamic, 16)
    for (long long t = 0; t < cnt; ++t) {
        int jx, jy, jz;
        if (idx) { jx = idx[3 * t]; jy = idx[3 * t + 1]; jz = idx[3 * t + 2]; }
        else { jx = (int)(t % nx); jy = (int)((t / nx) % ny); jz = (int)(t / ((size_t)nx * ny)); }
        double acc = 0.0;
        for (int iz = 0; iz < nz; ++iz) {
            int kz = (iz + jz) % nz;
            for (int iy = 0; iy < ny; ++iy) {
                int ky = (iy + jy) % ny;
                const double *r = rho + ((size_t)iz * ny + iy) * nx;
                const double *v = V + ((size_t)kz * ny + ky) * nx;
                for (int ix = 0; ix < nx; ++ix)
                    acc += r[ix] * v[(ix + jx) % nx];
            }
        }
        E[t] = dV * acc;
    }
}

/* Number of OpenMP threads the oracle runs with. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following parallel regions (the CPU baseline's one-thread run). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
