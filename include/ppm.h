/*
 * ppm.h -- C ABI of the MI355X probe-particle hot path.
 *
 * Paper: Oinonen et al., "Advancing Scanning Probe Microscopy Simulations:
 * A Decade of Development in Probe-Particle Models" (arXiv 2401.14564).
 *
 * The library computes, on one AMD Instinct MI355X (gfx950):
 *   1. the force-field grid of Lennard-Jones (Eq. 5) plus point-charge Coulomb
 *      (Eq. 6) energies and forces (F = -grad E, Sec. 2.2) on a uniform grid
 *      (Sec. 5.1.1, step 1)                                   -> ppm_build_ff
 *   2. the relaxed scan: for every tip column, descending in z, the probe
 *      particle is relaxed by FIRE (Sec. 5.1.1, step 2) under the tip springs
 *      (Eq. 2) plus the trilinearly interpolated grid force (Eq. 1), and the
 *      tip force is read out (text after Eq. 2)               -> ppm_relaxed_scan
 *   3. the frequency shift (Eq. 3, Giessibl), fused into the scan or
 *      standalone                                             -> ppm_df
 *   4. the gradient of a scalar function of the frequency-shift stack with
 *      respect to atom positions, charges and LJ parameters, by implicit
 *      differentiation of the equilibrium condition of Eq. 1
 *                                                 -> ppm_relaxed_scan_backward
 *   5. many molecules of different sizes in one launch per stage
 *                                                   -> ppm_batch_build_ff,
 *                                                      ppm_batch_relaxed_scan
 *   6. the stiffness of the probe's lateral vibration modes at the relaxed
 *      points (Sec. 3.3)                                -> ppm_lateral_stiffness
 *   7. the scan on a tricubic interpolant of an energy-only grid (Sec. 5.1.1)
 *                                 -> ppm_build_energy, ppm_relaxed_scan_tricubic
 *   8. a quadrupolar (d_z2) probe charge in the point-charge force field
 *      (Sec. 2.2.3, Sec. 2.2.5)                          -> ppm_probe.q_zz
 *   9. electrostatics from a sample potential on the grid, by cross-correlation
 *      with the probe's charge density (Sec. 2.2.3, Sec. 5.1.2)
 *                                          -> ppm_tip_density, ppm_hartree_ff
 *
 * Conventions shared by every entry point
 *   - Units: lengths in Angstrom, energies in eV, charges in e, forces in eV/A,
 *     spring constants in eV/A^2; the cantilever stiffness k_cant in N/m and
 *     f0 in Hz; frequency shifts in Hz.
 *   - z points up; the probe hangs below its anchor (d0 = (0, 0, -R0) for a
 *     symmetric tip).
 *   - Arrays are row-major [z][y][x] with x fastest.  Scan height index 0 is the
 *     highest anchor position; index k sits at z_top - k*dz.
 *   - Every array argument is a DEVICE pointer allocated and owned by the
 *     caller; the library keeps no pointer after the call returns.
 *   - Calls enqueue work on `stream` (a hipStream_t; NULL = the default stream)
 *     and return without synchronising.  Calls on different streams may run
 *     concurrently.
 *   - Every call validates its arguments on the host first and returns a
 *     ppm_status; on any error nothing is enqueued.  No C++ exception crosses
 *     the ABI.  PPM_EHIP reports a failed HIP launch (see ppm_last_hip_error).
 *   - Non-convergence of a relaxation is not an error: it is reported per point
 *     as a negative iteration count in the probe-state output.
 */
#ifndef PPM_H
#define PPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ppm_status;
#define PPM_OK 0
#define PPM_EINVAL (-1)        /* invalid argument (NULL, bad size, bad parameter) */
#define PPM_ERANGE (-2)        /* a size or index would overflow */
#define PPM_EHIP (-3)          /* a HIP runtime call or kernel launch failed */
#define PPM_EUNSUPPORTED (-4)  /* valid but outside what this build implements */

/* Uniform grid.  Voxel (ix, iy, iz) sits at origin + (ix*step[0], iy*step[1],
 * iz*step[2]); n = (nx, ny, nz).  With periodic_xy = 1 the sample is periodic in
 * x and y with periods n[0]*step[0] and n[1]*step[1]: each pair uses the
 * minimum image, is included iff rho^2 < cutoff^2, and is truncated with a
 * shifted force: along every ray from the atom each pair term Y(direction)
 * g(rho) (Y = 1 for LJ + Coulomb, 3 dz^2/rho^2 - 1 with g = rho^-3 for the d_z2
 * term) becomes g - g(cutoff) - (rho - cutoff) g'(cutoff), so its energy and
 * force vanish on the cutoff sphere (the paper names no cutoff scheme; a plain
 * truncation leaves a force step on every charged atom's sphere).  With periodic_xy = 0 the
 * sum runs over all atoms (open boundary) and cutoff is ignored.  For
 * interpolation a periodic grid wraps in x and y; an open grid is clamped to
 * its first/last cell in x and y (the field is continued constantly beyond
 * its edges, having no images to wrap to); z is always clamped (the field is
 * constant above and below the grid). */
typedef struct {
    double origin[3];
    double step[3];
    int32_t n[3];
    int32_t periodic_xy;
    double cutoff;
} ppm_grid;

/* Probe particle and tip (Sec. 2.1, Eq. 2; Sec. 2.2.1 mixing rules).
 * R_pp, eps_pp: LJ radius and depth of the probe; q_pp: its point charge (e).
 * k_lat: lateral stiffnesses (k_x, k_y); k_rad: radial stiffness (eV/A^2).
 * d0: rest displacement probe - anchor; R0 = |d0|.
 * q_zz: quadrupole moment of the probe's d_z2 charge (Sec. 2.2.3, e A^2; the
 * CO tip of Sec. 2.2.5 uses -0.05), taken as the point density
 * q_zz d^2 delta/dz^2, the limit of charges (+q, -2q, +q) at z+h, z, z-h with
 * q h^2 = q_zz; 0 for a point-charge probe. */
typedef struct {
    double R_pp, eps_pp, q_pp;
    double k_lat[2];
    double k_rad;
    double d0[3];
    double q_zz;
} ppm_probe;

/* FIRE relaxation parameters (Bitzek et al. 2006, as used in Sec. 5.1.1).
 * Per step: from the second step on, with P = G.v: if P > 0 the velocity is
 * mixed towards the force, v = (1-alpha) v + alpha |v| G/|G|, and after more
 * than n_min such steps in a row dt = min(dt*f_inc, dt_max), alpha *= f_alpha;
 * if P <= 0, v = 0, dt *= f_dec, alpha = alpha0.  Then v += G dt/mass,
 * r += v dt.  A point is converged when |G|_2 < f_conv (eV/A); after max_iter
 * steps it is recorded as not converged.  alpha and v restart at every
 * height; dt starts at dt0 and then continues from height to height (see
 * ppm_scan). */
typedef struct {
    double dt0, dt_max, f_inc, f_dec, alpha0, f_alpha, mass, f_conv;
    int32_t n_min, max_iter;
} ppm_fire;

/* Tip lattice: anchor of column (ix, iy) at height index k is
 * (x0 + ix*dx, y0 + iy*dy, z_top - k*dz), ix < nx, iy < ny, k < nz.
 * At k = 0 the probe starts at anchor + d0.  Warm start at k > 0: with
 * u(k) = relaxed position - anchor(k), the relaxation starts from
 * anchor(k) + u(k-1) + (u(k-1) - u(k-2)) (linear extrapolation; anchor(1) + u(0)
 * at k = 1), with zero velocity, alpha = alpha0 and the FIRE time step
 * continued from the previous height's final value (not below dt0). */
typedef struct {
    double x0, y0, dx, dy;
    int32_t nx, ny;
    double z_top, dz;
    int32_t nz;
} ppm_scan;

/* Frequency shift (Eq. 3): A = peak-to-peak amplitude (A), f0 (Hz), k_cant
 * (N/m).  The integral is evaluated exactly for the piecewise-linear
 * interpolant of the Fz samples: m = ceil(A/(2 dz) - 1e-9) samples on each side
 * of the centre; output o is centred at scan index o + m ("valid" outputs,
 * nz - 2m of them). */
typedef struct {
    double A, f0, k_cant;
} ppm_df_params;

/* Message for a status code (static storage). */
const char *ppm_status_string(ppm_status s);

/* The hipError_t of the last failed HIP call made by this library on the
 * calling thread (0 if none). */
int32_t ppm_last_hip_error(void);

/* Half-width m of the frequency-shift stencil for amplitude A and step dz,
 * or -1 if A <= 0 or dz <= 0. */
int32_t ppm_df_half_width(double A, double dz);

/*
 * ppm_build_ff -- force-field grid (Sec. 5.1.1 step 1; Eq. 5, Eq. 6, Sec. 2.2).
 * For every voxel v, with e_iP = sqrt(eps_i eps_pp), R_iP = R_i + R_pp,
 * kq_i = k_e q_i q_pp (k_e = 14.3996454784 eV*A/e^2), rho = |v - r_i|:
 *   E(v) = sum_i e_iP [(R_iP/rho)^12 - 2 (R_iP/rho)^6] + kq_i/rho
 *   F(v) = sum_i {12 e_iP [(R_iP/rho)^12 - (R_iP/rho)^6]/rho^2 + kq_i/rho^3} (v - r_i)
 * and, for a probe with q_zz != 0, per atom kQ_i (3 dz^2 - rho^2)/rho^5 in E
 * (kQ_i = k_e q_i q_zz, dz = z_v - z_i, i.e. q_zz d^2/dz^2 of the atom's
 * Coulomb potential) and its negative gradient in F.
 * in:  pos[n_atoms][3], q[n_atoms], R[n_atoms], eps[n_atoms] (FP64, device);
 *      n_atoms >= 0 (0 gives the zero field).
 * out: ff[nz][ny][nx][4] = (Fx, Fy, Fz, E), FP32, device.
 * Voxels closer than ~1e-3 A to an atom may hold inf.
 * Periodic grids are processed in bricks of 16 x 16 x 8 voxels, each atom taking
 * the image nearest to the brick centre; this is the exact minimum image for
 * every voxel of the brick when cutoff + h < min(Lx, Ly)/2, h being the brick's
 * half-diagonal (1.12 A at 0.1 A spacing).
 * Errors: PPM_EINVAL for NULL pointers (when n_atoms > 0), n[i] < 2, steps
 * <= 0, or periodic_xy with cutoff <= 0 or cutoff + h >= min(Lx, Ly)/2;
 * PPM_ERANGE if the grid has 2^31 voxels or more.
 */
ppm_status ppm_build_ff(const ppm_grid *grid, const ppm_probe *probe, int32_t n_atoms,
                        const double *pos, const double *q, const double *R,
                        const double *eps, float *ff, void *stream);

/*
 * ppm_relaxed_scan -- relaxed scan with optional fused frequency shift
 * (Sec. 2.1 Eq. 1-3, Sec. 5.1.1 step 2).
 * in:  ff[nz][ny][nx][4] from ppm_build_ff (only Fx, Fy, Fz are read).
 * Precision: when fire->f_conv >= 1e-5 eV/A the probe state (its displacement
 * from the tip anchor), FIRE, the springs (hardware 1/sqrt estimate) and the
 * trilinear combination are FP32 -- the force balance then carries about 1e-6
 * eV/A of rounding, an order below the threshold; otherwise all of them are
 * FP64 (absolute positions), so tight thresholds resolve the force balance
 * below FP32 rounding.
 * out (each may be NULL, at least one must be given):
 *   fz[scan.nz][scan.ny][scan.nx]  tip force Fz_tip = -F^T_z at the relaxed
 *                                   probe position (eV/A)
 *   pp[scan.nz][scan.ny][scan.nx][4] (ux, uy, uz, iters): relaxed probe
 *                                   position minus its rest position
 *                                   anchor + d0 (A), and the FIRE step count
 *                                   (negative if not converged)
 *   df[scan.nz-2m][scan.ny][scan.nx] frequency shift (Hz); requires dfp and
 *                                   scan.nz >= 2m+1; m <= 32; with more than
 *                                   256 heights fz must be given as well.
 * Errors: PPM_EINVAL for a bad grid/probe/fire/scan (f_conv <= 0, dt <= 0,
 * mass <= 0, negative stiffness, |d0| == 0, nz < 1, max_iter < 1), df without
 * dfp or with too few heights, or all outputs NULL; PPM_EUNSUPPORTED if m > 32
 * or if df is requested for more than 256 heights without fz.
 */
ppm_status ppm_relaxed_scan(const ppm_grid *grid, const float *ff, const ppm_probe *probe,
                            const ppm_fire *fire, const ppm_scan *scan, float *fz,
                            float *pp, const ppm_df_params *dfp, float *df, void *stream);

/* ------------------------------------------------------------------------
 * Launch shapes and their autotuner.  The force field is the step that
 * limits the two-step method (Sec. 5.1.1 step 1, Sec. 5.3), and the best
 * shapes depend on the probe (the d_z2 term adds ~11 instructions per pair,
 * which changes the register budget) and on the tip lattice (how many
 * columns fill the GPU, how many heights fit on chip).  The tuner times the
 * candidate shapes on the caller's own inputs and returns the fastest; the
 * calls below take the result.
 *   ff_nzb    voxels per thread along z in the force-field build (the brick
 *             is 16 x 16 x ff_nzb voxels): 0 (= 8), 6 or 8.  Brick-local
 *             coordinates depend on the brick, so builds with different depths
 *             differ in FP32 rounding (each within the parity bound); builds
 *             with the same depth, single or batched, are bit-identical.
 *   scan_tile relaxed-scan work-group: 0 (automatic: 16 x 16-column blocks of
 *             four waves where the heights fit the LDS staging, else 8 x 8),
 *             16 (16 x 16 where the requested outputs allow it) or 8 (8 x 8
 *             one-wave blocks).  Every scan shape gives the same bits.
 *   scan_fz_direct  0 or 1.  With 1, scan_tile 8 and an fz output, the scan
 *             writes each height's Fz straight to fz, instead of staging the
 *             column in LDS (4 B per height and column), and the frequency
 *             shift (if requested) follows as a second pass over fz, enqueued
 *             on the same stream by the same call: the scan's blocks then need
 *             no LDS, and large lattices keep all their waves resident at once.
 *             Ignored otherwise.  Same bits either way.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t ff_nzb;
    int32_t scan_tile;
    int32_t scan_fz_direct;
} ppm_tuning;

/* ppm_build_ff with the brick depth of `tuning` (NULL = defaults).  Errors as
 * ppm_build_ff, and PPM_EINVAL for a depth other than 0, 6, 8. */
ppm_status ppm_build_ff_tuned(const ppm_grid *grid, const ppm_probe *probe,
                              const ppm_tuning *tuning, int32_t n_atoms, const double *pos,
                              const double *q, const double *R, const double *eps, float *ff,
                              void *stream);

/* ppm_relaxed_scan with the work-group shape of `tuning` (NULL = automatic).
 * Errors as ppm_relaxed_scan, and PPM_EINVAL for a tile other than 0, 8, 16 or
 * a scan_fz_direct other than 0, 1. */
ppm_status ppm_relaxed_scan_tuned(const ppm_grid *grid, const float *ff,
                                  const ppm_probe *probe, const ppm_fire *fire,
                                  const ppm_scan *scan, const ppm_tuning *tuning, float *fz,
                                  float *pp, const ppm_df_params *dfp, float *df,
                                  void *stream);

/*
 * ppm_tune_build_ff -- autotuner of the force-field brick depth: builds the
 * grid (arguments as ppm_build_ff; ff is overwritten) with each candidate
 * depth (8, then 6), once untimed and three times timed with HIP events on
 * `stream`, and sets tuning->ff_nzb to the fastest (median); the other field
 * is left as it was.  ms (may be NULL) receives the two medians in that
 * order.  Blocks until the stream is idle; creates and destroys two events,
 * allocates no memory.  Errors as ppm_build_ff, PPM_EINVAL if tuning is NULL,
 * PPM_EHIP if an event call fails.
 */
ppm_status ppm_tune_build_ff(const ppm_grid *grid, const ppm_probe *probe, int32_t n_atoms,
                             const double *pos, const double *q, const double *R,
                             const double *eps, float *ff, void *stream, ppm_tuning *tuning,
                             float *ms);

/*
 * ppm_tune_relaxed_scan -- autotuner of the scan's work-group shape: runs the
 * scan (arguments as ppm_relaxed_scan; the outputs are overwritten, with the
 * same bits whatever the shape) with scan_tile 16, scan_tile 8 and, when fz
 * is given, scan_tile 8 with scan_fz_direct 1, each once untimed and three
 * times timed, and sets tuning->scan_tile and tuning->scan_fz_direct to the
 * fastest (median); ms (may be NULL, else three floats) receives the medians
 * in that order, 0 for a candidate not run.  Blocking, as ppm_tune_build_ff.
 */
ppm_status ppm_tune_relaxed_scan(const ppm_grid *grid, const float *ff, const ppm_probe *probe,
                                 const ppm_fire *fire, const ppm_scan *scan, float *fz,
                                 float *pp, const ppm_df_params *dfp, float *df, void *stream,
                                 ppm_tuning *tuning, float *ms);

/*
 * ppm_build_energy -- energy-only grid for the tricubic scan (Sec. 5.1.1 step 2:
 * interpolating the potential tricubically avoids storing the forces).  Same
 * sum and arguments as ppm_build_ff; out: E[nz][ny][nx] (FP32, eV).
 */
ppm_status ppm_build_energy(const ppm_grid *grid, const ppm_probe *probe, int32_t n_atoms,
                            const double *pos, const double *q, const double *R,
                            const double *eps, float *E, void *stream);

/*
 * ppm_relaxed_scan_tricubic -- the relaxed scan of ppm_relaxed_scan with the
 * sample force taken from a tricubic interpolant of the energy grid instead of
 * trilinear forces (the variant Sec. 5.1.1 step 2 describes as under test).
 * Interpolant: Catmull-Rom (Keys a = -1/2) cubic convolution per axis on the
 * stencil i-1..i+2; F = -grad of the interpolant.  x,y wrap on a periodic
 * grid; otherwise, and always in z, the point is clamped to the grid box:
 * outside [0, n-1] the force is continued constantly along that axis.
 * The stencil weights and contraction are FP32 (and the spring's 1/|d| the
 * hardware estimate) when fire->f_conv >= 1e-5 eV/A and FP64 otherwise, as for
 * ppm_relaxed_scan.
 * in:  E[nz][ny][nx] from ppm_build_energy.  Outputs, errors: as ppm_relaxed_scan.
 */
ppm_status ppm_relaxed_scan_tricubic(const ppm_grid *grid, const float *E,
                                     const ppm_probe *probe, const ppm_fire *fire,
                                     const ppm_scan *scan, float *fz, float *pp,
                                     const ppm_df_params *dfp, float *df, void *stream);

/*
 * ppm_df -- standalone frequency shift of an Fz stack (Eq. 3).
 * in:  fz[nz][ny][nx] in scan-index order (index 0 highest), height step dz.
 * out: df[nz-2m][ny][nx] (Hz).
 * Errors: PPM_EINVAL for NULL pointers, nz < 2m+1, ny or nx < 1, dz <= 0,
 * A <= 0, k_cant <= 0; PPM_EUNSUPPORTED if m > 32.
 */
ppm_status ppm_df(const float *fz, int32_t nz, int32_t ny, int32_t nx, double dz,
                  const ppm_df_params *dfp, float *df, void *stream);

/*
 * Workspace size (bytes, 256-byte aligned) needed by ppm_relaxed_scan_backward
 * for this scan and atom count.
 */
size_t ppm_backward_workspace_bytes(const ppm_scan *scan, int32_t n_atoms);

/*
 * ppm_relaxed_scan_backward -- gradient of L with respect to the atoms, given
 * grad_df = dL/d(df) for the stack produced by ppm_relaxed_scan with the same
 * arguments.  At every relaxed point G(r*) = F^T(r*) + F^S_h(r*) = 0 (Eq. 1), so
 * with J = dG/dr (3x3, trilinear cell Jacobian plus spring Jacobian),
 *   gbar_k = dL/dFz_k  (transposed Eq. 3 weights),
 *   mu = J^{-T} (gbar_k * grad_r F^T_z),
 *   dL/dtheta_i += mu . sum_corners w_c d f_i(v_c)/d theta_i
 * where f_i(v) is atom i's pair force at grid corner v, recomputed (the grid
 * gradient is never stored).  theta_i = (r_i, q_i, R_i, eps_i).
 * in:  grid, ff, probe, scan, dfp as in the forward call; pos, q, R, eps as in
 *      ppm_build_ff; pp = the forward call's probe-state output (required);
 *      grad_df[nz-2m][ny][nx] (FP32).
 * out: g_pos[n_atoms][3], g_q, g_R, g_eps (FP64, overwritten).
 * workspace: device buffer of at least ppm_backward_workspace_bytes() bytes.
 * Points recorded as not converged contribute nothing.  The result is
 * deterministic (fixed reduction order).
 * Errors: as ppm_relaxed_scan, plus PPM_EINVAL for NULL pointers or a
 * workspace that is too small.
 */
ppm_status ppm_relaxed_scan_backward(const ppm_grid *grid, const float *ff,
                                     const ppm_probe *probe, const ppm_scan *scan,
                                     const ppm_df_params *dfp, int32_t n_atoms,
                                     const double *pos, const double *q, const double *R,
                                     const double *eps, const float *pp,
                                     const float *grad_df, double *g_pos, double *g_q,
                                     double *g_R, double *g_eps, void *workspace,
                                     size_t workspace_bytes, void *stream);

/*
 * ppm_relaxed_scan_backward_noalloc -- for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): ppm_relaxed_scan_backward without the workspace argument.
 * The workspace is a static device array of PPM_NOALLOC_SCRATCH_BYTES (64 MiB)
 * that every GPU the library runs on holds until the process ends; its
 * address is looked up once per device (hipGetSymbolAddress, with that device
 * current).  The call allocates nothing and runs the same kernels, so its
 * gradients equal ppm_relaxed_scan_backward's bit for bit.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialised by the caller.
 * Errors: as ppm_relaxed_scan_backward; PPM_ERANGE when
 * ppm_backward_workspace_bytes(scan, n_atoms) exceeds PPM_NOALLOC_SCRATCH_BYTES
 * (the differentiation workload, 128 x 128 x 30 points and 60 atoms, needs
 * 34.5 MiB); PPM_EHIP if the array's address cannot be obtained.
 */
#define PPM_NOALLOC_SCRATCH_BYTES (64u * 1024u * 1024u)
ppm_status ppm_relaxed_scan_backward_noalloc(const ppm_grid *grid, const float *ff,
                                             const ppm_probe *probe, const ppm_scan *scan,
                                             const ppm_df_params *dfp, int32_t n_atoms,
                                             const double *pos, const double *q,
                                             const double *R, const double *eps, const float *pp,
                                             const float *grad_df, double *g_pos, double *g_q,
                                             double *g_R, double *g_eps, void *stream);

/*
 * ppm_lateral_stiffness -- stiffness of the probe's lateral vibration modes at
 * every relaxed point of a scan (Sec. 3.3: the curvature of the tip-sample
 * interaction shifts the lateral CO mode, the basis of the IETS contrast).
 * With K = -dG/dr at the relaxed position (spring Jacobian of Eq. 2 plus the
 * trilinear cell Jacobian of the grid force), k_out receives the two smallest
 * eigenvalues of (K + K^T)/2, ascending, in eV/A^2.
 * in:  grid, ff, probe, scan as given to ppm_relaxed_scan; pp = its probe-state
 *      output [scan.nz][scan.ny][scan.nx][4].
 * out: k_out[scan.nz][scan.ny][scan.nx][2] (FP32); NaN where the relaxation did
 *      not converge.
 * Errors: as ppm_relaxed_scan for grid/probe/scan; PPM_EINVAL for NULL pointers.
 */
ppm_status ppm_lateral_stiffness(const ppm_grid *grid, const float *ff, const ppm_probe *probe,
                                 const ppm_scan *scan, const float *pp, float *k_out,
                                 void *stream);

/* ------------------------------------------------------------------------
 * Electrostatics from a sample potential given on the grid (Sec. 2.2.3: the
 * probe's energy is the cross-correlation of its charge density with the
 * sample's Hartree potential; Sec. 5.1.2: evaluated by the convolution
 * theorem).  The grid is taken periodic in x, y and z (the potential of a
 * periodic DFT cell); periodic_xy and cutoff are ignored.  Each n[i] must be
 * 2^a 3^b 5^c and at most 1024, else PPM_EUNSUPPORTED.
 * ------------------------------------------------------------------------ */

/*
 * ppm_tip_density -- charge density of the probe particle on the grid's
 * lattice of offsets from the probe centre (index 0 is the centre; negative
 * offsets wrap to the far end):
 *   rho(r) = q_pp G(r) + q_zz d^2 G / dz^2,  G = (2 pi sigma^2)^(-3/2) exp(-r^2 / (2 sigma^2)),
 * a Gaussian-smeared point charge (e) and d_z2 quadrupole (e A^2, the moment
 * of ppm_probe.q_zz).  The cell should span several sigma on each side.
 * out: rho[nz][ny][nx] (FP32, e/A^3, device).
 * Errors: PPM_EINVAL for a bad grid, rho NULL, sigma <= 0 or non-finite charges.
 */
ppm_status ppm_tip_density(const ppm_grid *grid, double q_pp, double q_zz, double sigma,
                           float *rho, void *stream);

/* Workspace (bytes) ppm_hartree_ff needs for this grid: three complex FP64
 * grids and a few KiB of reduction scratch; 0 if the grid is invalid or
 * unsupported. */
size_t ppm_hartree_workspace_bytes(const ppm_grid *grid);

/*
 * ppm_hartree_ff -- energy and force of the probe in the sample potential V:
 *   E[j] = dV sum_i rho[i] V[(i + j) mod n],   dV = hx hy hz,
 *   F = -grad E (gradient of the trigonometric interpolant of E),
 * computed as E^ = dV conj(rho^) V^ and F^ = -i kappa E^ with FP64 FFTs.
 * in:  V[nz][ny][nx] (eV/e), rho[nz][ny][nx] from ppm_tip_density or any
 *      density on the same lattice of offsets (FP32, device).
 * out: ff[nz][ny][nx][4] = (Fx, Fy, Fz, E) (FP32), overwritten if accumulate
 *      is 0 or added to the values there if accumulate is 1 (e.g. onto the
 *      Lennard-Jones grid of ppm_build_ff with q_pp = q_zz = 0).
 * workspace: device buffer of at least ppm_hartree_workspace_bytes() bytes.
 * Errors: PPM_EINVAL for a bad grid, NULL pointers, accumulate not 0 or 1, or
 * a workspace that is too small; PPM_EUNSUPPORTED for axis lengths the FFT
 * does not handle.
 */
ppm_status ppm_hartree_ff(const ppm_grid *grid, const float *V, const float *rho,
                          int32_t accumulate, float *ff, void *workspace,
                          size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Batched pipeline (Sec. 4.4: large batches of simulated image stacks over
 * many molecules and tip parameters for machine-learning data; Sec. 5.3: the
 * per-run overheads that dominate small systems are paid once per batch):
 * many molecules of different sizes, each scanned with one
 * or more probes, in one launch per stage.  Host tables describe the work; the
 * same tables copied to device memory are read by the kernels.  Force fields,
 * tip forces and frequency shifts live in arenas (one device buffer each) at
 * the offsets ppm_batch_plan assigns.  The calls allocate nothing, so a
 * build + scan pair can be captured in a HIP graph and replayed.
 * ------------------------------------------------------------------------ */

/* One molecule.  atom_begin/n_atoms index the concatenated atom arrays
 * (positions [.][3], q, R, eps) shared by the whole batch; ff_nzb is the
 * force-field brick depth (0, 6 or 8, as ppm_tuning.ff_nzb): a molecule built
 * with the depth a single ppm_build_ff_tuned call uses gets the same bits. */
typedef struct {
    ppm_grid grid;
    int32_t atom_begin;
    int32_t n_atoms;
    int32_t ff_nzb;
    int32_t reserved;
    int64_t ff_offset;     /* set by ppm_batch_plan: first voxel in the FF arena */
    int64_t brick_begin;   /* set by ppm_batch_plan: first FF work item */
} ppm_batch_mol;

/* One scan job: molecule `mol` scanned with `probe` over `scan`.  The probe's
 * R_pp, eps_pp, q_pp and q_zz must equal those the batch's force fields were built
 * with; its springs and d0 may differ per job.  Outputs are stacks
 * [scan.nz][scan.ny][scan.nx] (fz) and [scan.nz-2m][scan.ny][scan.nx] (df). */
typedef struct {
    ppm_probe probe;
    ppm_scan scan;
    int32_t mol;
    int32_t reserved;
    int64_t fz_offset;     /* set by ppm_batch_plan: first value in the fz arena */
    int64_t df_offset;     /* set by ppm_batch_plan: first value in the df arena */
    int64_t tile_begin;    /* set by ppm_batch_plan: first scan work item */
} ppm_batch_scan;

/*
 * ppm_batch_plan -- host-only bookkeeping.  Validates the tables (host memory),
 * fills their offset fields in place and returns the sizes in totals[5]:
 *   totals[0] force-field voxels (the FF arena holds 4 floats per voxel)
 *   totals[1] force-field work items, totals[2] fz values, totals[3] df values
 *   (0 if dfp is NULL), totals[4] scan work items.
 * All jobs must share scan.dz when dfp is given, and R_pp, eps_pp, q_pp and
 * q_zz (the force fields are built once, with one probe).  Errors: PPM_EINVAL
 * for bad tables (as the single-molecule calls would report) or jobs whose
 * probe LJ parameters or charges differ from job 0's, PPM_EUNSUPPORTED for a
 * stencil wider than 32 or jobs with different dz.
 */
ppm_status ppm_batch_plan(int32_t n_mol, ppm_batch_mol *mols, int32_t n_jobs,
                          ppm_batch_scan *jobs, const ppm_df_params *dfp, int64_t *totals);

/*
 * ppm_batch_build_ff -- force fields of every molecule (as ppm_build_ff) in one
 * launch.  mols_host/mols_dev: the planned table in host and device memory
 * (same content); probe: the probe's LJ parameters and charge; pos/q/R/eps:
 * concatenated atoms (device, FP64); ff_arena: device, totals[0] x 4 floats.
 * Bricks are 16 x 16 x 8 voxels (as in ppm_build_ff), so a periodic molecule
 * needs cutoff + (half-diagonal of that brick, 1.12 A at 0.1 A) < min(Lx, Ly)/2.
 */
ppm_status ppm_batch_build_ff(int32_t n_mol, const ppm_batch_mol *mols_host,
                              const ppm_batch_mol *mols_dev, const ppm_probe *probe,
                              const double *pos, const double *q, const double *R,
                              const double *eps, float *ff_arena, void *stream);

/*
 * ppm_batch_relaxed_scan -- every scan job (as ppm_relaxed_scan, FIRE and
 * frequency-shift settings shared) in one launch, with the frequency shift
 * fused.  fz_arena (totals[2] floats) may be NULL when dfp is given; df_arena
 * (totals[3] floats) is required with dfp.  With more than 256 heights in any
 * job and a frequency shift, fz_arena is required.  PPM_EINVAL also when the
 * jobs' probe LJ parameters or charges differ from job 0's.
 */
ppm_status ppm_batch_relaxed_scan(int32_t n_mol, const ppm_batch_mol *mols_host,
                                  const ppm_batch_mol *mols_dev, int32_t n_jobs,
                                  const ppm_batch_scan *jobs_host,
                                  const ppm_batch_scan *jobs_dev, const ppm_fire *fire,
                                  const ppm_df_params *dfp, const float *ff_arena,
                                  float *fz_arena, float *df_arena, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PPM_H */
