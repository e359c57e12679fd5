// ppm_kernels.h -- launch-argument structs and launcher declarations shared by
// the HIP translation units of libppm (internal; the public ABI is ppm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "ppm.h"

namespace ppm {

// Coulomb constant e^2/(4 pi eps0) in eV*A.
constexpr double kCoulomb = 14.3996454784;
// 1 eV/A^2 in N/m (exact SI).
constexpr double kEvPerA2InNewtonPerM = 16.02176634;
// Largest supported frequency-shift half-width (samples on each side).
constexpr int kMaxDfHalfWidth = 32;
// Scan kernels take 64-bit grid offsets (WIDE) when the grid holds 4 GiB or
// more, or when a plane or the z extent reaches 2^24 voxels: below those bounds
// the 32-bit kernels form voxel indices with 24-bit multiplies.
inline bool scan_grid_wide(int nx, int ny, int nz, double bytes_per_voxel)
{
    return bytes_per_voxel * nx * (double)ny * nz >= 4294967296.0 ||
           (double)nx * ny >= 16777216.0 || nz >= 16777216;
}

// Largest scan height count whose per-lane Fz column (one 64-lane block) fits
// in 64 KiB of LDS; taller scans with a fused frequency shift need the fz output.
constexpr int kMaxScanLdsHeights = 256;

// ---------------------------------------------------------------- FF build
struct FFArgs {
    double ox, oy, oz;        // grid origin (A)
    double hx, hy, hz;        // voxel steps (A)
    int nx, ny, nz;
    int n_atoms;
    double R_pp, eps_pp;      // probe LJ parameters
    double kq_pp;             // k_e * q_pp
    double kQ_pp;             // k_e * q_zz (quadrupolar probe charge)
    double Lx, Ly;            // periods (periodic only)
    float rc2;                // cutoff^2 (periodic only)
    double cull2;             // (cutoff + brick half-diagonal)^2 (periodic only)
    double rc;                // cutoff (periodic only; shifted-force truncation)
};

hipError_t launch_build_ff_batch(const FFArgs &probe_args, const ppm_batch_mol *mols_dev,
                                 int n_mol, long long n_bricks, const double *pos,
                                 const double *q, const double *R, const double *eps,
                                 float4 *arena, hipStream_t stream);
// nzb: voxels per thread along z (the brick depth), 6 or 8 (0 = 8)
double ff_brick_half_diagonal(double hx, double hy, double hz, int nzb);
long long ff_brick_count(int nx, int ny, int nz, int nzb);

hipError_t launch_build_ff(const FFArgs &a, const double *pos, const double *q,
                           const double *R, const double *eps, float4 *ff,
                           hipStream_t stream, int nzb);

// ------------------------------------------------------------ relaxed scan
// Smallest convergence threshold (eV/A) for which the scan combines the eight
// FP32 corner forces in FP32 and takes the spring's 1/|d| from the hardware
// estimate: both then err at about 1e-7 of the force, at least two orders of
// magnitude below the threshold for forces up to ~10 eV/A.  Tighter thresholds
// use FP64 throughout, so the force balance can be resolved below FP32 rounding
// (differentiation, finite-difference checks).
constexpr double kLerp32MinFconv = 1e-5;

struct ScanArgs {
    // grid (interpolation)
    double ox, oy, oz;
    double ihx, ihy, ihz;     // inverse steps
    double oxi, oyi, ozi;     // -origin * inverse step (grid coordinate = r * ih + oi)
    double ignx, igny;        // 1/gnx, 1/gny
    int gnx, gny, gnz;
    int periodic;             // 1: x,y wrap (periodic sample); 0: clamped like z
    // probe
    double kx, ky, kR, R0;
    double d0x, d0y, d0z;
    // FIRE
    double dt0, dt_max, f_inc, f_dec, alpha0, f_alpha, inv_mass, f_conv2;
    int n_min, max_iter;
    int lerp32;               // 1: FP32-level interpolation and spring arithmetic (f_conv >= kLerp32MinFconv)
    // tip lattice
    double x0, y0, sdx, sdy, z_top, sdz;
    int snx, sny, snz;
    // frequency shift
    int m;                    // half-width, 0 if no fused output
    int ndf;                  // snz - 2m
    int tiles_x, n_tiles;     // tile decomposition of the tip lattice
};

// Grid, probe and tip-lattice fields of ScanArgs (FIRE, frequency-shift and
// tiling fields are set by the caller).  Used on the host for single scans and
// per block on the device for batched scans.
__host__ __device__ inline void fill_scan_geometry(ScanArgs &a, const ppm_grid &g,
                                                   const ppm_probe &p, const ppm_scan &s)
{
    a.ox = g.origin[0];
    a.oy = g.origin[1];
    a.oz = g.origin[2];
    a.ihx = 1.0 / g.step[0];
    a.ihy = 1.0 / g.step[1];
    a.ihz = 1.0 / g.step[2];
    a.oxi = -g.origin[0] / g.step[0];
    a.oyi = -g.origin[1] / g.step[1];
    a.ozi = -g.origin[2] / g.step[2];
    a.gnx = g.n[0];
    a.gny = g.n[1];
    a.gnz = g.n[2];
    a.ignx = 1.0 / g.n[0];
    a.igny = 1.0 / g.n[1];
    a.periodic = g.periodic_xy ? 1 : 0;
    a.kx = p.k_lat[0];
    a.ky = p.k_lat[1];
    a.kR = p.k_rad;
    a.d0x = p.d0[0];
    a.d0y = p.d0[1];
    a.d0z = p.d0[2];
    a.R0 = sqrt(p.d0[0] * p.d0[0] + p.d0[1] * p.d0[1] + p.d0[2] * p.d0[2]);
    a.x0 = s.x0;
    a.y0 = s.y0;
    a.sdx = s.dx;
    a.sdy = s.dy;
    a.z_top = s.z_top;
    a.sdz = s.dz;
    a.snx = s.nx;
    a.sny = s.ny;
    a.snz = s.nz;
}

// Frequency-shift weights padded to the ring-buffer length 2*kMaxDfHalfWidth+1,
// prefactor included: df(o) = sum_j w[j] * ring[j], ring[j] = Fz(k - (2M - j)).
struct DfWeights {
    float w[2 * kMaxDfHalfWidth + 1];
};

// tile: ppm_tuning.scan_tile; fz_direct: ppm_tuning.scan_fz_direct
hipError_t launch_relaxed_scan(const ScanArgs &a, const DfWeights &w, const float4 *ff,
                               float *fz, float4 *pp, float *df, hipStream_t stream, int tile,
                               bool fz_direct);

// Batched scan: one 8x8 column tile per block over all jobs of the batch.
// `proto` carries the FIRE and frequency-shift fields shared by the batch.
hipError_t launch_relaxed_scan_batch(const ScanArgs &proto, const DfWeights &w,
                                     const ppm_batch_mol *mols_dev,
                                     const ppm_batch_scan *jobs_dev, int n_jobs,
                                     long long n_tiles, int max_nz, bool wide,
                                     const float4 *arena, float *fz_arena, float *df_arena,
                                     hipStream_t stream);
long long scan_tile_count(int nx, int ny);

hipError_t launch_relaxed_scan_tricubic(const ScanArgs &a, const DfWeights &w, const float *En,
                                        float *fz, float4 *pp, float *df, hipStream_t stream);
hipError_t launch_build_energy(const FFArgs &a, const double *pos, const double *q,
                               const double *R, const double *eps, float *E, hipStream_t stream);

hipError_t launch_lateral_stiffness(const ScanArgs &a, const float4 *ff, const float4 *pp,
                                    float *out, hipStream_t stream);

hipError_t launch_df(const float *fz, int nz, int ny, int nx, int m, const DfWeights &w,
                     float *df, hipStream_t stream);

// ------------------------------------------------ grid electrostatics (FFT)
constexpr int kMaxFftLength = 1024;      // points per axis
constexpr int kMaxFftStages = 16;

// Radix sequence of one axis and the number of lines a block transforms.  For
// each stage, the divisors the Stockham indexing needs (n/P and the product m of
// the previous radices) as multiply-high reciprocals: x / d = umulhi(x, M) with
// M = floor(2^32 / d) + 1, exact for x < 2^13 and d <= 2048 (0 marks d = 1).
struct FftPlan {
    int n;
    int lines;
    int n_stages;
    int radix[kMaxFftStages];
    unsigned rcp_nb[kMaxFftStages];
    unsigned rcp_m[kMaxFftStages];
    unsigned rcp_n, rcp_lines;     // of n and of lines (load/store index split)
};

// false if n is not 2^a 3^b 5^c with 2 <= n <= kMaxFftLength
bool fft_plan(int n, FftPlan *p);
hipError_t launch_tip_density(int nx, int ny, int nz, double hx, double hy, double hz,
                              double q_pp, double q_zz, double sigma, float *rho,
                              hipStream_t stream);
// scratch: hartree_scratch_bytes() of device memory (reduction partials, alpha)
size_t hartree_scratch_bytes();
hipError_t launch_hartree(const FftPlan plans[3], int nx, int ny, int nz, double hx, double hy,
                          double hz, const float *V, const float *rho, int accumulate,
                          float4 *ff, double2 *Z, double2 *A, double2 *B, void *scratch,
                          hipStream_t stream);

// ---------------------------------------------------------------- backward
struct BwdArgs {
    ScanArgs s;               // same grid/probe/scan description as the forward
    double hx, hy, hz;        // grid steps
    int periodic;             // minimum image in x,y and shifted-force cutoff rc
    double Lx, Ly;
    float rc2;
    double rc;
    int n_atoms;
    double R_pp, eps_pp, kq_pp, ke_qpp;
    double kQ_pp;             // k_e * q_zz; the scatter adds the quadrupole terms if != 0
    int eq_per_block;         // equilibria handled by one block of the scatter
    int n_eq_blocks;          // number of equilibrium chunks
};

hipError_t launch_backward(const BwdArgs &a, const DfWeights &w, const float4 *ff,
                           const float4 *pp, const float *grad_df, const double *pos,
                           const double *q, const double *R, const double *eps,
                           float4 *eq_ws, double *partial_ws, double *g_pos, double *g_q,
                           double *g_R, double *g_eps, hipStream_t stream);

}  // namespace ppm
