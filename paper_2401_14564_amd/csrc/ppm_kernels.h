// ppm_kernels.h -- launch-argument structs and launcher declarations shared by
// the HIP translation units of libppm (internal; the public ABI is ppm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppm {

// Coulomb constant e^2/(4 pi eps0) in eV*A.
constexpr double kCoulomb = 14.3996454784;
// 1 eV/A^2 in N/m (exact SI).
constexpr double kEvPerA2InNewtonPerM = 16.02176634;
// Largest supported frequency-shift half-width (samples on each side).
constexpr int kMaxDfHalfWidth = 32;

// ---------------------------------------------------------------- FF build
struct FFArgs {
    double ox, oy, oz;        // grid origin (A)
    double hx, hy, hz;        // voxel steps (A)
    int nx, ny, nz;
    int n_atoms;
    double R_pp, eps_pp;      // probe LJ parameters
    double kq_pp;             // k_e * q_pp
    double Lx, Ly;            // periods (periodic only)
    float rc2;                // cutoff^2 (periodic only)
    double cull2;             // (cutoff + brick half-diagonal)^2 (periodic only)
};

hipError_t launch_build_ff(const FFArgs &a, const double *pos, const double *q,
                           const double *R, const double *eps, float4 *ff,
                           hipStream_t stream);

// ------------------------------------------------------------ relaxed scan
struct ScanArgs {
    // grid (interpolation)
    double ox, oy, oz;
    double ihx, ihy, ihz;     // inverse steps
    int gnx, gny, gnz;
    // probe
    double kx, ky, kR, R0;
    double d0x, d0y, d0z;
    // FIRE
    double dt0, dt_max, f_inc, f_dec, alpha0, f_alpha, inv_mass, f_conv2;
    int n_min, max_iter;
    // tip lattice
    double x0, y0, sdx, sdy, z_top, sdz;
    int snx, sny, snz;
    // frequency shift
    int m;                    // half-width, 0 if no fused output
    int ndf;                  // snz - 2m
    int tiles_x, n_tiles;     // tile decomposition of the tip lattice
};

// Frequency-shift weights padded to the ring-buffer length 2*kMaxDfHalfWidth+1,
// prefactor included: df(o) = sum_j w[j] * ring[j], ring[j] = Fz(k - (2M - j)).
struct DfWeights {
    float w[2 * kMaxDfHalfWidth + 1];
};

hipError_t launch_relaxed_scan(const ScanArgs &a, const DfWeights &w, const float4 *ff,
                               float *fz, float4 *pp, float *df, hipStream_t stream);

hipError_t launch_df(const float *fz, int nz, int ny, int nx, int m, const DfWeights &w,
                     float *df, hipStream_t stream);

// ---------------------------------------------------------------- backward
struct BwdArgs {
    ScanArgs s;               // same grid/probe/scan description as the forward
    double hx, hy, hz;        // grid steps
    int periodic;             // minimum image in x,y
    double Lx, Ly;
    float rc2;
    int n_atoms;
    double R_pp, eps_pp, kq_pp, ke_qpp;
    int eq_per_block;         // equilibria handled by one block of the scatter
    int n_eq_blocks;          // number of equilibrium chunks
};

hipError_t launch_backward(const BwdArgs &a, const DfWeights &w, const float4 *ff,
                           const float4 *pp, const float *grad_df, const double *pos,
                           const double *q, const double *R, const double *eps,
                           float4 *eq_ws, double *partial_ws, double *g_pos, double *g_q,
                           double *g_R, double *g_eps, hipStream_t stream);

}  // namespace ppm
