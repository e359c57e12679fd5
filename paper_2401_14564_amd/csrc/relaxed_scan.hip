// relaxed_scan.hip -- relaxed probe-particle scan with fused frequency shift.
//
// For every tip column independently, the anchor descends in z; at each height
// the probe particle is relaxed by FIRE (Sec. 5.1.1 step 2) on the net force
//   G(r) = F^T(r) + F^S_h(r)                                      (Eq. 1)
// with the tip springs F^T of Eq. 2 and F^S_h the trilinear interpolation of the
// force-field grid.  The tip force is read out as -F^T_z at the relaxed
// position (text after Eq. 2) and fed into the Giessibl frequency shift
// (Eq. 3), evaluated as a sliding dot product over a register ring.
//
// Design:
//  * One lane per tip column; a block of 16 x 16 lanes covers a compact tile of
//    columns so the gathers of a wave touch neighbouring voxels.  Tiles are
//    assigned so that consecutive tiles land on the same XCD (the hardware
//    deals blocks round-robin over 8 XCDs), which keeps a tile neighbourhood's
//    force-field band in one L2.
//  * Heights progress per lane: a lane that converges moves to its next height
//    in the same loop, so a wave runs for the largest per-column total of FIRE
//    steps rather than the sum of per-height maxima.
//  * Probe state (position, velocity, FIRE scalars) and the interpolation are
//    FP64: on gfx950 FP64 FMA issues at the same rate as unpacked FP32, and the
//    scan is bound by gather latency, so FP64 costs nothing measurable while the
//    force balance can be resolved far below the FP32 rounding of absolute
//    coordinates.  The grid itself is FP32 (16 B per voxel, one float4 gather
//    per corner).
#include "ppm_kernels.h"

namespace ppm {
namespace {

constexpr int kTX = 16, kTY = 16;

struct Cell {
    int i000;                  // flat index of corner (ix, iy, iz)
    int dx1, dy1, dz1;         // index offsets to the +x, +y, +z corners
    double tx, ty, tz;         // fractional position in the cell
    bool zin;                  // false when z was clamped
};

__device__ __forceinline__ int wrap_index(double f, int n)
{
    // f is integral; return f mod n in [0, n).  NaN, inf or huge values map to a
    // valid index (the conversion below is only reached with a finite, in-range w).
    double w = f - (double)n * floor(f / (double)n);
    if (!(w >= 0.0 && w < (double)n)) w = 0.0;
    const int i = (int)w;
    return i >= n ? n - 1 : i;
}

__device__ __forceinline__ Cell locate(const ScanArgs &a, double x, double y, double z)
{
    Cell c;
    const double ux = (x - a.ox) * a.ihx, uy = (y - a.oy) * a.ihy, uz = (z - a.oz) * a.ihz;
    const double fx = floor(ux), fy = floor(uy);
    c.tx = ux - fx;
    c.ty = uy - fy;
    const int ix = wrap_index(fx, a.gnx), iy = wrap_index(fy, a.gny);
    double fz = floor(uz);
    c.zin = true;
    if (!(fz >= 0.0)) {   // below the grid, or NaN
        fz = 0.0;
        c.tz = 0.0;
        c.zin = false;
    } else if (fz > (double)(a.gnz - 2)) {
        fz = (double)(a.gnz - 2);
        c.tz = 1.0;
        c.zin = false;
    } else {
        c.tz = uz - fz;
    }
    const int iz = (int)fz;
    const int plane = a.gnx * a.gny;
    c.i000 = iz * plane + iy * a.gnx + ix;
    c.dx1 = (ix + 1 < a.gnx) ? 1 : 1 - a.gnx;
    c.dy1 = (iy + 1 < a.gny) ? a.gnx : a.gnx * (1 - a.gny);
    c.dz1 = plane;
    return c;
}

// Trilinear interpolation of (Fx, Fy, Fz) in FP64 from FP32 corner values.
__device__ __forceinline__ void interp(const float4 *__restrict__ ff, const Cell &c,
                                       double &Fx, double &Fy, double &Fz)
{
    const int i0 = c.i000;
    const float4 v000 = ff[i0];
    const float4 v100 = ff[i0 + c.dx1];
    const float4 v010 = ff[i0 + c.dy1];
    const float4 v110 = ff[i0 + c.dx1 + c.dy1];
    const float4 v001 = ff[i0 + c.dz1];
    const float4 v101 = ff[i0 + c.dz1 + c.dx1];
    const float4 v011 = ff[i0 + c.dz1 + c.dy1];
    const float4 v111 = ff[i0 + c.dz1 + c.dx1 + c.dy1];
    const double tx = c.tx, ty = c.ty, tz = c.tz;
    const double sx = 1.0 - tx, sy = 1.0 - ty, sz = 1.0 - tz;
    const double w00 = sy * sz, w10 = ty * sz, w01 = sy * tz, w11 = ty * tz;
    const double w000 = sx * w00, w100 = tx * w00, w010 = sx * w10, w110 = tx * w10;
    const double w001 = sx * w01, w101 = tx * w01, w011 = sx * w11, w111 = tx * w11;
    Fx = w000 * v000.x + w100 * v100.x + w010 * v010.x + w110 * v110.x +
         w001 * v001.x + w101 * v101.x + w011 * v011.x + w111 * v111.x;
    Fy = w000 * v000.y + w100 * v100.y + w010 * v010.y + w110 * v110.y +
         w001 * v001.y + w101 * v101.y + w011 * v011.y + w111 * v111.y;
    Fz = w000 * v000.z + w100 * v100.z + w010 * v010.z + w110 * v110.z +
         w001 * v001.z + w101 * v101.z + w011 * v011.z + w111 * v111.z;
}

// Tip springs, Eq. 2: F^T = -k_R (|d| - R0) d/|d| - k_xy (.) (d - d0).
__device__ __forceinline__ void tip_force(const ScanArgs &a, double dx, double dy, double dz,
                                          double &Fx, double &Fy, double &Fz)
{
    const double dn = sqrt(dx * dx + dy * dy + dz * dz);
    const double fr = -a.kR * (dn - a.R0) / dn;
    Fx = fr * dx - a.kx * (dx - a.d0x);
    Fy = fr * dy - a.ky * (dy - a.d0y);
    Fz = fr * dz;
}

template <int M>
__global__ __launch_bounds__(kTX * kTY) void relaxed_scan_kernel(
    const ScanArgs a, const DfWeights wts, const float4 *__restrict__ ff, float *__restrict__ fz_out,
    float4 *__restrict__ pp_out, float *__restrict__ df_out)
{
    // XCD-aware tile order: hardware block b runs on XCD b % 8; give each XCD a
    // contiguous range of tiles.
    const int nb = gridDim.x;
    const int b = blockIdx.x;
    const int per = (nb + 7) / 8;
    const int rem = nb % 8;
    const int xcd = b % 8, loc = b / 8;
    // tiles are split into 8 ranges; ranges of the first `rem` XCDs have `per`
    // tiles, the others per-1 (when rem != 0)
    int tile;
    if (rem == 0) tile = xcd * per + loc;
    else tile = (xcd < rem) ? xcd * per + loc : rem * per + (xcd - rem) * (per - 1) + loc;
    const int ix = (tile % a.tiles_x) * kTX + (int)threadIdx.x;
    const int iy = (tile / a.tiles_x) * kTY + (int)threadIdx.y;
    if (ix >= a.snx || iy >= a.sny) return;

    const size_t plane = (size_t)a.snx * a.sny;
    const size_t col = (size_t)iy * a.snx + ix;
    const double ax = a.x0 + ix * a.sdx, ay = a.y0 + iy * a.sdy;

    // frequency-shift ring: ring[j] holds Fz of height k - (2M - j)
    float ring[2 * M + 1];
#pragma unroll
    for (int j = 0; j < 2 * M + 1; ++j) ring[j] = 0.0f;

    int k = 0;
    double az = a.z_top;
    double rx = ax + a.d0x, ry = ay + a.d0y, rz = az + a.d0z;
    double vx = 0.0, vy = 0.0, vz = 0.0;
    double dt = a.dt0, alpha = a.alpha0;
    int npos = 0, it = 0;

    while (true) {
        double Sx, Sy, Sz, Tx, Ty, Tz;
        const Cell c = locate(a, rx, ry, rz);
        interp(ff, c, Sx, Sy, Sz);
        tip_force(a, rx - ax, ry - ay, rz - az, Tx, Ty, Tz);
        const double Gx = Tx + Sx, Gy = Ty + Sy, Gz = Tz + Sz;
        const double g2 = Gx * Gx + Gy * Gy + Gz * Gz;
        if (g2 < a.f_conv2 || it >= a.max_iter) {
            // record this height
            const float fzv = (float)(-Tz);
            const size_t o = (size_t)k * plane + col;
            if (fz_out) fz_out[o] = fzv;
            if (pp_out) {
                const float itf = (g2 < a.f_conv2) ? (float)it : -(float)it;
                pp_out[o] = make_float4((float)(rx - ax - a.d0x), (float)(ry - ay - a.d0y),
                                        (float)(rz - az - a.d0z), itf);
            }
            if (M > 0) {
#pragma unroll
                for (int j = 0; j < 2 * M; ++j) ring[j] = ring[j + 1];
                ring[2 * M] = fzv;
                if (df_out && k >= 2 * a.m) {
                    float s = 0.0f;
#pragma unroll
                    for (int j = 0; j < 2 * M + 1; ++j) s = fmaf(wts.w[j], ring[j], s);
                    df_out[(size_t)(k - 2 * a.m) * plane + col] = s;
                }
            }
            if (++k >= a.snz) break;
            // warm start: keep the relaxed position, move with the anchor
            const double naz = a.z_top - k * a.sdz;
            rz += naz - az;
            az = naz;
            vx = vy = vz = 0.0;
            dt = a.dt0;
            alpha = a.alpha0;
            npos = 0;
            it = 0;
            continue;
        }
        if (it > 0) {
            const double P = Gx * vx + Gy * vy + Gz * vz;
            if (P > 0.0) {
                const double vn2 = vx * vx + vy * vy + vz * vz;
                const double sc = alpha * sqrt(vn2 / g2);
                const double om = 1.0 - alpha;
                vx = om * vx + sc * Gx;
                vy = om * vy + sc * Gy;
                vz = om * vz + sc * Gz;
                if (++npos > a.n_min) {
                    dt = fmin(dt * a.f_inc, a.dt_max);
                    alpha *= a.f_alpha;
                }
            } else {
                vx = vy = vz = 0.0;
                dt *= a.f_dec;
                alpha = a.alpha0;
                npos = 0;
            }
        }
        const double h = dt * a.inv_mass;
        vx += Gx * h;
        vy += Gy * h;
        vz += Gz * h;
        rx += vx * dt;
        ry += vy * dt;
        rz += vz * dt;
        ++it;
    }
}

// Standalone frequency shift: one lane per (x, y) column sliding along z.
template <int M>
__global__ __launch_bounds__(256) void df_kernel(const float *__restrict__ fz, int nz, int ny,
                                                  int nx, int m, const DfWeights wts,
                                                  float *__restrict__ df)
{
    const size_t plane = (size_t)nx * ny;
    const size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= plane) return;
    float ring[2 * M + 1];
#pragma unroll
    for (int j = 0; j < 2 * M + 1; ++j) ring[j] = 0.0f;
    for (int k = 0; k < nz; ++k) {
#pragma unroll
        for (int j = 0; j < 2 * M; ++j) ring[j] = ring[j + 1];
        ring[2 * M] = fz[(size_t)k * plane + col];
        if (k >= 2 * m) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j < 2 * M + 1; ++j) s = fmaf(wts.w[j], ring[j], s);
            df[(size_t)(k - 2 * m) * plane + col] = s;
        }
    }
}

// Pad the weights of half-width m into the ring layout of capacity M.
DfWeights repad(const DfWeights &w, int m, int M)
{
    DfWeights o{};
    // w.w[j] is given for capacity kMaxDfHalfWidth: ring index j <-> lag 2K - j
    const int K = kMaxDfHalfWidth;
    for (int lag = 0; lag <= 2 * m; ++lag) o.w[2 * M - lag] = w.w[2 * K - lag];
    return o;
}

}  // namespace

hipError_t launch_relaxed_scan(const ScanArgs &a, const DfWeights &w, const float4 *ff,
                               float *fz, float4 *pp, float *df, hipStream_t stream)
{
    dim3 block(kTX, kTY, 1);
    ScanArgs b = a;
    b.tiles_x = (a.snx + kTX - 1) / kTX;
    b.n_tiles = b.tiles_x * ((a.sny + kTY - 1) / kTY);
    dim3 grid(b.n_tiles, 1, 1);
    if (b.m == 0) {
        hipLaunchKernelGGL((relaxed_scan_kernel<0>), grid, block, 0, stream, b, w, ff, fz, pp,
                           nullptr);
    } else if (b.m <= 8) {
        hipLaunchKernelGGL((relaxed_scan_kernel<8>), grid, block, 0, stream, b, repad(w, b.m, 8),
                           ff, fz, pp, df);
    } else if (b.m <= 16) {
        hipLaunchKernelGGL((relaxed_scan_kernel<16>), grid, block, 0, stream, b,
                           repad(w, b.m, 16), ff, fz, pp, df);
    } else {
        hipLaunchKernelGGL((relaxed_scan_kernel<32>), grid, block, 0, stream, b,
                           repad(w, b.m, 32), ff, fz, pp, df);
    }
    return hipGetLastError();
}

hipError_t launch_df(const float *fz, int nz, int ny, int nx, int m, const DfWeights &w,
                     float *df, hipStream_t stream)
{
    const size_t plane = (size_t)nx * ny;
    dim3 block(256, 1, 1);
    dim3 grid((unsigned)((plane + 255) / 256), 1, 1);
    if (m <= 8)
        hipLaunchKernelGGL((df_kernel<8>), grid, block, 0, stream, fz, nz, ny, nx, m,
                           repad(w, m, 8), df);
    else if (m <= 16)
        hipLaunchKernelGGL((df_kernel<16>), grid, block, 0, stream, fz, nz, ny, nx, m,
                           repad(w, m, 16), df);
    else
        hipLaunchKernelGGL((df_kernel<32>), grid, block, 0, stream, fz, nz, ny, nx, m,
                           repad(w, m, 32), df);
    return hipGetLastError();
}

}  // namespace ppm
