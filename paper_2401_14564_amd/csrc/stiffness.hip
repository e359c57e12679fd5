// stiffness.hip -- lateral vibration stiffness of the probe at relaxed points.
//
// The stiffness of the probe's lateral vibration modes is changed by the
// curvature of the tip-sample interaction (Sec. 3.3, the basis of the IETS
// contrast).  At a relaxed point the stiffness matrix is K = -dG/dr, G = F^T +
// F^S_h (Eq. 1, Eq. 2, trilinear cell Jacobian of the grid force); the
// symmetric part of K has one stiff (radial) mode and two soft (lateral)
// modes, whose eigenvalues this post-pass writes for every point of a scan.
//
// One lane per relaxed point; the eigenvalues of the symmetric 3x3 matrix come
// from the closed-form trigonometric solution of its characteristic cubic.
#include "ppm.h"
#include "ppm_device.h"
#include "ppm_kernels.h"

namespace ppm {
namespace {

template <bool WIDE>
__global__ __launch_bounds__(256) void lateral_stiffness_kernel(const ScanArgs a,
                                                                const float4 *__restrict__ ff,
                                                                const float4 *__restrict__ pp,
                                                                float2 *__restrict__ out)
{
    const size_t plane = (size_t)a.snx * a.sny;
    const size_t n = plane * a.snz;
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const float4 st = pp[idx];
    if (!(st.w >= 0.0f)) {   // not converged: no stiffness
        out[idx] = make_float2(__builtin_nanf(""), __builtin_nanf(""));
        return;
    }
    const int k = (int)(idx / plane);
    const size_t col = idx - (size_t)k * plane;
    const int iy = (int)(col / a.snx), ix = (int)(col - (size_t)iy * a.snx);
    const double dx = a.d0x + st.x, dy = a.d0y + st.y, dz = a.d0z + st.z;   // r - anchor
    const double x = a.x0 + ix * a.sdx + dx, y = a.y0 + iy * a.sdy + dy,
                 z = a.z_top - k * a.sdz + dz;
    const Cell c = locate(a, x, y, z);
    float3 v[8];
    gather8<WIDE>(ff, c, v);
    const double tx = c.tx, ty = c.ty, tz = c.tz;
    const double sx = 1.0 - tx, sy = 1.0 - ty, sz = 1.0 - tz;
    const double ihx = c.xin ? a.ihx : 0.0, ihy = c.yin ? a.ihy : 0.0;
    const double ihz = c.zin ? a.ihz : 0.0;
    // trilinear Jacobian J[r][s] = dF_r / d x_s
    double J[3][3];
    const double wyz[4] = {sy * sz, ty * sz, sy * tz, ty * tz};   // weights of the x-edges
    const double wxz[4] = {sx * sz, tx * sz, sx * tz, tx * tz};   // of the y-edges
    const double wxy[4] = {sx * sy, tx * sy, sx * ty, tx * ty};   // of the z-edges
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // x-edge e joins corners (0, j, k) and (1, j, k) with j = e & 1, k = e >> 1
            const int j = e & 1, kk = e >> 1;
            const float3 a0 = v[2 * j + 4 * kk], a1 = v[1 + 2 * j + 4 * kk];
            // y-edge e joins (i, 0, k) and (i, 1, k) with i = e & 1
            const float3 b0 = v[(e & 1) + 4 * kk], b1 = v[(e & 1) + 2 + 4 * kk];
            // z-edge e joins (i, j, 0) and (i, j, 1) with i = e & 1, j = e >> 1
            const float3 c0 = v[(e & 1) + 2 * (e >> 1)], c1 = v[(e & 1) + 2 * (e >> 1) + 4];
            const double da = r == 0 ? (double)a1.x - a0.x : (r == 1 ? (double)a1.y - a0.y
                                                                        : (double)a1.z - a0.z);
            const double db = r == 0 ? (double)b1.x - b0.x : (r == 1 ? (double)b1.y - b0.y
                                                                        : (double)b1.z - b0.z);
            const double dc = r == 0 ? (double)c1.x - c0.x : (r == 1 ? (double)c1.y - c0.y
                                                                        : (double)c1.z - c0.z);
            gx += wyz[e] * da;
            gy += wxz[e] * db;
            gz += wxy[e] * dc;
        }
        J[r][0] = gx * ihx;
        J[r][1] = gy * ihy;
        J[r][2] = gz * ihz;
    }
    // spring Jacobian dF^T/dr = -k_R [(1 - R0/|d|) I + R0 d d^T/|d|^3] - diag(kx, ky, 0)
    const double id = rsqrt_d(dx * dx + dy * dy + dz * dz);
    const double c1 = 1.0 - a.R0 * id, c2 = a.R0 * id * id * id;
    const double d[3] = {dx, dy, dz};
    double S[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double jt = -a.kR * ((i == j ? c1 : 0.0) + c2 * d[i] * d[j]);
            S[i][j] = -(jt + 0.5 * (J[i][j] + J[j][i]));
        }
    S[0][0] += a.kx;
    S[1][1] += a.ky;
    // eigenvalues of the symmetric S (characteristic cubic, trigonometric form)
    const double p1 = S[0][1] * S[0][1] + S[0][2] * S[0][2] + S[1][2] * S[1][2];
    double e0, e1, e2;
    if (p1 == 0.0) {
        e0 = S[0][0];
        e1 = S[1][1];
        e2 = S[2][2];
    } else {
        const double q = (S[0][0] + S[1][1] + S[2][2]) / 3.0;
        const double a0 = S[0][0] - q, a1 = S[1][1] - q, a2 = S[2][2] - q;
        const double p2 = a0 * a0 + a1 * a1 + a2 * a2 + 2.0 * p1;
        const double p = sqrt(p2 / 6.0);
        const double ip = 1.0 / p;
        const double b00 = a0 * ip, b11 = a1 * ip, b22 = a2 * ip;
        const double b01 = S[0][1] * ip, b02 = S[0][2] * ip, b12 = S[1][2] * ip;
        double rr = 0.5 * (b00 * (b11 * b22 - b12 * b12) - b01 * (b01 * b22 - b12 * b02) +
                           b02 * (b01 * b12 - b11 * b02));
        rr = fmin(fmax(rr, -1.0), 1.0);
        const double phi = acos(rr) / 3.0;
        e2 = q + 2.0 * p * cos(phi);                               // largest
        e0 = q + 2.0 * p * cos(phi + 2.0943951023931954923);       // smallest
        e1 = 3.0 * q - e0 - e2;
    }
    // two smallest, ascending
    double lo = fmin(e0, fmin(e1, e2)), hi_ = fmax(e0, fmax(e1, e2));
    const double mid = e0 + e1 + e2 - lo - hi_;
    out[idx] = make_float2((float)lo, (float)mid);
}

}  // namespace

hipError_t launch_lateral_stiffness(const ScanArgs &a, const float4 *ff, const float4 *pp,
                                    float *out, hipStream_t stream)
{
    const size_t n = (size_t)a.snx * a.sny * a.snz;
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256), 1, 1);
    const double bytes = 16.0 * a.gnx * (double)a.gny * a.gnz;
    if (bytes >= 4294967296.0)
        hipLaunchKernelGGL((lateral_stiffness_kernel<true>), grid, dim3(256), 0, stream, a, ff, pp,
                           reinterpret_cast<float2 *>(out));
    else
        hipLaunchKernelGGL((lateral_stiffness_kernel<false>), grid, dim3(256), 0, stream, a, ff,
                           pp, reinterpret_cast<float2 *>(out));
    return hipGetLastError();
}

}  // namespace ppm
