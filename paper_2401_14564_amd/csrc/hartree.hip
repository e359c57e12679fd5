// hartree.hip -- electrostatics of the probe from a sample potential given on
// the grid (Sec. 2.2.3), by the convolution theorem (Sec. 5.1.2).
//
// The probe's energy is the cross-correlation of its charge density rho with
// the sample potential V,
//     E[j] = dV sum_i rho[i] V[i + j]          (periodic grid, dV = hx hy hz),
// and its force is F = -grad E, the gradient of E's trigonometric interpolant.
// In Fourier space (unnormalised forward DFT, hat) this is
//     E^ = dV conj(rho^) V^,      F^_c = -i kappa_c E^,
// kappa the signed angular wavenumbers (Nyquist term of an even axis zeroed so
// that every output stays real).
//
// Pipeline (all FP64 complex, the grid taken periodic in x, y and z):
//   absmax    alpha = 2^(e_V - e_rho), e the binary exponents of max|V|, max|rho|
//             (two deterministic reduction kernels; no atomics)
//   pack      Z = V + i alpha rho                (two real fields, one transform;
//             alpha puts both on one scale, so that splitting the transform into
//             its Hermitian parts does not bury rho^ under the rounding of V^,
//             and, being a power of two, changes no digit)
//   3 x fft   Z^ (forward), one kernel per axis
//   spectral  V^ = (Z^[k] + conj Z^[-k]) / 2,  rho^ = (Z^[k] - conj Z^[-k]) / (2i alpha),
//             A = E^ + i F^_z = (1 + kappa_z) E^,  B = F^_x + i F^_y = (kappa_y - i kappa_x) E^,
//             with 1/N folded into E^
//   6 x fft   A, B (inverse)
//   unpack    ff = (Re B, Im B, Im A, Re A), written or added to the grid
//
// FFT kernel: a block transforms L lines of one axis in LDS with a mixed-radix
// (4, 2, 3, 5) Stockham sequence; each stage reads its inputs into registers,
// synchronises, and writes its outputs back (one LDS buffer plus a table of
// the n twiddles exp(-2 pi i t / n), made with sincospi).  x-lines are
// contiguous; y- and z-lines are loaded L at a time from L consecutive
// x-positions, so every row of a load is one contiguous run of L * 16 bytes.
// The transforms are HBM-bound: each axis pass reads and writes 16 B per point.
#include "ppm.h"
#include "ppm_kernels.h"

namespace ppm {
namespace {

constexpr int kFftThreads = 512;
constexpr int kFftLdsElems = 4096;       // 64 KiB of double2: data + twiddles

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b)
{
    return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 csub(double2 a, double2 b)
{
    return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 cconj_if(double2 a, bool c)
{
    return make_double2(a.x, c ? -a.y : a.y);
}

// Offsets of line l, element t of an axis pass (see the header comment).
struct AxisMap {
    long long base;      // global index of (l = 0, t = 0)
    long long lstride;   // step between lines
    long long tstride;   // step between elements of a line
    int nl;              // valid lines in this block
};

__device__ __forceinline__ AxisMap axis_map(int axis, int nx, int ny, int nz, int L)
{
    AxisMap m;
    const long long nxy = (long long)nx * ny;
    if (axis == 0) {
        const long long lines = (long long)ny * nz;
        const long long l0 = (long long)blockIdx.x * L;
        m.base = l0 * nx;
        m.lstride = nx;
        m.tstride = 1;
        m.nl = (int)min((long long)L, lines - l0);
    } else {
        const int gx = (nx + L - 1) / L;          // x-groups per (z or y) row
        const int x0 = (blockIdx.x % gx) * L;
        const int r = blockIdx.x / gx;            // z (axis 1) or y (axis 2)
        m.base = (axis == 1) ? (long long)r * nxy + x0 : (long long)r * nx + x0;
        m.lstride = 1;
        m.tstride = (axis == 1) ? nx : nxy;
        m.nl = min(L, nx - x0);
    }
    return m;
}

// One Stockham stage of radix P over L lines of length n held in LDS (line
// stride LS).  m = product of the radices of the previous stages.
template <int P>
__device__ __forceinline__ void fft_stage(double2 *buf, const double2 *tw, int n, int m, int L,
                                          int LS, bool inverse)
{
    constexpr int NB = (kFftLdsElems / P + kFftThreads - 1) / kFftThreads;
    const int nb = n / P;
    const int tot = L * nb;
    const int stride = n / (m * P);          // twiddle step of this stage
    const int root = n / P;                  // table step of the radix-P roots
    double2 y[NB][P];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int b = threadIdx.x + r * kFftThreads;
        if (b < tot) {
            const int l = b / nb, j = b - l * nb;
            const int k = j % m;
            double2 u[P];
#pragma unroll
            for (int t = 0; t < P; ++t) {
                const double2 x = buf[l * LS + j + t * nb];
                u[t] = (t == 0) ? x : cmul(x, cconj_if(tw[k * t * stride], inverse));
            }
            if (P == 2) {
                y[r][0] = cadd(u[0], u[1]);
                y[r][1] = csub(u[0], u[1]);
            } else if (P == 4) {
                // (sign i)^(s t): forward sign -1, inverse +1
                const double2 a = cadd(u[0], u[2]), b2 = csub(u[0], u[2]);
                const double2 c = cadd(u[1], u[3]), d = csub(u[1], u[3]);
                const double2 id = inverse ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);
                y[r][0] = cadd(a, c);
                y[r][1] = cadd(b2, id);
                y[r][2] = csub(a, c);
                y[r][3] = csub(b2, id);
            } else {
#pragma unroll
                for (int t = 0; t < P; ++t) {
                    double2 acc = u[0];
#pragma unroll
                    for (int s = 1; s < P; ++s)
                        acc = cadd(acc, cmul(u[s], cconj_if(tw[((s * t) % P) * root], inverse)));
                    y[r][t] = acc;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int b = threadIdx.x + r * kFftThreads;
        if (b < tot) {
            const int l = b / nb, j = b - l * nb;
            const int k = j % m;
            const int o = l * LS + (j / m) * m * P + k;
#pragma unroll
            for (int t = 0; t < P; ++t) buf[o + t * m] = y[r][t];
        }
    }
    __syncthreads();
}

// Transform every line of one axis in place.
__global__ __launch_bounds__(kFftThreads) void fft_axis_kernel(double2 *__restrict__ data,
                                                               FftPlan plan, int axis, int nx,
                                                               int ny, int nz, int inverse)
{
    __shared__ double2 lds[kFftLdsElems];
    const int n = plan.n, L = plan.lines, LS = n + 1;
    double2 *tw = lds;
    double2 *buf = lds + n;
    for (int t = threadIdx.x; t < n; t += kFftThreads) {
        double s, c;
        sincospi(-2.0 * t / n, &s, &c);
        tw[t] = make_double2(c, s);
    }
    const AxisMap am = axis_map(axis, nx, ny, nz, L);
    // load: l fastest for strided axes (one contiguous run per element row)
    for (int e = threadIdx.x; e < L * n; e += kFftThreads) {
        int l, t;
        if (axis == 0) { l = e / n; t = e - l * n; }
        else { t = e / L; l = e - t * L; }
        double2 v = make_double2(0.0, 0.0);
        if (l < am.nl) v = data[am.base + l * am.lstride + (long long)t * am.tstride];
        buf[l * LS + t] = v;
    }
    __syncthreads();
    int m = 1;
    const bool inv = inverse != 0;
    for (int s = 0; s < plan.n_stages; ++s) {
        const int P = plan.radix[s];
        if (P == 4) fft_stage<4>(buf, tw, n, m, L, LS, inv);
        else if (P == 2) fft_stage<2>(buf, tw, n, m, L, LS, inv);
        else if (P == 3) fft_stage<3>(buf, tw, n, m, L, LS, inv);
        else fft_stage<5>(buf, tw, n, m, L, LS, inv);
        m *= P;
    }
    for (int e = threadIdx.x; e < L * n; e += kFftThreads) {
        int l, t;
        if (axis == 0) { l = e / n; t = e - l * n; }
        else { t = e / L; l = e - t * L; }
        if (l < am.nl) data[am.base + l * am.lstride + (long long)t * am.tstride] = buf[l * LS + t];
    }
}

__global__ __launch_bounds__(256) void tip_density_kernel(int nx, int ny, int nz, double hx,
                                                          double hy, double hz, double q_pp,
                                                          double q_zz, double sigma,
                                                          float *__restrict__ rho)
{
    const long long N = (long long)nx * ny * nz;
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int ix = (int)(v % nx), iy = (int)((v / nx) % ny), iz = (int)(v / ((long long)nx * ny));
    // signed offset from the probe centre (index 0), wrapped
    const double x = ((2 * ix < nx) ? ix : ix - nx) * hx;
    const double y = ((2 * iy < ny) ? iy : iy - ny) * hy;
    const double z = ((2 * iz < nz) ? iz : iz - nz) * hz;
    const double s2 = sigma * sigma;
    const double G = exp(-(x * x + y * y + z * z) / (2.0 * s2)) /
                     (2.0 * 3.14159265358979323846 * s2 * sqrt(2.0 * 3.14159265358979323846 * s2));
    rho[v] = (float)(G * (q_pp + q_zz * (z * z / (s2 * s2) - 1.0 / s2)));
}

constexpr int kMaxParts = 1024;          // blocks of the first reduction pass

// Per-block maxima of |V| and |rho| (grid-stride; partial[b] = (max|V|, max|rho|)).
__global__ __launch_bounds__(256) void absmax_partial_kernel(const float *__restrict__ V,
                                                             const float *__restrict__ rho,
                                                             long long N,
                                                             float2 *__restrict__ partial)
{
    __shared__ float2 s[256];
    float mv = 0.0f, mr = 0.0f;
    for (long long v = (long long)blockIdx.x * 256 + threadIdx.x; v < N;
         v += (long long)gridDim.x * 256) {
        mv = fmaxf(mv, fabsf(V[v]));
        mr = fmaxf(mr, fabsf(rho[v]));
    }
    s[threadIdx.x] = make_float2(mv, mr);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const float2 o = s[threadIdx.x + w];
            s[threadIdx.x] = make_float2(fmaxf(s[threadIdx.x].x, o.x), fmaxf(s[threadIdx.x].y, o.y));
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

// alpha = 2^(e_V - e_rho) from the partial maxima (1 if either field is zero).
__global__ __launch_bounds__(256) void absmax_final_kernel(const float2 *__restrict__ partial,
                                                           int n_parts, double *__restrict__ alpha)
{
    __shared__ float2 s[256];
    float mv = 0.0f, mr = 0.0f;
    for (int b = threadIdx.x; b < n_parts; b += 256) {
        mv = fmaxf(mv, partial[b].x);
        mr = fmaxf(mr, partial[b].y);
    }
    s[threadIdx.x] = make_float2(mv, mr);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const float2 o = s[threadIdx.x + w];
            s[threadIdx.x] = make_float2(fmaxf(s[threadIdx.x].x, o.x), fmaxf(s[threadIdx.x].y, o.y));
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const float a = s[0].x, b = s[0].y;
        double r = 1.0;
        if (a > 0.0f && b > 0.0f && isfinite(a) && isfinite(b)) r = ldexp(1.0, ilogbf(a) - ilogbf(b));
        alpha[0] = r;
    }
}

__global__ __launch_bounds__(256) void pack_kernel(const float *__restrict__ V,
                                                   const float *__restrict__ rho,
                                                   const double *__restrict__ alpha,
                                                   double2 *__restrict__ Z, long long N)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < N) Z[v] = make_double2((double)V[v], alpha[0] * (double)rho[v]);
}

__device__ __forceinline__ double wavenumber(int i, int n, double two_pi_over_L)
{
    if (2 * i == n) return 0.0;
    return ((2 * i < n) ? i : i - n) * two_pi_over_L;
}

__global__ __launch_bounds__(256) void spectral_kernel(const double2 *__restrict__ Z,
                                                       double2 *__restrict__ A,
                                                       double2 *__restrict__ B, int nx, int ny,
                                                       int nz, double kx0, double ky0,
                                                       double kz0, double scale0,
                                                       const double *__restrict__ alpha)
{
    const double scale = scale0 / alpha[0];        // alpha is a power of two: exact
    const long long N = (long long)nx * ny * nz;
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const int ix = (int)(v % nx), iy = (int)((v / nx) % ny), iz = (int)(v / ((long long)nx * ny));
    const int jx = ix ? nx - ix : 0, jy = iy ? ny - iy : 0, jz = iz ? nz - iz : 0;
    const double2 zk = Z[v];
    const double2 zm = Z[((long long)jz * ny + jy) * nx + jx];
    // V^ = (zk + conj zm)/2 ; rho^ = (zk - conj zm)/(2i)
    const double2 Vh = make_double2(0.5 * (zk.x + zm.x), 0.5 * (zk.y - zm.y));
    const double2 d = make_double2(zk.x - zm.x, zk.y + zm.y);      // zk - conj zm
    const double2 Rh = make_double2(0.5 * d.y, -0.5 * d.x);         // d / (2i)
    // E^ = scale conj(rho^) V^
    const double2 Eh = make_double2(scale * (Rh.x * Vh.x + Rh.y * Vh.y),
                                    scale * (Rh.x * Vh.y - Rh.y * Vh.x));
    const double kx = wavenumber(ix, nx, kx0), ky = wavenumber(iy, ny, ky0),
                 kz = wavenumber(iz, nz, kz0);
    A[v] = make_double2((1.0 + kz) * Eh.x, (1.0 + kz) * Eh.y);
    // (ky - i kx) E^
    B[v] = make_double2(ky * Eh.x + kx * Eh.y, ky * Eh.y - kx * Eh.x);
}

__global__ __launch_bounds__(256) void unpack_kernel(const double2 *__restrict__ A,
                                                     const double2 *__restrict__ B,
                                                     float4 *__restrict__ ff, long long N,
                                                     int accumulate)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const double2 a = A[v], b = B[v];
    float4 o = make_float4((float)b.x, (float)b.y, (float)a.y, (float)a.x);
    if (accumulate) {
        const float4 p = ff[v];
        o = make_float4(p.x + o.x, p.y + o.y, p.z + o.z, p.w + o.w);
    }
    ff[v] = o;
}

unsigned blocks_for(long long N, int T) { return (unsigned)((N + T - 1) / T); }

hipError_t launch_fft3(double2 *data, const FftPlan plans[3], int nx, int ny, int nz, int inverse,
                       hipStream_t stream)
{
    for (int axis = 0; axis < 3; ++axis) {
        const int L = plans[axis].lines;
        unsigned grid;
        if (axis == 0) grid = blocks_for((long long)ny * nz, L);
        else grid = (unsigned)((nx + L - 1) / L) * (unsigned)(axis == 1 ? nz : ny);
        hipLaunchKernelGGL(fft_axis_kernel, dim3(grid), dim3(kFftThreads), 0, stream, data,
                           plans[axis], axis, nx, ny, nz, inverse);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

bool fft_plan(int n, FftPlan *p)
{
    if (n < 2 || n > kMaxFftLength) return false;
    p->n = n;
    p->n_stages = 0;
    int r = n;
    const int radices[4] = {4, 2, 3, 5};
    for (int k = 0; k < 4; ++k) {
        const int P = radices[k];
        while (r % P == 0) {
            if (p->n_stages >= kMaxFftStages) return false;
            p->radix[p->n_stages++] = P;
            r /= P;
        }
    }
    if (r != 1) return false;
    // lines per block: data (L lines of stride n + 1) plus n twiddles in LDS
    int L = (kFftLdsElems - n) / (n + 1);
    if (L > 16) L = 16;
    if (L < 1) return false;
    p->lines = L;
    return true;
}

hipError_t launch_tip_density(int nx, int ny, int nz, double hx, double hy, double hz,
                              double q_pp, double q_zz, double sigma, float *rho,
                              hipStream_t stream)
{
    const long long N = (long long)nx * ny * nz;
    hipLaunchKernelGGL(tip_density_kernel, dim3(blocks_for(N, 256)), dim3(256), 0, stream, nx, ny,
                       nz, hx, hy, hz, q_pp, q_zz, sigma, rho);
    return hipGetLastError();
}

size_t hartree_scratch_bytes() { return kMaxParts * sizeof(float2) + 256; }

hipError_t launch_hartree(const FftPlan plans[3], int nx, int ny, int nz, double hx, double hy,
                          double hz, const float *V, const float *rho, int accumulate,
                          float4 *ff, double2 *Z, double2 *A, double2 *B, void *scratch,
                          hipStream_t stream)
{
    const long long N = (long long)nx * ny * nz;
    const unsigned g = blocks_for(N, 256);
    float2 *partial = static_cast<float2 *>(scratch);
    double *alpha = reinterpret_cast<double *>(static_cast<char *>(scratch) +
                                               kMaxParts * sizeof(float2));
    const long long pb = (N + 256 * 8 - 1) / (256 * 8);
    const int n_parts = (int)(pb < kMaxParts ? pb : kMaxParts);
    hipLaunchKernelGGL(absmax_partial_kernel, dim3(n_parts), dim3(256), 0, stream, V, rho, N,
                       partial);
    hipLaunchKernelGGL(absmax_final_kernel, dim3(1), dim3(256), 0, stream, partial, n_parts,
                       alpha);
    hipLaunchKernelGGL(pack_kernel, dim3(g), dim3(256), 0, stream, V, rho, alpha, Z, N);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_fft3(Z, plans, nx, ny, nz, 0, stream)) != hipSuccess) return e;
    const double two_pi = 6.283185307179586476925286766559;
    const double scale = hx * hy * hz / (double)N;
    hipLaunchKernelGGL(spectral_kernel, dim3(g), dim3(256), 0, stream, Z, A, B, nx, ny, nz,
                       two_pi / (nx * hx), two_pi / (ny * hy), two_pi / (nz * hz), scale, alpha);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fft3(A, plans, nx, ny, nz, 1, stream)) != hipSuccess) return e;
    if ((e = launch_fft3(B, plans, nx, ny, nz, 1, stream)) != hipSuccess) return e;
    hipLaunchKernelGGL(unpack_kernel, dim3(g), dim3(256), 0, stream, A, B, ff, N, accumulate);
    return hipGetLastError();
}

}  // namespace ppm
