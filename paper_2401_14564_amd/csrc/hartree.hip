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
//   pack      Z = V + i alpha rho, formed by the first x pass as it reads the two
//             real fields (one transform for both; alpha puts them on one scale,
//             so that splitting the transform into its Hermitian parts does not
//             bury rho^ under the rounding of V^, and, being a power of two,
//             changes no digit)
//   3 x fft   Z^ (forward), one kernel per axis
//   spectral  V^ = (Z^[k] + conj Z^[-k]) / 2,  rho^ = (Z^[k] - conj Z^[-k]) / (2i alpha),
//             A = E^ + i F^_z = (1 + kappa_z) E^,  B = F^_x + i F^_y = (kappa_y - i kappa_x) E^,
//             with 1/N folded into E^
//   6 x fft   A, B (inverse); the last z pass of B writes
//             ff = (Re B, Im B, Im A, Re A) to the grid (or adds to it)
//
// FFT kernel: a block transforms L lines of one axis in LDS with a mixed-radix
// (16, 15, 4, 2, 3, 5) Stockham sequence, radix 16 and 15 computed in registers
// as 4 x 4 and 3 x 5; each stage reads its inputs into registers,
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
constexpr int kFftLdsElems = 4096;       // at most 64 KiB of double2: data + twiddles
constexpr int kFftMaxLines = 16;         // lines per block (runs of 16 x 16 B on y/z)

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

// x / d for the small indices of the FFT (see FftPlan): rcp = 0 means d = 1.
__device__ __forceinline__ int fdiv(int x, unsigned rcp)
{
    return rcp ? (int)__umulhi((unsigned)x, rcp) : x;
}

// In-place DFT of u[0 .. P-1] (forward sign -1, inverse +1), natural order in
// and out.  P = 2, 3, 4, 5: butterflies on exact constants.  P = 16 = 4 x 4 and
// P = 15 = 3 x 5: Cooley-Tukey in registers, X[k1 + N1 k2] =
// sum_b W_P^(b k1) W_N2^(b k2) sum_a u[N2 a + b] W_N1^(a k1), the internal
// twiddles W_P^j read from the line's twiddle table (tw[j n / P]).
template <int P>
__device__ __forceinline__ void dft(double2 *u, bool inverse, const double2 *tw, int n)
{
    if constexpr (P == 2) {
        const double2 a = u[0], b = u[1];
        u[0] = cadd(a, b);
        u[1] = csub(a, b);
    } else if constexpr (P == 4) {
        // (sign i)^(s t): forward sign -1, inverse +1
        const double2 a = cadd(u[0], u[2]), b2 = csub(u[0], u[2]);
        const double2 c = cadd(u[1], u[3]), d = csub(u[1], u[3]);
        const double2 id = inverse ? make_double2(-d.y, d.x) : make_double2(d.y, -d.x);
        u[0] = cadd(a, c);
        u[1] = cadd(b2, id);
        u[2] = csub(a, c);
        u[3] = csub(b2, id);
    } else if constexpr (P == 3) {
        // w = exp(-+2 pi i / 3): y1,2 = u0 - a/2 -+ i sqrt(3)/2 b
        const double2 a = cadd(u[1], u[2]), d = csub(u[1], u[2]);
        const double2 t = make_double2(u[0].x - 0.5 * a.x, u[0].y - 0.5 * a.y);
        const double h = 0.86602540378443864676;                 // sqrt(3)/2
        const double2 ib = inverse ? make_double2(-h * d.y, h * d.x)
                                   : make_double2(h * d.y, -h * d.x);   // -+ i h d
        u[0] = cadd(u[0], a);
        u[1] = cadd(t, ib);
        u[2] = csub(t, ib);
    } else if constexpr (P == 5) {
        // radix 5 from the symmetric pairs u1 +- u4, u2 +- u3 and the
        // cosines/sines of 2 pi/5 and 4 pi/5
        const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;
        const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;
        const double2 a1 = cadd(u[1], u[4]), b1 = csub(u[1], u[4]);
        const double2 a2 = cadd(u[2], u[3]), b2 = csub(u[2], u[3]);
        const double2 t1 = make_double2(u[0].x + c1 * a1.x + c2 * a2.x,
                                        u[0].y + c1 * a1.y + c2 * a2.y);
        const double2 t2 = make_double2(u[0].x + c2 * a1.x + c1 * a2.x,
                                        u[0].y + c2 * a1.y + c1 * a2.y);
        const double2 t3 = make_double2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
        const double2 t4 = make_double2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
        // forward: y1 = t1 - i t3, y4 = t1 + i t3, y2 = t2 - i t4, y3 = t2 + i t4
        const double2 i3 = inverse ? make_double2(-t3.y, t3.x) : make_double2(t3.y, -t3.x);
        const double2 i4 = inverse ? make_double2(-t4.y, t4.x) : make_double2(t4.y, -t4.x);
        u[0] = make_double2(u[0].x + a1.x + a2.x, u[0].y + a1.y + a2.y);
        u[1] = cadd(t1, i3);
        u[4] = csub(t1, i3);
        u[2] = cadd(t2, i4);
        u[3] = csub(t2, i4);
    } else {
        static_assert(P == 16 || P == 15, "radix");
        constexpr int N1 = P == 16 ? 4 : 3, N2 = P == 16 ? 4 : 5;
        const int step = n / P;
        double2 y[N2][N1];
#pragma unroll
        for (int b = 0; b < N2; ++b) {
            double2 v[N1];
#pragma unroll
            for (int a = 0; a < N1; ++a) v[a] = u[N2 * a + b];
            dft<N1>(v, inverse, tw, n);
#pragma unroll
            for (int k1 = 0; k1 < N1; ++k1)
                y[b][k1] = (b == 0 || k1 == 0)
                               ? v[k1] : cmul(v[k1], cconj_if(tw[b * k1 * step], inverse));
        }
#pragma unroll
        for (int k1 = 0; k1 < N1; ++k1) {
            double2 z[N2];
#pragma unroll
            for (int b = 0; b < N2; ++b) z[b] = y[b][k1];
            dft<N2>(z, inverse, tw, n);
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) u[k1 + N1 * k2] = z[k2];
        }
    }
}

// One Stockham stage of radix P over L lines of length n held in LDS (line
// stride LS).  m = product of the radices of the previous stages; rcp_nb and
// rcp_m the reciprocals of n/P and m.
template <int P>
__device__ __forceinline__ void fft_stage(double2 *buf, const double2 *tw, int n, int m, int L,
                                          int LS, bool inverse, unsigned rcp_nb, unsigned rcp_m)
{
    constexpr int NB = (kFftLdsElems / P + kFftThreads - 1) / kFftThreads;
    const int nb = n / P;
    const int tot = L * nb;
    const int stride = n / (m * P);          // twiddle step of this stage
    double2 y[NB][P];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int b = threadIdx.x + r * kFftThreads;
        if (b < tot) {
            const int l = fdiv(b, rcp_nb), j = b - l * nb;
            const int k = j - fdiv(j, rcp_m) * m;
            double2 u[P];
#pragma unroll
            for (int t = 0; t < P; ++t) {
                const double2 x = buf[l * LS + j + t * nb];
                u[t] = (t == 0) ? x : cmul(x, cconj_if(tw[k * t * stride], inverse));
            }
            dft<P>(u, inverse, tw, n);
#pragma unroll
            for (int t = 0; t < P; ++t) y[r][t] = u[t];
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < NB; ++r) {
        const int b = threadIdx.x + r * kFftThreads;
        if (b < tot) {
            const int l = fdiv(b, rcp_nb), j = b - l * nb;
            const int q = fdiv(j, rcp_m);
            const int k = j - q * m;
            const int o = l * LS + q * m * P + k;
#pragma unroll
            for (int t = 0; t < P; ++t) buf[o + t * m] = y[r][t];
        }
    }
    __syncthreads();
}

// Inputs and outputs of the passes that absorb the packing and unpacking.
struct FftIo {
    const float *V, *rho;         // MODE 1: the real fields packed as V + i alpha rho
    const double *alpha;
    const double2 *A;             // MODE 2: finished E + i Fz, read beside Fx + i Fy
    float4 *ff;                   // MODE 2: output grid
    int accumulate;
};

// Transform every line of one axis in place.  MODE 0: data in, data out.
// MODE 1 (first forward pass): the lines are read from V and rho instead of
// data.  MODE 2 (last inverse pass of Fx + i Fy): instead of storing the lines,
// (Fx, Fy, Fz, E) = (Re, Im of the line, Im, Re of A) is written or added to ff.
template <int MODE>
__global__ __launch_bounds__(kFftThreads) void fft_axis_kernel(double2 *__restrict__ data,
                                                               FftPlan plan, int axis, int nx,
                                                               int ny, int nz, int inverse,
                                                               FftIo io)
{
    extern __shared__ double2 lds[];        // n twiddles + L lines of stride n + 1
    const int n = plan.n, L = plan.lines, LS = n + 1;
    double2 *tw = lds;
    double2 *buf = lds + n;
    const AxisMap am = axis_map(axis, nx, ny, nz, L);
    // load: l fastest for strided axes (one contiguous run per element row);
    // all of a thread's loads are issued before the first LDS store
    constexpr int kPer = kFftLdsElems / kFftThreads;
    double2 v[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int e = threadIdx.x + r * kFftThreads;
        int l, t;
        if (axis == 0) { l = fdiv(e, plan.rcp_n); t = e - l * n; }
        else { t = fdiv(e, plan.rcp_lines); l = e - t * L; }
        v[r] = make_double2(0.0, 0.0);
        if (e < L * n && l < am.nl) {
            const long long g = am.base + l * am.lstride + (long long)t * am.tstride;
            if (MODE == 1) v[r] = make_double2((double)io.V[g], io.alpha[0] * (double)io.rho[g]);
            else v[r] = data[g];
        }
    }
    // twiddles while the loads are in flight
    for (int t = threadIdx.x; t < n; t += kFftThreads) {
        double s, c;
        sincospi(-2.0 * t / n, &s, &c);
        tw[t] = make_double2(c, s);
    }
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int e = threadIdx.x + r * kFftThreads;
        int l, t;
        if (axis == 0) { l = fdiv(e, plan.rcp_n); t = e - l * n; }
        else { t = fdiv(e, plan.rcp_lines); l = e - t * L; }
        if (e < L * n) buf[l * LS + t] = v[r];
    }
    __syncthreads();
    int m = 1;
    const bool inv = inverse != 0;
    for (int s = 0; s < plan.n_stages; ++s) {
        const int P = plan.radix[s];
        const unsigned rn = plan.rcp_nb[s], rm = plan.rcp_m[s];
        if (P == 16) fft_stage<16>(buf, tw, n, m, L, LS, inv, rn, rm);
        else if (P == 15) fft_stage<15>(buf, tw, n, m, L, LS, inv, rn, rm);
        else if (P == 4) fft_stage<4>(buf, tw, n, m, L, LS, inv, rn, rm);
        else if (P == 2) fft_stage<2>(buf, tw, n, m, L, LS, inv, rn, rm);
        else if (P == 3) fft_stage<3>(buf, tw, n, m, L, LS, inv, rn, rm);
        else fft_stage<5>(buf, tw, n, m, L, LS, inv, rn, rm);
        m *= P;
    }
    for (int e = threadIdx.x; e < L * n; e += kFftThreads) {
        int l, t;
        if (axis == 0) { l = fdiv(e, plan.rcp_n); t = e - l * n; }
        else { t = fdiv(e, plan.rcp_lines); l = e - t * L; }
        if (l < am.nl) {
            const long long g = am.base + l * am.lstride + (long long)t * am.tstride;
            if (MODE == 2) {
                const double2 a = io.A[g], b = buf[l * LS + t];
                float4 o = make_float4((float)b.x, (float)b.y, (float)a.y, (float)a.x);
                if (io.accumulate) {
                    const float4 p = io.ff[g];
                    o = make_float4(p.x + o.x, p.y + o.y, p.z + o.z, p.w + o.w);
                }
                io.ff[g] = o;
            } else {
                data[g] = buf[l * LS + t];
            }
        }
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

unsigned blocks_for(long long N, int T) { return (unsigned)((N + T - 1) / T); }

// 3-D transform: x, y, z passes.  first: MODE of the x pass (1 reads the real
// inputs); last: MODE of the z pass (2 unpacks into the grid).
hipError_t launch_fft3(double2 *data, const FftPlan plans[3], int nx, int ny, int nz, int inverse,
                       int first, int last, const FftIo &io, hipStream_t stream)
{
    for (int axis = 0; axis < 3; ++axis) {
        const int L = plans[axis].lines;
        unsigned grid;
        if (axis == 0) grid = blocks_for((long long)ny * nz, L);
        else grid = (unsigned)((nx + L - 1) / L) * (unsigned)(axis == 1 ? nz : ny);
        const size_t lds = (size_t)(plans[axis].n + L * (plans[axis].n + 1)) * sizeof(double2);
        const int mode = axis == 0 ? first : (axis == 2 ? last : 0);
        if (mode == 1)
            hipLaunchKernelGGL((fft_axis_kernel<1>), dim3(grid), dim3(kFftThreads), lds, stream,
                               data, plans[axis], axis, nx, ny, nz, inverse, io);
        else if (mode == 2)
            hipLaunchKernelGGL((fft_axis_kernel<2>), dim3(grid), dim3(kFftThreads), lds, stream,
                               data, plans[axis], axis, nx, ny, nz, inverse, io);
        else
            hipLaunchKernelGGL((fft_axis_kernel<0>), dim3(grid), dim3(kFftThreads), lds, stream,
                               data, plans[axis], axis, nx, ny, nz, inverse, io);
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
    // 16 = 4 x 4 and 15 = 3 x 5 first: each is one LDS round trip for what would
    // be two stages (a 240-point line takes two stages instead of four)
    const int radices[6] = {16, 15, 4, 2, 3, 5};
    for (int k = 0; k < 6; ++k) {
        const int P = radices[k];
        while (r % P == 0) {
            if (p->n_stages >= kMaxFftStages) return false;
            p->radix[p->n_stages++] = P;
            r /= P;
        }
    }
    if (r != 1) return false;
    // multiply-high reciprocals of n/P and of m for each stage
    int m = 1;
    for (int s = 0; s < p->n_stages; ++s) {
        const unsigned nb = (unsigned)(n / p->radix[s]);
        p->rcp_nb[s] = nb == 1 ? 0u : (unsigned)((1ull << 32) / nb + 1);
        p->rcp_m[s] = m == 1 ? 0u : (unsigned)((1ull << 32) / (unsigned)m + 1);
        m *= p->radix[s];
    }
    // lines per block: data (L lines of stride n + 1) plus n twiddles in LDS
    int L = (kFftLdsElems - n) / (n + 1);
    if (L > kFftMaxLines) L = kFftMaxLines;
    if (L < 1) return false;
    p->lines = L;
    p->rcp_n = (unsigned)((1ull << 32) / (unsigned)n + 1);               // n >= 2
    p->rcp_lines = L == 1 ? 0u : (unsigned)((1ull << 32) / (unsigned)L + 1);
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
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    FftIo io{V, rho, alpha, A, ff, accumulate};
    if ((e = launch_fft3(Z, plans, nx, ny, nz, 0, 1, 0, io, stream)) != hipSuccess) return e;
    const double two_pi = 6.283185307179586476925286766559;
    const double scale = hx * hy * hz / (double)N;
    hipLaunchKernelGGL(spectral_kernel, dim3(g), dim3(256), 0, stream, Z, A, B, nx, ny, nz,
                       two_pi / (nx * hx), two_pi / (ny * hy), two_pi / (nz * hz), scale, alpha);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_fft3(A, plans, nx, ny, nz, 1, 0, 0, io, stream)) != hipSuccess) return e;
    return launch_fft3(B, plans, nx, ny, nz, 1, 0, 2, io, stream);
}

}  // namespace ppm
