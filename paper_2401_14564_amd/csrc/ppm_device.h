// ppm_device.h -- device helpers shared by the scan and backward kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ppm_kernels.h"

namespace ppm {

// f is an integral value (a floor); return f mod n in [0, n) without a division.
// NaN, inf or huge values map to a valid index, so a diverging probe can never
// address outside the grid.
__device__ __forceinline__ int wrap_index(double f, int n, double inv_n)
{
    const double dn = (double)n;
    double w = f - dn * floor(f * inv_n);
    if (w < 0.0) w += dn;
    else if (w >= dn) w -= dn;
    if (!(w >= 0.0 && w < dn)) w = 0.0;
    return (int)w;
}

// 1/sqrt(x) in FP64: hardware estimate plus one Newton step.
__device__ __forceinline__ double rsqrt_d(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x * y;
    const double r = fma(-h, y, 0.5);      // 0.5 (1 - x y^2)
    return fma(y, r, y);
}

struct Cell {
    uint32_t i000;             // flat index of corner (ix, iy, iz)
    int dx1, dy1, dz1;         // index offsets to the +x, +y, +z corners
    double tx, ty, tz;         // fractional position in the cell
    bool xin, yin, zin;        // false when the axis was clamped (field constant along it)
};

// Cell of a grid coordinate along an axis clamped to its first/last cell:
// index in [0, n-2], t in [0, 1); outside the grid the field is continued
// constantly (in = false).  The coordinate is clamped to [0, top] first, top
// the largest double below n-1 (fmax returns the non-NaN operand, so NaN lands
// at 0, in the first cell); then the truncation is the floor and at most n-2,
// and u >= n-1 gives the last cell at t = 1 - ulp(n-1), within 1e-13 of the
// edge value.
__device__ __forceinline__ int clamp_cell(double u, int n, double &t, bool &in)
{
    in = (u >= 0.0) && (u < (double)(n - 1));
    const double top =
        __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, (double)(n - 1)) - 1u);
    const double uc = fmin(fmax(u, 0.0), top);
    t = __builtin_amdgcn_fract(uc);
    return (int)uc;
}

// Cell of a grid coordinate along a periodic axis: floor(u) mod n and u - floor(u).
// A NaN or huge coordinate is clamped before the integer conversion so the
// index is always inside [0, n).
__device__ __forceinline__ int periodic_cell(double u, int n, double &t)
{
    double f = floor(u);
    t = u - f;
    f = fmin(fmax(f, -1.0e9), 1.0e9);
    int i = (int)f;
    i += (i < 0) ? n : 0;
    i -= (i >= n) ? n : 0;
    if ((unsigned)i >= (unsigned)n) {   // more than one period away (rare)
        i %= n;
        i += (i < 0) ? n : 0;
    }
    return i;
}

// Grid geometry of a kernel instance: open (x, y clamped like z), periodic in
// x and y, or read from ScanArgs::periodic at run time.
enum GridGeom { kOpen = 0, kPeriodic = 1, kRuntimeGeom = 2 };

template <int GEOM>
__device__ __forceinline__ Cell locate(const ScanArgs &a, double x, double y, double z)
{
    Cell c;
    int ix, iy;
    const bool periodic = GEOM == kRuntimeGeom ? a.periodic != 0 : GEOM == kPeriodic;
    if (periodic) {
        ix = periodic_cell(fma(x, a.ihx, a.oxi), a.gnx, c.tx);
        iy = periodic_cell(fma(y, a.ihy, a.oyi), a.gny, c.ty);
        c.xin = c.yin = true;
        c.dx1 = (ix + 1 < a.gnx) ? 1 : 1 - a.gnx;
        c.dy1 = (iy + 1 < a.gny) ? a.gnx : a.gnx * (1 - a.gny);
    } else {
        // a sample without periodic images: x,y clamped like z; the clamped
        // cell index is at most n-2, so the +x/+y corners never wrap
        ix = clamp_cell(fma(x, a.ihx, a.oxi), a.gnx, c.tx, c.xin);
        iy = clamp_cell(fma(y, a.ihy, a.oyi), a.gny, c.ty, c.yin);
        c.dx1 = 1;
        c.dy1 = a.gnx;
    }
    // z is clamped to the first/last cell: outside the grid the field is constant
    const int iz = clamp_cell(fma(z, a.ihz, a.ozi), a.gnz, c.tz, c.zin);
    const int plane = a.gnx * a.gny;
    c.i000 = (uint32_t)(iz * plane + iy * a.gnx + ix);
    c.dz1 = plane;
    return c;
}

__device__ __forceinline__ Cell locate(const ScanArgs &a, double x, double y, double z)
{
    return locate<kRuntimeGeom>(a, x, y, z);
}

// Corner load.  WIDE grids (16 B x voxels >= 4 GiB) need 64-bit addressing;
// otherwise a 32-bit byte offset from the (scalar) base address suffices.
template <bool WIDE>
__device__ __forceinline__ float3 corner(const float4 *__restrict__ ff, uint32_t i)
{
    if (WIDE) {
        const float4 *p = ff + (size_t)i;
        return make_float3(p->x, p->y, p->z);
    } else {
        const float4 *p = reinterpret_cast<const float4 *>(
            reinterpret_cast<const char *>(ff) + (uint32_t)(i * 16u));
        return make_float3(p->x, p->y, p->z);
    }
}

// The eight corner values (Fx, Fy, Fz) of a cell: v[i + 2j + 4k] is corner
// (ix + i, iy + j, iz + k).  XSTEP1: the +x corner is always the next voxel
// (clamped x), so with 32-bit offsets its 16-byte step folds into the load's
// immediate offset.
template <bool WIDE, bool XSTEP1 = false, typename CellT = Cell>
__device__ __forceinline__ void gather8(const float4 *__restrict__ ff, const CellT &c, float3 *v)
{
    if constexpr (!WIDE && XSTEP1) {
        const char *b = reinterpret_cast<const char *>(ff);
        const uint32_t o00 = c.i000 * 16u;
        const uint32_t o10 = o00 + (uint32_t)c.dy1 * 16u;
        const uint32_t o01 = o00 + (uint32_t)c.dz1 * 16u;
        const uint32_t o11 = o01 + (uint32_t)c.dy1 * 16u;
        const char *p00 = b + o00, *p10 = b + o10, *p01 = b + o01, *p11 = b + o11;
        auto ld = [](const char *p) {
            const float4 *q = reinterpret_cast<const float4 *>(p);
            return make_float3(q->x, q->y, q->z);
        };
        v[0] = ld(p00);
        v[1] = ld(p00 + 16);
        v[2] = ld(p10);
        v[3] = ld(p10 + 16);
        v[4] = ld(p01);
        v[5] = ld(p01 + 16);
        v[6] = ld(p11);
        v[7] = ld(p11 + 16);
        // keep the offsets live past the loads: a load whose destination is the
        // address register of the load before it costs a wait state on gfx950,
        // which the register allocator would otherwise create
        asm volatile("" ::"v"(o00), "v"(o10), "v"(o01), "v"(o11));
    } else if constexpr (!WIDE) {
        const char *b = reinterpret_cast<const char *>(ff);
        uint32_t o[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            o[k] = (c.i000 + ((k & 1) ? (uint32_t)c.dx1 : 0u) + ((k & 2) ? (uint32_t)c.dy1 : 0u) +
                    ((k & 4) ? (uint32_t)c.dz1 : 0u)) * 16u;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float4 *q = reinterpret_cast<const float4 *>(b + o[k]);
            v[k] = make_float3(q->x, q->y, q->z);
        }
        asm volatile("" ::"v"(o[0]), "v"(o[1]), "v"(o[2]), "v"(o[3]), "v"(o[4]), "v"(o[5]),
                     "v"(o[6]), "v"(o[7]));
    } else {
        const uint32_t i0 = c.i000;
        v[0] = corner<WIDE>(ff, i0);
        v[1] = corner<WIDE>(ff, i0 + c.dx1);
        v[2] = corner<WIDE>(ff, i0 + c.dy1);
        v[3] = corner<WIDE>(ff, i0 + c.dx1 + c.dy1);
        v[4] = corner<WIDE>(ff, i0 + c.dz1);
        v[5] = corner<WIDE>(ff, i0 + c.dz1 + c.dx1);
        v[6] = corner<WIDE>(ff, i0 + c.dz1 + c.dy1);
        v[7] = corner<WIDE>(ff, i0 + c.dz1 + c.dx1 + c.dy1);
    }
}

}  // namespace ppm
