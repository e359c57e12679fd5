// ppm_device.h -- device helpers shared by the scan and backward kernels.
#pragma once

#include <hip/hip_runtime.h>

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

}  // namespace ppm
