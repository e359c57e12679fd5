// microbench.hip -- ceilings for the two hot kernels' rooflines on gfx950.
//
// Measurement kernels only (libppm_microbench.so, loaded by the benchmark); the
// probe-particle library does not use them.
//
//  * mb_gather: the access pattern of the relaxed scan's force evaluation --
//    each lane loads the eight float4 corners of one trilinear cell per step --
//    at full occupancy with cell positions that do not depend on the loaded
//    values, so the rate is what the memory hierarchy delivers rather than a
//    dependency chain.  The band (at most 2 MiB, so that every XCD's 4 MiB L2
//    holds it) makes the traffic L2-resident after the first touch.  Coherent
//    mode: a wave's 64 lanes are 16 x 4 neighbouring columns that drift down in
//    z with a one-voxel lateral jitter, as the scan's probes do; random mode:
//    every lane picks its cell anywhere in the band (L1 misses, L2 hits).
//  * mb_pair: the force-field build's pair body (LJ + Coulomb, FP32, one
//    v_rsq_f32 per pair, packed FP32 disabled like the library) over eight
//    voxels of a thread's z-column, atoms broadcast from LDS, no global memory
//    traffic and no culling: the issue ceiling of that instruction mix.  The
//    periodic variant adds the cutoff mask and the shifted-force terms.
//  * mb_issue: the VALU issue rate of one instruction kind, eight independent
//    chains per lane at 32 waves per CU: FP32 FMA with vector operands only,
//    FP32 FMA with one wave-uniform (scalar-register) factor, FP64 FMA with
//    vector operands, FP32 reciprocal square root.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ppm_microbench.h"

namespace {

__device__ __forceinline__ uint32_t mb_hash(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// band: float4 [bz][by][bx] with bx = by = 64, bz = 32 (2 MiB)
constexpr int kBX = 64, kBY = 64, kBZ = 32;

template <bool COHERENT>
__global__ __launch_bounds__(256) void mb_gather_kernel(const float4 *__restrict__ band,
                                                        int iters, uint32_t seed,
                                                        float4 *__restrict__ out)
{
    const int tid = blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    uint32_t s = mb_hash(seed ^ (uint32_t)tid);
    // the wave's tile of 16 x 4 columns, placed at random (same for all lanes)
    const uint32_t w = mb_hash(seed + 0x9e3779b9u * (uint32_t)(tid >> 6));
    const int tx = (int)(w & 31u), ty = (int)((w >> 5) & 31u), tz = (int)((w >> 10) & 31u);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    constexpr size_t plane = (size_t)kBX * kBY;
    for (int i = 0; i < iters; ++i) {
        s = s * 1664525u + 1013904223u;
        int ix, iy, iz;
        if (COHERENT) {
            ix = tx + (lane & 15) + (int)((s >> 20) & 1u);
            iy = ty + (lane >> 4) + (int)((s >> 21) & 1u);
            iz = (tz + (i >> 2)) & (kBZ - 1);
        } else {
            ix = (int)((s >> 8) & (kBX - 1));
            iy = (int)((s >> 14) & (kBY - 1));
            iz = (int)((s >> 20) & (kBZ - 1));
        }
        ix = min(ix, kBX - 2);
        iy = min(iy, kBY - 2);
        iz = min(iz, kBZ - 2);
        const float4 *p = band + (size_t)iz * plane + (size_t)iy * kBX + ix;
        const float4 v0 = p[0], v1 = p[1], v2 = p[kBX], v3 = p[kBX + 1];
        const float4 v4 = p[plane], v5 = p[plane + 1], v6 = p[plane + kBX],
                     v7 = p[plane + kBX + 1];
        acc.x += ((v0.x + v1.x) + (v2.x + v3.x)) + ((v4.x + v5.x) + (v6.x + v7.x));
        acc.y += ((v0.y + v1.y) + (v2.y + v3.y)) + ((v4.y + v5.y) + (v6.y + v7.y));
        acc.z += ((v0.z + v1.z) + (v2.z + v3.z)) + ((v4.z + v5.z) + (v6.z + v7.z));
        acc.w += ((v0.w + v1.w) + (v2.w + v3.w)) + ((v4.w + v5.w) + (v6.w + v7.w));
    }
    out[tid] = acc;
}

constexpr int kPairVox = 8;

template <bool PERIODIC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 4))) void mb_pair_kernel(
    int reps, float *__restrict__ out)
{
    __shared__ float4 s_geo[256], s_par[256];
    __shared__ float2 s_sf[256];
    const int tid = threadIdx.x;
    {   // synthetic atoms 3 to 11 A from the brick centre
        const uint32_t h = mb_hash(0x51ed27u + (uint32_t)tid);
        const float r = 3.0f + 8.0f * (float)(h & 1023u) / 1024.0f;
        const float th = 3.14159265f * (float)((h >> 10) & 1023u) / 1024.0f;
        const float ph = 6.2831853f * (float)((h >> 20) & 1023u) / 1024.0f;
        // A = e R^12 and B = 2 e R^6 for e = 0.005 eV, R^2 = 12 A^2
        s_geo[tid] = make_float4(r * sinf(th) * cosf(ph), r * sinf(th) * sinf(ph), r * cosf(th),
                                 14929.92f);
        s_par[tid] = make_float4(179159.04f, -103.68f, 0.2f * ((tid & 1) ? 1.f : -1.f), -17.28f);
        s_sf[tid] = make_float2(1e-3f, 2e-2f);
    }
    __syncthreads();
    const float vx = 0.1f * (float)(tid & 15) - 0.75f, vy = 0.1f * (float)(tid >> 4) - 0.75f;
    float vz[kPairVox];
#pragma unroll
    for (int k = 0; k < kPairVox; ++k) vz[k] = 0.1f * (float)k - 0.35f;
    float Fx[kPairVox], Fy[kPairVox], Fz[kPairVox], E[kPairVox];
#pragma unroll
    for (int k = 0; k < kPairVox; ++k) Fx[k] = Fy[k] = Fz[k] = E[k] = 0.f;
    const float rc2 = 144.0f;
    for (int rep = 0; rep < reps; ++rep) {
        for (int j = 0; j < 256; ++j) {
            const float4 g = s_geo[j];
            const float4 p = s_par[j];
            const float2 sf = PERIODIC ? s_sf[j] : make_float2(0.f, 0.f);
            const float dx = vx - g.x, dy = vy - g.y;
            const float dxy2 = fmaf(dx, dx, dy * dy);
#pragma unroll
            for (int k = 0; k < kPairVox; ++k) {
                const float dz = vz[k] - g.z;
                const float r2 = fmaf(dz, dz, dxy2);
                float ir = __builtin_amdgcn_rsqf(r2);
                const bool in = !PERIODIC || r2 < rc2;
                if (PERIODIC) ir = in ? ir : 0.0f;
                const float ir2 = ir * ir;
                const float ir4 = ir2 * ir2;
                const float ir6 = ir4 * ir2;
                const float ec = p.z * ir;
                float e = fmaf(fmaf(g.w, ir6, p.w), ir6, E[k]);
                if (PERIODIC) {
                    e += fmaf(fmaf(sf.x, r2, p.z), ir, in ? -sf.y : 0.0f);
                } else {
                    e += ec;
                }
                E[k] = e;
                float f = fmaf(fmaf(p.x, ir6, p.y), ir6, ec) * ir2;
                if (PERIODIC) f = fmaf(-sf.x, ir, f);
                Fx[k] = fmaf(f, dx, Fx[k]);
                Fy[k] = fmaf(f, dy, Fy[k]);
                Fz[k] = fmaf(f, dz, Fz[k]);
            }
        }
    }
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kPairVox; ++k) acc += Fx[k] + Fy[k] + Fz[k] + E[k];
    out[blockIdx.x * 256 + tid] = acc;
}

// VALU issue-rate chains.  y: lane-varying factors (vector registers); s: a
// kernel argument, so the compiler reads it from a scalar register.
template <int KIND>
__global__ __launch_bounds__(256) void mb_issue_kernel(int iters, float s, float *__restrict__ out)
{
    const int tid = threadIdx.x;
    using T = typename std::conditional<KIND == 2, double, float>::type;
    T x[8], y[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        x[c] = (T)(1.0f + 1e-3f * (float)((tid + c) & 7));
        y[c] = (T)(0.5f + 1e-3f * (float)((tid * 3 + c) & 7));
    }
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if constexpr (KIND == 0 || KIND == 2) x[c] = x[c] * y[c] + y[(c + 1) & 7];
            if constexpr (KIND == 1) x[c] = fmaf(x[c], s, y[c]);
            if constexpr (KIND == 3) x[c] = __builtin_amdgcn_rsqf(x[c]);
        }
    }
    T acc = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) acc += x[c];
    out[blockIdx.x * 256 + tid] = (float)acc;
}

}  // namespace

extern "C" {

size_t ppm_mb_gather_band_bytes(void) { return (size_t)kBX * kBY * kBZ * sizeof(float4); }

int ppm_mb_gather(const float *band, int coherent, int blocks, int iters, uint32_t seed,
                  float *out, void *stream)
{
    if (!band || !out || blocks < 1 || iters < 1) return -1;
    const float4 *b = reinterpret_cast<const float4 *>(band);
    float4 *o = reinterpret_cast<float4 *>(out);
    if (coherent)
        hipLaunchKernelGGL(mb_gather_kernel<true>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           b, iters, seed, o);
    else
        hipLaunchKernelGGL(mb_gather_kernel<false>, dim3(blocks), dim3(256), 0,
                           (hipStream_t)stream, b, iters, seed, o);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ppm_mb_pair(int periodic, int blocks, int reps, float *out, void *stream)
{
    if (!out || blocks < 1 || reps < 1) return -1;
    if (periodic)
        hipLaunchKernelGGL(mb_pair_kernel<true>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           reps, out);
    else
        hipLaunchKernelGGL(mb_pair_kernel<false>, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           reps, out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int ppm_mb_issue(int kind, int blocks, int iters, float *out, void *stream)
{
    if (!out || blocks < 1 || iters < 1 || kind < 0 || kind > 3) return -1;
    const hipStream_t st = (hipStream_t)stream;
    switch (kind) {
    case 0: hipLaunchKernelGGL(mb_issue_kernel<0>, dim3(blocks), dim3(256), 0, st, iters, 0.5f, out); break;
    case 1: hipLaunchKernelGGL(mb_issue_kernel<1>, dim3(blocks), dim3(256), 0, st, iters, 0.5f, out); break;
    case 2: hipLaunchKernelGGL(mb_issue_kernel<2>, dim3(blocks), dim3(256), 0, st, iters, 0.5f, out); break;
    default: hipLaunchKernelGGL(mb_issue_kernel<3>, dim3(blocks), dim3(256), 0, st, iters, 0.5f, out); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
