// relaxed_scan.hip -- relaxed probe-particle scan with fused frequency shift.
//
// For every tip column independently, the anchor descends in z; at each height
// the probe particle is relaxed by FIRE (Sec. 5.1.1 step 2) on the net force
//   G(r) = F^T(r) + F^S_h(r)                                      (Eq. 1)
// with the tip springs F^T of Eq. 2 and F^S_h the trilinear interpolation of the
// force-field grid.  The tip force is read out as -F^T_z at the relaxed
// position (text after Eq. 2) and fed into the Giessibl frequency shift
// (Eq. 3), evaluated from the lane's finished Fz column (the standalone
// df_kernel slides a register ring over a stored stack instead).
//
// Design:
//  * One lane per tip column; a block covers a compact tile of columns (16 x 16,
//    four waves, for single scans; 8 x 8 for batches) so its gathers touch
//    neighbouring voxels.  Single scans of open grids add a fifth, helper wave
//    that loads the planes the block's probes are about to enter into L2 (the
//    block publishes its per-lane progress in LDS): a gather instruction waits
//    for the slowest of the cache lines it touches, and a first touch of a
//    plane otherwise goes past L2.  Measured, the loads gain about 1% and the
//    helper's mere presence as an active, polling wave about 3% (more the more
//    often it polls; the clock is unchanged), so it keeps polling until every
//    lane is done.  Tiles are
//    assigned so that consecutive tiles land on the same XCD (the hardware
//    deals blocks round-robin over 8 XCDs), which keeps a tile neighbourhood's
//    force-field band in one L2.
//  * Heights progress per lane: a lane that converges moves to its next height
//    in the same loop, so a wave runs for the largest per-column total of FIRE
//    steps rather than the sum of per-height maxima.
//  * Two precision tiers by the convergence threshold.  Far above FP32 rounding
//    (f_conv >= kLerp32MinFconv) the probe state is its FP32 displacement from
//    the tip anchor, and FIRE, the springs (hardware 1/sqrt estimate) and the
//    interpolation are FP32 (scan_column_f32).  Below it the state is the
//    absolute FP64 position and everything is FP64 (scan_column), so the force
//    balance is resolved far below the FP32 rounding of absolute coordinates.
//    The grid is FP32 in both (16 B per voxel, one float4 gather per corner).
//  * Multiply-adds are fused only within one expression (contract(on), placed
//    before the includes so it also covers the device helpers): the kernel
//    instances (tile shape, geometry, precision, batched or single) differ in
//    control flow, and cross-statement fusion would then round differently in
//    each, while a batched scan must reproduce single scans bit for bit.
#pragma clang fp contract(on)
#include <atomic>

#include "ppm.h"
#include "ppm_device.h"
#include "ppm_kernels.h"

namespace ppm {
namespace {

constexpr int kTX = 8, kTY = 8;

// Trilinear combination of the eight corner values v[i + 2j + 4k] (gather8).
// LERP32: combine in FP32.  The corners are FP32, so FP32 weights and sums add
// rounding of the size the grid values already carry (about 1e-7 of the force)
// and save the 24 FP32 -> FP64 conversions of the FP64 combination on the
// critical path; used when the convergence threshold is far above that
// rounding (kLerp32MinFconv).
template <bool LERP32>
__device__ __forceinline__ void trilerp(const float3 *v, const Cell &c, double &Fx, double &Fy,
                                        double &Fz)
{
    const float3 v000 = v[0], v100 = v[1], v010 = v[2], v110 = v[3];
    const float3 v001 = v[4], v101 = v[5], v011 = v[6], v111 = v[7];
    if constexpr (LERP32) {
        const float tx = (float)c.tx, ty = (float)c.ty, tz = (float)c.tz;
        const float sx = 1.0f - tx, sy = 1.0f - ty, sz = 1.0f - tz;
        const float w00 = sy * sz, w10 = ty * sz, w01 = sy * tz, w11 = ty * tz;
        const float w000 = sx * w00, w100 = tx * w00, w010 = sx * w10, w110 = tx * w10;
        const float w001 = sx * w01, w101 = tx * w01, w011 = sx * w11, w111 = tx * w11;
        Fx = (double)(w000 * v000.x + w100 * v100.x + w010 * v010.x + w110 * v110.x +
                      w001 * v001.x + w101 * v101.x + w011 * v011.x + w111 * v111.x);
        Fy = (double)(w000 * v000.y + w100 * v100.y + w010 * v010.y + w110 * v110.y +
                      w001 * v001.y + w101 * v101.y + w011 * v011.y + w111 * v111.y);
        Fz = (double)(w000 * v000.z + w100 * v100.z + w010 * v010.z + w110 * v110.z +
                      w001 * v001.z + w101 * v101.z + w011 * v011.z + w111 * v111.z);
    } else {
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
}

// Tip springs, Eq. 2: F^T = -k_R (|d| - R0) d/|d| - k_xy (.) (d - d0),
// with (|d| - R0)/|d| = 1 - R0/|d|.  FAST: 1/|d| is the hardware estimate
// (relative error at most 5.3e-8 measured over [0.25, 400) A^2, an FP32-level
// error: k_R R0 5.3e-8 ~ 3e-7 eV/A for the usual springs), used together with
// the FP32 interpolation; otherwise refined by a Newton step.
template <bool FAST>
__device__ __forceinline__ void tip_force(const ScanArgs &a, double dx, double dy, double dz,
                                          double &Fx, double &Fy, double &Fz)
{
    const double d2 = dx * dx + dy * dy + dz * dz;
    const double id = FAST ? __builtin_amdgcn_rsq(d2) : rsqrt_d(d2);
    const double fr = -a.kR * fma(-a.R0, id, 1.0);
    Fx = fr * dx - a.kx * (dx - a.d0x);
    Fy = fr * dy - a.ky * (dy - a.d0y);
    Fz = fr * dz;
}

// Arithmetic type of an interpolation: FP32 when LERP32, else FP64.
template <bool LERP32> struct InterpReal { using type = double; };
template <> struct InterpReal<true> { using type = float; };

// Catmull-Rom (Keys, a = -1/2) weights of the stencil offsets -1, 0, 1, 2 and
// their derivatives with respect to the fraction t.
template <typename T>
__device__ __forceinline__ void cr_weights(T t, T *w, T *dw)
{
    const T t2 = t * t, t3 = t2 * t;
    w[0] = T(0.5) * (-t3 + T(2) * t2 - t);
    w[1] = T(0.5) * (T(3) * t3 - T(5) * t2 + T(2));
    w[2] = T(0.5) * (T(-3) * t3 + T(4) * t2 + t);
    w[3] = T(0.5) * (t3 - t2);
    dw[0] = T(0.5) * (T(-3) * t2 + T(4) * t - T(1));
    dw[1] = T(0.5) * (T(9) * t2 - T(10) * t);
    dw[2] = T(0.5) * (T(-9) * t2 + T(8) * t + T(1));
    dw[3] = T(0.5) * (T(3) * t2 - T(2) * t);
}

// Cell of the cubic stencil along a clamped axis: the trilinear lookup's
// clamp_cell (coordinate clamped to the grid box, NaN to 0; cell index at most
// n-2, so the top node is the last cell at t = 1 - ulp), written branch-free,
// so the lookup issues no compare/select chains (each costs wait states on
// gfx950).
__device__ __forceinline__ int cubic_clamp_cell(double u, int n, double &t)
{
    bool in;
    return clamp_cell(u, n, t, in);
}

// Sample force from the tricubic interpolant of the energy grid En[nz][ny][nx]
// (the paper's experimental variant of Sec. 5.1.1 step 2): F = -grad E_int,
// a 4x4x4 stencil contracted axis by axis, in FP64, or in FP32 when LERP32
// (the same threshold rule as the trilinear combination; FP32 saves the 64
// FP32 -> FP64 conversions per evaluation).  x,y wrap on a periodic
// grid; otherwise, and always for z, the point is clamped to the grid box:
// outside [0, n-1] the force is continued constantly along that axis.
// WIDE: the energy grid has 2^30 voxels or more (4 GiB), so the loads need
// 64-bit offsets; otherwise each of the 64 loads is a 32-bit byte offset (row
// offset + column offset, both computed once) from the scalar base address.
// vals/key: the stencil values of the lane's previous evaluation and the flat
// index of their cell; the 64 values are reloaded only when the cell changes.
template <bool WIDE, bool LERP32>
__device__ __forceinline__ void tricubic_force(const ScanArgs &a, const float *__restrict__ En,
                                               double x, double y, double z, float *vals,
                                               uint32_t &key, double &Fx, double &Fy,
                                               double &Fz)
{
    using T = typename InterpReal<LERP32>::type;
    double tx, ty, tz;
    int ix, iy;
    if (a.periodic) {
        ix = periodic_cell(fma(x, a.ihx, a.oxi), a.gnx, tx);
        iy = periodic_cell(fma(y, a.ihy, a.oyi), a.gny, ty);
    } else {
        ix = cubic_clamp_cell(fma(x, a.ihx, a.oxi), a.gnx, tx);
        iy = cubic_clamp_cell(fma(y, a.ihy, a.oyi), a.gny, ty);
    }
    const int iz = cubic_clamp_cell(fma(z, a.ihz, a.ozi), a.gnz, tz);
    T wx[4], dwx[4], wy[4], dwy[4], wz[4], dwz[4];
    cr_weights<T>((T)tx, wx, dwx);
    cr_weights<T>((T)ty, wy, dwy);
    cr_weights<T>((T)tz, wz, dwz);
    const uint32_t cell = (uint32_t)((iz * a.gny + iy) * a.gnx + ix);   // < 2^31 voxels
    // open x axis with n >= 4: every stencil row is read as four contiguous voxels
    // from bx = clamp(ix - 1, 0, n - 4), one 16-byte load per row; at the two edge
    // cells the clamped stencil repeats an edge voxel, which is folded into the
    // x weights below (shift = -1: nodes 0,0,1,2; +1: nodes n-3,n-2,n-1,n-1)
    const bool rows = !a.periodic && a.gnx >= 4;
    const int bx = min(max(ix - 1, 0), a.gnx - 4);
    if (cell != key) {
        key = cell;
        int xs[4], ys[4], zs[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            int i = ix + s - 1, j = iy + s - 1, k = iz + s - 1;
            if (a.periodic) {
                i += (i < 0) ? a.gnx : 0;
                i -= (i >= a.gnx) ? a.gnx : 0;
                j += (j < 0) ? a.gny : 0;
                j -= (j >= a.gny) ? a.gny : 0;
            } else {
                // min/max rather than compare-and-select (no vcc, no wait states)
                i = min(max(i, 0), a.gnx - 1);
                j = min(max(j, 0), a.gny - 1);
            }
            k = min(max(k, 0), a.gnz - 1);
            xs[s] = i;
            ys[s] = j;
            zs[s] = k;
        }
        // issue all loads first, then contract (their latency overlaps)
        if (rows) {
            struct alignas(4) Row4 { float v[4]; };
            if (WIDE) {
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const Row4 r = *reinterpret_cast<const Row4 *>(
                            En + ((size_t)zs[c] * a.gny + ys[b]) * a.gnx + bx);
#pragma unroll
                        for (int i = 0; i < 4; ++i) vals[16 * c + 4 * b + i] = r.v[i];
                    }
            } else {
                const char *base = reinterpret_cast<const char *>(En);
                uint32_t ro[16];
#pragma unroll
                for (int c = 0; c < 4; ++c)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        ro[4 * c + b] = (uint32_t)((zs[c] * a.gny + ys[b]) * a.gnx + bx) * 4u;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const Row4 v = *reinterpret_cast<const Row4 *>(base + ro[r]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) vals[4 * r + i] = v.v[i];
                }
                // offsets stay live past the loads (no load then overwrites the
                // address register of the load before it: a wait state on gfx950)
                asm volatile("" ::"v"(ro[0]), "v"(ro[1]), "v"(ro[2]), "v"(ro[3]), "v"(ro[4]),
                             "v"(ro[5]), "v"(ro[6]), "v"(ro[7]), "v"(ro[8]), "v"(ro[9]),
                             "v"(ro[10]), "v"(ro[11]), "v"(ro[12]), "v"(ro[13]), "v"(ro[14]),
                             "v"(ro[15]));
            }
        } else if (WIDE) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const float *row = En + ((size_t)zs[c] * a.gny + ys[b]) * a.gnx;
#pragma unroll
                    for (int i = 0; i < 4; ++i) vals[16 * c + 4 * b + i] = row[xs[i]];
                }
        } else {
            const char *base = reinterpret_cast<const char *>(En);
            uint32_t xo[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) xo[i] = (uint32_t)xs[i] * 4u;
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const uint32_t ro = (uint32_t)((zs[c] * a.gny + ys[b]) * a.gnx) * 4u;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        vals[16 * c + 4 * b + i] =
                            *reinterpret_cast<const float *>(base + (ro + xo[i]));
                }
        }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (rows) {
        const int shift = (ix - 1) - bx;
        const bool lo = shift < 0, hi = shift > 0;
        auto fold = [lo, hi](T *w) {
            const T w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
            w[0] = lo ? w0 + w1 : (hi ? T(0) : w0);
            w[1] = lo ? w2 : (hi ? w0 : w1);
            w[2] = lo ? w3 : (hi ? w1 : w2);
            w[3] = lo ? T(0) : (hi ? w2 + w3 : w3);
        };
        fold(wx);
        fold(dwx);
    }
    T gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const T v0 = vals[16 * c + 4 * b], v1 = vals[16 * c + 4 * b + 1],
                    v2 = vals[16 * c + 4 * b + 2], v3 = vals[16 * c + 4 * b + 3];
            const T r0 = wx[0] * v0 + wx[1] * v1 + wx[2] * v2 + wx[3] * v3;
            const T r1 = dwx[0] * v0 + dwx[1] * v1 + dwx[2] * v2 + dwx[3] * v3;
            s0 += wy[b] * r0;
            s1 += dwy[b] * r0;
            s2 += wy[b] * r1;
        }
        gx += wz[c] * s2;
        gy += wz[c] * s1;
        gz += dwz[c] * s0;
    }
    Fx = -(double)gx * a.ihx;
    Fy = -(double)gy * a.ihy;
    Fz = -(double)gz * a.ihz;
}

// A finished column's outputs: the staged Fz column written out (STAGE), and
// Eq. 3 over it: output o uses samples o .. o + 2m, wts.w[j] weighting sample
// o + j (read back from LDS, or from fz_out when not staged).
template <bool STAGE, int NL>
__device__ __forceinline__ void column_outputs(const ScanArgs &a, const DfWeights &wts,
                                               size_t col, int lane, float *__restrict__ fz_out,
                                               float *__restrict__ df_out, const float *s_col)
{
    const size_t plane = (size_t)a.snx * a.sny;
    if (STAGE && fz_out) {
        for (int kk = 0; kk < a.snz; ++kk) fz_out[(size_t)kk * plane + col] = s_col[kk * NL + lane];
    }
    if (df_out) {
        const int m2 = 2 * a.m;
        for (int o = 0; o + m2 < a.snz; ++o) {
            float s = 0.0f;
            for (int j = 0; j <= m2; ++j) {
                const float f = STAGE ? s_col[(o + j) * NL + lane]
                                      : fz_out[(size_t)(o + j) * plane + col];
                s = fmaf(wts.w[j], f, s);
            }
            df_out[(size_t)o * plane + col] = s;
        }
    }
}

// One tip column (ix, iy): all heights, then its fz output and (df_out != null)
// its frequency shift.  NL = lanes per block (the stride of the per-lane Fz
// columns in LDS).  STAGE: each finished height's Fz goes to the lane's LDS
// column s_col[k][lane] and the column is written out after the last height;
// the loop then issues no global store (on gfx950 the gathers' vmcnt waits
// also wait for earlier stores).  Otherwise Fz is stored to fz_out as each
// height finishes and the frequency shift re-reads it.
// INTERP 0: trilinear forces from the float4 grid ff; 1: tricubic potential
// from the energy grid En.  GEOM: grid geometry of the trilinear lookup
// (GridGeom).  LERP32: FP32-level arithmetic where the threshold allows it (FP32
// interpolation, hardware 1/sqrt estimate in the springs); the kernels route
// the FP32-level trilinear instances to scan_column_f32 instead, so here it
// serves the tricubic scan.
template <bool STAGE, bool WIDE, int NL, int INTERP, int GEOM, bool LERP32, bool PROG = false>
__device__ __forceinline__ void scan_column(const ScanArgs &a, const DfWeights &wts, int ix,
                                            int iy, int lane, const float4 *__restrict__ ff,
                                            float *__restrict__ fz_out,
                                            float4 *__restrict__ pp_out,
                                            float *__restrict__ df_out, float *s_col,
                                            const float *__restrict__ En = nullptr,
                                            int *s_prog = nullptr)
{
    const size_t plane = (size_t)a.snx * a.sny;
    const size_t col = (size_t)iy * a.snx + ix;
    const double ax = a.x0 + ix * a.sdx, ay = a.y0 + iy * a.sdy;

    int k = 0;
    double az = a.z_top;
    double rx = ax + a.d0x, ry = ay + a.d0y, rz = az + a.d0z;
    double vx = 0.0, vy = 0.0, vz = 0.0;
    double dt = a.dt0, alpha = a.alpha0;
    double u1x = 0.0, u1y = 0.0, u1z = 0.0;      // relaxed displacement of the previous height
    int npos = 0, it = 0;

    // One loop iteration = one force evaluation of every lane.  A lane whose
    // probe has converged (or hit max_iter) records the height and starts its
    // next height in the same iteration; the others take a FIRE step.  Both
    // successor states are computed and merged by selects, so the loop has a
    // single back edge: with a conditional `continue` the compiler splits it
    // into a per-height inner loop, and every lane then waits at each height
    // for the slowest lane of its wave.
    // corner forces (trilinear) or stencil energies (tricubic) of the lane's
    // current cell, reloaded only when the probe enters another cell (most
    // FIRE steps stay inside one voxel), so a wave's gathers carry only the
    // lanes that moved
    float3 cv[8];
    float tv[INTERP == 0 ? 1 : 64];
    uint32_t cell = 0xffffffffu;
    while (true) {
        double Gx, Gy, Gz, g2;
        bool done;
        {
            double Sx, Sy, Sz, Tx, Ty, Tz;
            if (INTERP == 0) {
                // issue the eight gathers, then evaluate the springs (independent
                // of them) while they are in flight, then interpolate
                const Cell c = locate<GEOM>(a, rx, ry, rz);
                if (c.i000 != cell) {
                    gather8<WIDE, GEOM == kOpen>(ff, c, cv);
                    cell = c.i000;
                }
                __builtin_amdgcn_sched_barrier(0);   // keep the spring math ahead of the waits
                tip_force<LERP32>(a, rx - ax, ry - ay, rz - az, Tx, Ty, Tz);
                __builtin_amdgcn_sched_barrier(0);
                trilerp<LERP32>(cv, c, Sx, Sy, Sz);
            } else {
                tricubic_force<WIDE, LERP32>(a, En, rx, ry, rz, tv, cell, Sx, Sy, Sz);
                tip_force<LERP32>(a, rx - ax, ry - ay, rz - az, Tx, Ty, Tz);
            }
            Gx = Tx + Sx;
            Gy = Ty + Sy;
            Gz = Tz + Sz;
            g2 = Gx * Gx + Gy * Gy + Gz * Gz;
            const bool conv = g2 < a.f_conv2;
            done = conv || it >= a.max_iter;
            {
                // record this height.  The LDS slots of the current height are
                // written on every iteration (the last write, at convergence,
                // is the one that stays), so no branch is needed.
                const float fzv = (float)(-Tz);
                const size_t o = (size_t)k * plane + col;
                if (STAGE) s_col[k * NL + lane] = fzv;
                else if (fz_out && done) fz_out[o] = fzv;
                if (PROG)
                    __hip_atomic_store(s_prog + lane, done ? k + 1 : k, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                if (pp_out) {
                    if (done)
                        pp_out[o] = make_float4((float)(rx - ax - a.d0x), (float)(ry - ay - a.d0y),
                                                (float)(rz - az - a.d0z),
                                                conv ? (float)it : -(float)it);
                }
            }
        }
        if (done && k + 1 >= a.snz) break;
        // (a) FIRE step.  Velocity update, branch-free (lanes of a wave disagree
        // on the sign of P): from the second step on, P > 0 mixes v towards G
        // and, after n_min such steps, grows dt and shrinks alpha; P <= 0 stops
        // the particle, shrinks dt and resets alpha.
        const double P = Gx * vx + Gy * vy + Gz * vz;
        const bool pos = (it > 0) && (P > 0.0);
        const bool neg = (it > 0) && !(P > 0.0);
        const double vn2 = vx * vx + vy * vy + vz * vz;
        // alpha |v| / |G|: a step-size heuristic, so the hardware estimate of
        // 1/sqrt (no Newton step) is accurate enough
        const double mix = alpha * vn2 * __builtin_amdgcn_rsq(vn2 * g2);
        const double sc = pos ? mix : 0.0;
        const double om = pos ? 1.0 - alpha : (neg ? 0.0 : 1.0);
        double fvx = om * vx + sc * Gx;
        double fvy = om * vy + sc * Gy;
        double fvz = om * vz + sc * Gz;
        const int fnpos = pos ? npos + 1 : (neg ? 0 : npos);
        const bool grow = pos && fnpos > a.n_min;
        // The empty asm statements pin the alternatives of each select into the
        // straight-line code: left alone, the compiler sinks them into
        // exec-masked branches, and on a single wave per SIMD the branch and
        // mask bookkeeping costs more than the selects (measured 2-6% of the
        // scan).  They change no value.
        double dtg = fmin(dt * a.f_inc, a.dt_max), dtn = dt * a.f_dec, alg = alpha * a.f_alpha;
        asm volatile("" : "+v"(dtg), "+v"(dtn), "+v"(alg));
        const double fdt = grow ? dtg : (neg ? dtn : dt);
        const double falpha = grow ? alg : (neg ? a.alpha0 : alpha);
        const double h = fdt * a.inv_mass;
        fvx += Gx * h;
        fvy += Gy * h;
        fvz += Gz * h;
        const double frx = rx + fvx * fdt, fry = ry + fvy * fdt, frz = rz + fvz * fdt;

        // (b) next height.  Warm start: the next height starts from its anchor
        // plus the relaxed displacement extrapolated linearly from this height
        // and the previous one (just the displacement after the first height);
        // v and alpha restart, dt carries over (not below dt0).
        const double ux = rx - ax, uy = ry - ay, uz = rz - az;
        const bool lin = k >= 1;
        const double ex = lin ? ux - u1x : 0.0, ey = lin ? uy - u1y : 0.0,
                     ez = lin ? uz - u1z : 0.0;
        const int kn = k + 1;
        const double azn = a.z_top - kn * a.sdz;

        // merge
        double nrx = ax + (ux + ex), nry = ay + (uy + ey), nrz = azn + (uz + ez);
        double ndt = fmax(dt, a.dt0);
        double frx_ = frx, fry_ = fry, frz_ = frz;
        asm volatile("" : "+v"(nrx), "+v"(nry), "+v"(nrz), "+v"(ndt), "+v"(frx_), "+v"(fry_),
                     "+v"(frz_));
        rx = done ? nrx : frx_;
        ry = done ? nry : fry_;
        rz = done ? nrz : frz_;
        vx = done ? 0.0 : fvx;
        vy = done ? 0.0 : fvy;
        vz = done ? 0.0 : fvz;
        dt = done ? ndt : fdt;
        alpha = done ? a.alpha0 : falpha;
        npos = done ? 0 : fnpos;
        it = done ? 0 : it + 1;
        u1x = done ? ux : u1x;
        u1y = done ? uy : u1y;
        u1z = done ? uz : u1z;
        az = done ? azn : az;
        k = done ? kn : k;
    }

    column_outputs<STAGE, NL>(a, wts, col, lane, fz_out, df_out, s_col);
}

// FP32 probe state for the FP32-level instances (LERP32, trilinear): the state is
// the displacement u = r - anchor (|u| ~ R0, so FP32 resolves it to ~5e-7 A),
// the cell lookup works on FP32 grid coordinates (the anchor's, rounded once per
// column, with the height's as top - k dz/h in FP32, plus u / h), and FIRE runs
// in FP32.  At the FP32-level thresholds this path serves (f_conv >=
// kLerp32MinFconv) the rounding of the force balance stays well below f_conv:
// ~1e-6 eV/A from the interpolation and the springs, and (stiffness x ~3e-6 A)
// from the rounded anchor coordinates (half an FP32 ulp of a grid coordinate
// below 512, times the step).
// FP64 and FP32 operations issue at the same rate on gfx950; the FP32 state
// saves the conversions around the FP32 interpolation, one of the two halves of
// every select and move, and the anchor arithmetic of the warm start.
struct CellF {
    uint32_t i000;
    int dx1, dy1, dz1;
    float tx, ty, tz;
};

// FP32 counterparts of clamp_cell / periodic_cell (same rules).
__device__ __forceinline__ int clamp_cell_f(float u, int n, float &t)
{
    const float top =
        __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, (float)(n - 1)) - 1u);
    const float uc = __builtin_amdgcn_fmed3f(u, 0.0f, top);   // clamp to [0, top]
    t = __builtin_amdgcn_fractf(uc);
    return (int)uc;
}

__device__ __forceinline__ int periodic_cell_f(float u, int n, float &t)
{
    float f = floorf(u);
    t = u - f;
    f = __builtin_amdgcn_fmed3f(f, -1.0e9f, 1.0e9f);
    int i = (int)f;
    i += (i < 0) ? n : 0;
    i -= (i >= n) ? n : 0;
    if ((unsigned)i >= (unsigned)n) {
        i %= n;
        i += (i < 0) ? n : 0;
    }
    return i;
}

template <int GEOM, bool WIDE>
__device__ __forceinline__ CellF locate_f(const ScanArgs &a, float gx, float gy, float gz)
{
    CellF c;
    int ix, iy;
    const bool periodic = GEOM == kRuntimeGeom ? a.periodic != 0 : GEOM == kPeriodic;
    if (periodic) {
        ix = periodic_cell_f(gx, a.gnx, c.tx);
        iy = periodic_cell_f(gy, a.gny, c.ty);
        // the wrapped offsets are wave-uniform; kept opaque so that the
        // selects stay selects (not a per-lane multiply of a selected factor)
        int wrap_x = 1 - a.gnx, wrap_y = a.gnx * (1 - a.gny);
        asm volatile("" : "+s"(wrap_x), "+s"(wrap_y));
        c.dx1 = (ix + 1 < a.gnx) ? 1 : wrap_x;
        c.dy1 = (iy + 1 < a.gny) ? a.gnx : wrap_y;
    } else {
        ix = clamp_cell_f(gx, a.gnx, c.tx);
        iy = clamp_cell_f(gy, a.gny, c.ty);
        c.dx1 = 1;
        c.dy1 = a.gnx;
    }
    const int iz = clamp_cell_f(gz, a.gnz, c.tz);
    const int plane = a.gnx * a.gny;
    // 32-bit kernels: planes and z extents below 2^24 voxels (scan_grid_wide)
    c.i000 = WIDE ? (uint32_t)(iz * plane + iy * a.gnx + ix)
                  : __umul24(iz, plane) + __umul24(iy, a.gnx) + (uint32_t)ix;
    c.dz1 = plane;
    return c;
}

// Trilinear combination in FP32 (the weights and summation order of trilerp).
__device__ __forceinline__ void trilerp_f(const float3 *v, float tx, float ty, float tz,
                                          float &Fx, float &Fy, float &Fz)
{
    const float3 v000 = v[0], v100 = v[1], v010 = v[2], v110 = v[3];
    const float3 v001 = v[4], v101 = v[5], v011 = v[6], v111 = v[7];
    const float sx = 1.0f - tx, sy = 1.0f - ty, sz = 1.0f - tz;
    const float w00 = sy * sz, w10 = ty * sz, w01 = sy * tz, w11 = ty * tz;
    const float w000 = sx * w00, w100 = tx * w00, w010 = sx * w10, w110 = tx * w10;
    const float w001 = sx * w01, w101 = tx * w01, w011 = sx * w11, w111 = tx * w11;
    Fx = w000 * v000.x + w100 * v100.x + w010 * v010.x + w110 * v110.x + w001 * v001.x +
         w101 * v101.x + w011 * v011.x + w111 * v111.x;
    Fy = w000 * v000.y + w100 * v100.y + w010 * v010.y + w110 * v110.y + w001 * v001.y +
         w101 * v101.y + w011 * v011.y + w111 * v111.y;
    Fz = w000 * v000.z + w100 * v100.z + w010 * v010.z + w110 * v110.z + w001 * v001.z +
         w101 * v101.z + w011 * v011.z + w111 * v111.z;
}

// scan_column for the FP32-level trilinear instances: the same loop (one force
// evaluation per lane per iteration, per-lane heights, cell cache, staged Fz,
// straight-line merge) on the FP32 displacement state described above.
template <bool STAGE, bool WIDE, int NL, int GEOM, bool PROG = false>
__device__ __forceinline__ void scan_column_f32(const ScanArgs &a, const DfWeights &wts, int ix,
                                                int iy, int lane, const float4 *__restrict__ ff,
                                                float *__restrict__ fz_out,
                                                float4 *__restrict__ pp_out,
                                                float *__restrict__ df_out, float *s_col,
                                                int *s_prog = nullptr)
{
    const size_t plane = (size_t)a.snx * a.sny;
    const size_t col = (size_t)iy * a.snx + ix;
    const double ax = a.x0 + ix * a.sdx, ay = a.y0 + iy * a.sdy;
    // grid coordinates of the anchor (x, y per column, z per height)
    const float gx0 = (float)fma(ax, a.ihx, a.oxi), gy0 = (float)fma(ay, a.ihy, a.oyi);
    const float ihx = (float)a.ihx, ihy = (float)a.ihy, ihz = (float)a.ihz;
    const float kx = (float)a.kx, ky = (float)a.ky, kR = (float)a.kR, R0 = (float)a.R0;
    const float d0x = (float)a.d0x, d0y = (float)a.d0y, d0z = (float)a.d0z;
    const float f_conv2 = (float)a.f_conv2, inv_mass = (float)a.inv_mass;
    const float dt0 = (float)a.dt0, dt_max = (float)a.dt_max, f_inc = (float)a.f_inc;
    const float f_dec = (float)a.f_dec, alpha0 = (float)a.alpha0, f_alpha = (float)a.f_alpha;

    int k = 0;
    // anchor height k at grid coordinate gztop - k dgz
    const float gztop = (float)fma(a.z_top, a.ihz, a.ozi), dgz = (float)(a.sdz * a.ihz);
    float gz0 = gztop;
    float ux = d0x, uy = d0y, uz = d0z;
    float vx = 0.0f, vy = 0.0f, vz = 0.0f;
    float dt = dt0, alpha = alpha0;
    float u1x = 0.0f, u1y = 0.0f, u1z = 0.0f;   // relaxed displacement of the previous height
    int npos = 0, it = 0;
    float3 cv[8];
    uint32_t cell = 0xffffffffu;
    while (true) {
        float Gx, Gy, Gz, g2, Tz;
        bool done;
        {
            float Sx, Sy, Sz, Tx, Ty;
            // issue the eight gathers, then the springs (independent of them)
            // while they are in flight, then interpolate
            const CellF c = locate_f<GEOM, WIDE>(a, fmaf(ux, ihx, gx0), fmaf(uy, ihy, gy0),
                                           fmaf(uz, ihz, gz0));
            if (c.i000 != cell) {
                gather8<WIDE, GEOM == kOpen>(ff, c, cv);
                cell = c.i000;
            }
            __builtin_amdgcn_sched_barrier(0);
            // tip springs, Eq. 2, on d = u: F^T = -k_R (1 - R0/|d|) d - k_xy (.) (d - d0)
            const float d2 = ux * ux + uy * uy + uz * uz;
            const float fr = -kR * fmaf(-R0, __builtin_amdgcn_rsqf(d2), 1.0f);
            Tx = fr * ux - kx * (ux - d0x);
            Ty = fr * uy - ky * (uy - d0y);
            Tz = fr * uz;
            __builtin_amdgcn_sched_barrier(0);
            trilerp_f(cv, c.tx, c.ty, c.tz, Sx, Sy, Sz);
            Gx = Tx + Sx;
            Gy = Ty + Sy;
            Gz = Tz + Sz;
            g2 = Gx * Gx + Gy * Gy + Gz * Gz;
            const bool conv = g2 < f_conv2;
            done = conv || it >= a.max_iter;
            // record this height (the LDS slot of the current height is written
            // on every iteration; the write at convergence is the one that stays)
            const size_t o = (size_t)k * plane + col;
            if (STAGE) s_col[k * NL + lane] = -Tz;
            else if (fz_out && done) fz_out[o] = -Tz;
            if (PROG)
                __hip_atomic_store(s_prog + lane, done ? k + 1 : k, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            if (pp_out) {
                if (done)
                    pp_out[o] = make_float4(ux - d0x, uy - d0y, uz - d0z,
                                            conv ? (float)it : -(float)it);
            }
        }
        if (done && k + 1 >= a.snz) break;
        // (a) FIRE step (the rules of scan_column, in FP32)
        const float P = Gx * vx + Gy * vy + Gz * vz;
        const bool pos = (it > 0) && (P > 0.0f);
        const bool neg = (it > 0) && !(P > 0.0f);
        const float vn2 = vx * vx + vy * vy + vz * vz;
        const float mix = alpha * vn2 * __builtin_amdgcn_rsqf(vn2 * g2);
        const float sc = pos ? mix : 0.0f;
        const float om = pos ? 1.0f - alpha : (neg ? 0.0f : 1.0f);
        float fvx = om * vx + sc * Gx;
        float fvy = om * vy + sc * Gy;
        float fvz = om * vz + sc * Gz;
        const int fnpos = pos ? npos + 1 : (neg ? 0 : npos);
        const bool grow = pos && fnpos > a.n_min;
        // (empty asm: keep the alternatives in straight-line code, as in scan_column;
        // min/max as compare-and-select, which needs no canonicalised operands)
        const float dti = dt * f_inc;
        float dtg = dti < dt_max ? dti : dt_max, dtn = dt * f_dec, alg = alpha * f_alpha;
        asm volatile("" : "+v"(dtg), "+v"(dtn), "+v"(alg));
        const float fdt = grow ? dtg : (neg ? dtn : dt);
        const float falpha = grow ? alg : (neg ? alpha0 : alpha);
        const float h = fdt * inv_mass;
        fvx += Gx * h;
        fvy += Gy * h;
        fvz += Gz * h;
        float fux = ux + fvx * fdt, fuy = uy + fvy * fdt, fuz = uz + fvz * fdt;

        // (b) next height: warm start from the displacement extrapolated
        // linearly from this height and the previous one; v and alpha restart,
        // dt carries over (not below dt0)
        const bool lin = k >= 1;
        const float ex = lin ? ux - u1x : 0.0f, ey = lin ? uy - u1y : 0.0f,
                    ez = lin ? uz - u1z : 0.0f;
        float nux = ux + ex, nuy = uy + ey, nuz = uz + ez;
        float ndt = dt > dt0 ? dt : dt0;
        asm volatile("" : "+v"(nux), "+v"(nuy), "+v"(nuz), "+v"(ndt), "+v"(fux), "+v"(fuy),
                     "+v"(fuz));
        const int kn = k + 1;
        const float ngz0 = fmaf(-(float)kn, dgz, gztop);
        u1x = done ? ux : u1x;
        u1y = done ? uy : u1y;
        u1z = done ? uz : u1z;
        ux = done ? nux : fux;
        uy = done ? nuy : fuy;
        uz = done ? nuz : fuz;
        vx = done ? 0.0f : fvx;
        vy = done ? 0.0f : fvy;
        vz = done ? 0.0f : fvz;
        dt = done ? ndt : fdt;
        alpha = done ? alpha0 : falpha;
        npos = done ? 0 : fnpos;
        it = done ? 0 : it + 1;
        gz0 = done ? ngz0 : gz0;
        k = done ? kn : k;
    }
    column_outputs<STAGE, NL>(a, wts, col, lane, fz_out, df_out, s_col);
}

// Grid prefetch by one extra wave per block (single scans of open grids): the
// heights ahead of the block's fastest lane whose planes are loaded, the
// lateral and vertical margins (Angstrom) around the tile's probe rest
// positions, and a bound on the polls so that the wave always ends.
constexpr int kPfAhead = 3;
constexpr double kPfHalo = 1.0, kPfZMargin = 0.5;
constexpr int kPfMaxPolls = 1 << 22;

// The helper wave reads the block's progress (s_prog[lane]: the height the lane
// works on, snz once its column is done) and loads one word of every 64-byte
// segment of the planes the probes will reach next, with device scope (they
// bypass the CU's L1 and stay in L2), so that the compute waves' gathers find
// them in L2.  The values are not used.  It polls until every lane is done
// (ending once the last planes are loaded measured slower).  hl: the helper's
// lane, 0..63.
template <int TX, int TY, typename T>
__device__ void prefetch_planes(const ScanArgs &a, const T *__restrict__ grid, int tx0,
                                int ty0, const int *s_prog, int hl)
{
    constexpr int kSeg = 64 / (int)sizeof(T);   // voxels per 64-byte segment
    auto vox = [](double u, int n) { return (int)floor(fmin(fmax(u, 0.0), (double)(n - 1))); };
    const double xl = a.x0 + tx0 * a.sdx + a.d0x, xh = xl + (TX - 1) * a.sdx;
    const double yl = a.y0 + ty0 * a.sdy + a.d0y, yh = yl + (TY - 1) * a.sdy;
    const int ix0 = vox(fma(xl - kPfHalo, a.ihx, a.oxi), a.gnx) & ~(kSeg - 1);
    const int ix1 = min(vox(fma(xh + kPfHalo, a.ihx, a.oxi), a.gnx) + 1, a.gnx - 1);
    const int iy0 = vox(fma(yl - kPfHalo, a.ihy, a.oyi), a.gny);
    const int iy1 = min(vox(fma(yh + kPfHalo, a.ihy, a.oyi), a.gny) + 1, a.gny - 1);
    const int nseg = (ix1 - ix0) / kSeg + 1;
    const int per_plane = nseg * (iy1 - iy0 + 1);
    int zlo = min(vox(fma(a.z_top + a.d0z + kPfZMargin, a.ihz, a.ozi), a.gnz) + 1, a.gnz - 1) + 1;
    unsigned acc = 0;
    for (int poll = 0; poll < kPfMaxPolls; ++poll) {
        int kmin = a.snz, kmax = 0;
        for (int j = hl; j < TX * TY; j += 64) {
            const int p = __hip_atomic_load(s_prog + j, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_WORKGROUP);
            kmin = min(kmin, p);
            kmax = max(kmax, p);
        }
        for (int o = 32; o; o >>= 1) {
            kmin = min(kmin, __shfl_xor(kmin, o));
            kmax = max(kmax, __shfl_xor(kmax, o));
        }
        if (kmin >= a.snz) break;
        const int target = min(kmax + kPfAhead, a.snz - 1);
        const int izl =
            vox(fma(a.z_top - target * a.sdz + a.d0z - kPfZMargin, a.ihz, a.ozi), a.gnz);
        if (izl < zlo) {
            const int total = (zlo - izl) * per_plane;
            for (int t0 = 0; t0 < total; t0 += 8 * 64) {
                unsigned v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int t = t0 + j * 64 + hl;
                    v[j] = 0;
                    if (t < total) {
                        const int iz = zlo - 1 - t / per_plane;
                        const int r = t % per_plane;
                        const int y = iy0 + r / nseg;
                        const int x = min(ix0 + kSeg * (r % nseg), a.gnx - 1);
                        const size_t idx = ((size_t)iz * a.gny + y) * a.gnx + x;
                        v[j] = __hip_atomic_load(reinterpret_cast<const unsigned *>(grid + idx),
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) acc += v[j];
            }
            zlo = izl;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    asm volatile("" ::"v"(acc));   // the loads' only use: keeps them from being dropped
}

template <int TX, int TY, bool STAGE, bool WIDE, int INTERP, int GEOM, bool LERP32,
          bool PF = false>
__global__ __launch_bounds__(TX * TY + (PF ? 64 : 0)) void relaxed_scan_kernel(
    const ScanArgs a, const DfWeights wts, const float4 *__restrict__ ff,
    const float *__restrict__ En, float *__restrict__ fz_out, float4 *__restrict__ pp_out,
    float *__restrict__ df_out)
{
    extern __shared__ float s_col[];   // STAGE: [snz][TX * TY]
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
    const int lane = (int)threadIdx.y * TX + (int)threadIdx.x;
    const int tiles_x = (a.snx + TX - 1) / TX;
    const int ix = (tile % tiles_x) * TX + (int)threadIdx.x;
    const int iy = (tile / tiles_x) * TY + (int)threadIdx.y;
    int *s_prog = reinterpret_cast<int *>(s_col + (STAGE ? (size_t)a.snz * TX * TY : 0));
    if constexpr (PF) {
        // threads with threadIdx.y >= TY form the helper wave; s_prog[lane] is
        // the height lane works on (snz for lanes without a column)
        if (lane < TX * TY) s_prog[lane] = (ix < a.snx && iy < a.sny) ? 0 : a.snz;
        __syncthreads();
        if ((int)threadIdx.y >= TY) {
            const int tx0 = (tile % tiles_x) * TX, ty0 = (tile / tiles_x) * TY;
            if constexpr (INTERP == 0)
                prefetch_planes<TX, TY>(a, ff, tx0, ty0, s_prog, lane - TX * TY);
            else
                prefetch_planes<TX, TY>(a, En, tx0, ty0, s_prog, lane - TX * TY);
            return;
        }
    }
    if (ix >= a.snx || iy >= a.sny) return;
    if constexpr (INTERP == 0 && LERP32)
        scan_column_f32<STAGE, WIDE, TX * TY, GEOM, PF>(a, wts, ix, iy, lane, ff, fz_out, pp_out,
                                                       df_out, s_col, s_prog);
    else
        scan_column<STAGE, WIDE, TX * TY, INTERP, GEOM, LERP32, PF>(
            a, wts, ix, iy, lane, ff, fz_out, pp_out, df_out, s_col, En, s_prog);
}

// Batched scan: one 8x8 column tile per block over all jobs of the batch.  The
// job of a tile is found by a binary search over tile_begin (wave-uniform);
// the job's probe and tip lattice, its molecule's grid and the arena offsets
// come from the tables; FIRE and frequency-shift settings are shared.
template <bool STAGE, bool WIDE, bool LERP32>
__global__ __launch_bounds__(kTX * kTY) void relaxed_scan_batch_kernel(
    const ScanArgs proto, const DfWeights wts, const ppm_batch_mol *__restrict__ mols,
    const ppm_batch_scan *__restrict__ jobs, int n_jobs, const float4 *__restrict__ arena,
    float *__restrict__ fz_arena, float *__restrict__ df_arena)
{
    extern __shared__ float s_col[];
    // XCD-aware order (as for single scans): hardware block b runs on XCD b % 8,
    // each XCD takes a contiguous range of tiles, so a job's neighbouring tiles
    // share one L2
    const long long nb = (long long)gridDim.x * gridDim.y;
    const long long b = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    const long long per = (nb + 7) / 8, rem = nb % 8, xcd = b % 8, loc = b / 8;
    const long long t = (rem == 0 || xcd < rem) ? xcd * per + loc
                                                : rem * per + (xcd - rem) * (per - 1) + loc;
    int lo = 0, hi = n_jobs - 1;              // last job with tile_begin <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].tile_begin <= t) lo = mid;
        else hi = mid - 1;
    }
    const ppm_batch_scan &J = jobs[lo];
    const ppm_batch_mol &M = mols[J.mol];
    ScanArgs a = proto;
    fill_scan_geometry(a, M.grid, J.probe, J.scan);
    const int tiles_x = (J.scan.nx + kTX - 1) / kTX;
    const long long local = t - J.tile_begin;
    if (local >= (long long)tiles_x * ((J.scan.ny + kTY - 1) / kTY)) return;   // past the end
    const int lane = (int)threadIdx.y * kTX + (int)threadIdx.x;
    const int ix = (int)(local % tiles_x) * kTX + (int)threadIdx.x;
    const int iy = (int)(local / tiles_x) * kTY + (int)threadIdx.y;
    if (ix >= a.snx || iy >= a.sny) return;
    float *fzo = fz_arena ? fz_arena + J.fz_offset : nullptr;
    float *dfo = df_arena ? df_arena + J.df_offset : nullptr;
    if constexpr (LERP32)
        scan_column_f32<STAGE, WIDE, kTX * kTY, kRuntimeGeom>(a, wts, ix, iy, lane,
                                                              arena + M.ff_offset, fzo, nullptr,
                                                              dfo, s_col);
    else
        scan_column<STAGE, WIDE, kTX * kTY, 0, kRuntimeGeom, LERP32>(
            a, wts, ix, iy, lane, arena + M.ff_offset, fzo, nullptr, dfo, s_col);
}

// Standalone frequency shift, Eq. 3: one lane per (x, y) column and chunk of
// kDfChunk consecutive outputs (blockIdx.y), so that a lattice's columns give
// enough lanes to keep the loads in flight (one lane per column walking all of
// z left the pass latency-bound).  The lane loads its window of kDfChunk + 2m
// samples into registers (zero past the stack and up to kDfChunk + 2M); output o sums
// wts.w[j] * Fz(o + j) for j = 0 .. 2M in sample order, the weights beyond 2m
// being zero, so every output rounds as the end-of-column evaluation does.
constexpr int kDfChunk = 16;

template <int M>
__global__ __launch_bounds__(256) void df_kernel(const float *__restrict__ fz, int nz, int ny,
                                                  int nx, int m, const DfWeights wts,
                                                  float *__restrict__ df)
{
    const size_t plane = (size_t)nx * ny;
    const size_t col = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (col >= plane) return;
    const int n_out = nz - 2 * m;
    // chunks blockIdx.y, blockIdx.y + gridDim.y, ... (gridDim.y is capped)
    for (long long o0 = (long long)blockIdx.y * kDfChunk; o0 < n_out;
         o0 += (long long)gridDim.y * kDfChunk) {
        float win[kDfChunk + 2 * M];
#pragma unroll
        for (int j = 0; j < kDfChunk + 2 * M; ++j)
            win[j] = (j <= kDfChunk - 1 + 2 * m && o0 + j < nz)
                         ? fz[(size_t)(o0 + j) * plane + col] : 0.0f;
#pragma unroll
        for (int c = 0; c < kDfChunk; ++c) {
            float s = 0.0f;
#pragma unroll
            for (int j = 0; j <= 2 * M; ++j) s = fmaf(wts.w[j], win[c + j], s);
            if (o0 + c < n_out) df[(size_t)(o0 + c) * plane + col] = s;
        }
    }
}

// Weights in sample order for the end-of-column evaluation: o.w[j] multiplies
// sample o + j of output o, i.e. lag 2m - j in the ring layout.
DfWeights sample_weights(const DfWeights &w, int m)
{
    DfWeights o{};
    const int K = kMaxDfHalfWidth;
    for (int j = 0; j <= 2 * m; ++j) o.w[j] = w.w[2 * K - (2 * m - j)];
    return o;
}

}  // namespace

// Largest dynamic LDS allocation of one block on the current device (bytes),
// queried once per device; concurrent first calls store the same value.
size_t max_block_lds()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v == 0) {
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess || v <= 0)
            v = 65536;
        cache[dev].store(v, std::memory_order_relaxed);
    }
    return (size_t)v;
}

// Opt a kernel in to more than 64 KiB of dynamic LDS.  A refusal is cleared
// here; the launch that follows then reports the error.
template <typename Kernel>
void allow_lds(Kernel kernel, size_t bytes)
{
    if (bytes <= 65536) return;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        (void)hipGetLastError();
}

template <int TX, int TY, bool WIDE, int INTERP, int GEOM, bool LERP32, bool PF>
void launch_scan_tile(const ScanArgs &b, bool stage, const DfWeights &w, const float4 *ff,
                      const float *En, float *fz, float4 *pp, float *df, hipStream_t stream)
{
    dim3 block(TX, TY + (PF ? 64 / TX : 0), 1);
    dim3 grid((unsigned)(((b.snx + TX - 1) / TX) * ((b.sny + TY - 1) / TY)), 1, 1);
    const size_t prog = PF ? (size_t)TX * TY * sizeof(int) : 0;
    if (stage) {
        const size_t lds = (size_t)b.snz * TX * TY * sizeof(float) + prog;
        auto kernel = relaxed_scan_kernel<TX, TY, true, WIDE, INTERP, GEOM, LERP32, PF>;
        allow_lds(kernel, lds);
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, b, w, ff, En, fz, pp, df);
    } else {
        hipLaunchKernelGGL((relaxed_scan_kernel<TX, TY, false, WIDE, INTERP, GEOM, LERP32, PF>),
                           grid, block, prog, stream, b, w, ff, En, fz, pp, df);
    }
}

// The helper wave's plane windows assume an open grid (no wrap in x, y).
template <int TX, int TY, bool WIDE, int INTERP, int GEOM, bool LERP32>
void launch_scan_geom(const ScanArgs &b, bool stage, const DfWeights &w, const float4 *ff,
                      const float *En, float *fz, float4 *pp, float *df, hipStream_t stream)
{
    if constexpr (GEOM == kOpen || (INTERP != 0 && GEOM == kRuntimeGeom)) {
        if (!b.periodic) {
            launch_scan_tile<TX, TY, WIDE, INTERP, GEOM, LERP32, true>(b, stage, w, ff, En, fz,
                                                                        pp, df, stream);
            return;
        }
    }
    launch_scan_tile<TX, TY, WIDE, INTERP, GEOM, LERP32, false>(b, stage, w, ff, En, fz, pp, df,
                                                                 stream);
}

// Block shape: 16 x 16 lanes (four waves, one per SIMD of the CU that runs the
// block, plus the helper wave on open grids).  The kernel's time is the serial
// FIRE chain of its hardest columns, so those must not share a SIMD; one-wave
// blocks leave the pairing of waves on SIMDs to the dispatcher.  Fz is staged in
// LDS when the block's columns fit (up to 159 heights in gfx950's 160 KiB beside
// the progress array); beyond that the fz output is
// written directly (and re-read for the frequency shift), or, without fz,
// 8 x 8 blocks stage up to 256 heights.
//
// tile (the autotuner's choice, ppm_tuning.scan_tile): 0 = this automatic
// choice, 16 = 16 x 16 blocks wherever the outputs allow them, 8 = 8 x 8
// one-wave blocks (Fz staged in 8 KiB-per-32-heights LDS columns, several
// blocks per CU; with fz_direct and an fz output, Fz goes straight to fz and
// the frequency shift is a second pass over it, so the blocks take no LDS and
// every block of a large lattice can be resident at once).  Every route
// writes the same bits.
template <bool WIDE, int INTERP, int GEOM, bool LERP32>
void launch_scan_mode(const ScanArgs &b, const DfWeights &w, const float4 *ff, const float *En,
                      float *fz, float4 *pp, float *df, hipStream_t stream, int tile,
                      bool fz_direct)
{
    const bool want_df = b.m != 0 && df;
    const DfWeights sw = want_df ? sample_weights(w, b.m) : w;
    float *dfo = want_df ? df : nullptr;
    const size_t column = (size_t)b.snz * sizeof(float);
    const bool fits16 = (column + sizeof(int)) * 256 <= max_block_lds();
    const bool fits8 = b.snz <= kMaxScanLdsHeights;
    if (tile == 8 && fz_direct && fz) {
        // Fz straight to fz; the frequency shift then runs as its own pass over
        // fz (df_kernel, the same sums): fused, each lane would re-read its
        // column once per tap at the end of its FIRE chain (0.14 ms on the
        // large periodic scan against 0.07 ms for the pass)
        launch_scan_geom<kTX, kTY, WIDE, INTERP, GEOM, LERP32>(b, false, sw, ff, En, fz, pp,
                                                               nullptr, stream);
        if (want_df) launch_df(fz, b.snz, b.sny, b.snx, b.m, w, df, stream);
        return;
    }
    if (tile == 8) {
        launch_scan_geom<kTX, kTY, WIDE, INTERP, GEOM, LERP32>(b, (fz || want_df) && fits8, sw,
                                                               ff, En, fz, pp, dfo, stream);
        return;
    }
    if (!fz && !want_df)
        launch_scan_geom<16, 16, WIDE, INTERP, GEOM, LERP32>(b, false, sw, ff, En, fz, pp, dfo,
                                                             stream);
    else if (fits16)
        launch_scan_geom<16, 16, WIDE, INTERP, GEOM, LERP32>(b, true, sw, ff, En, fz, pp, dfo,
                                                             stream);
    else if (fz)
        launch_scan_geom<16, 16, WIDE, INTERP, GEOM, LERP32>(b, false, sw, ff, En, fz, pp, dfo,
                                                             stream);
    else
        launch_scan_geom<kTX, kTY, WIDE, INTERP, GEOM, LERP32>(b, true, sw, ff, En, fz, pp, dfo,
                                                               stream);
}

// The trilinear lookup is compiled per grid geometry (open grids have constant
// +x/+y corner offsets) and combination precision; the tricubic stencil reads
// the geometry at run time.
template <bool WIDE, int INTERP>
void launch_scan_variant(const ScanArgs &b, const DfWeights &w, const float4 *ff,
                         const float *En, float *fz, float4 *pp, float *df, hipStream_t stream,
                         int tile, bool fz_direct)
{
    if constexpr (INTERP != 0) {
        if (b.lerp32)
            launch_scan_mode<WIDE, INTERP, kRuntimeGeom, true>(b, w, ff, En, fz, pp, df, stream,
                                                               tile, fz_direct);
        else
            launch_scan_mode<WIDE, INTERP, kRuntimeGeom, false>(b, w, ff, En, fz, pp, df, stream,
                                                                tile, fz_direct);
    } else if (b.periodic) {
        if (b.lerp32)
            launch_scan_mode<WIDE, 0, kPeriodic, true>(b, w, ff, En, fz, pp, df, stream, tile,
                                                       fz_direct);
        else
            launch_scan_mode<WIDE, 0, kPeriodic, false>(b, w, ff, En, fz, pp, df, stream, tile,
                                                        fz_direct);
    } else {
        if (b.lerp32)
            launch_scan_mode<WIDE, 0, kOpen, true>(b, w, ff, En, fz, pp, df, stream, tile,
                                                   fz_direct);
        else
            launch_scan_mode<WIDE, 0, kOpen, false>(b, w, ff, En, fz, pp, df, stream, tile,
                                                    fz_direct);
    }
}

hipError_t launch_relaxed_scan(const ScanArgs &a, const DfWeights &w, const float4 *ff,
                               float *fz, float4 *pp, float *df, hipStream_t stream, int tile,
                               bool fz_direct)
{
    if (scan_grid_wide(a.gnx, a.gny, a.gnz, 16.0))
        launch_scan_variant<true, 0>(a, w, ff, nullptr, fz, pp, df, stream, tile, fz_direct);
    else
        launch_scan_variant<false, 0>(a, w, ff, nullptr, fz, pp, df, stream, tile, fz_direct);
    return hipGetLastError();
}

hipError_t launch_relaxed_scan_tricubic(const ScanArgs &a, const DfWeights &w,
                                        const float *En, float *fz, float4 *pp, float *df,
                                        hipStream_t stream)
{
    if (scan_grid_wide(a.gnx, a.gny, a.gnz, 4.0))
        launch_scan_variant<true, 1>(a, w, nullptr, En, fz, pp, df, stream, 0, false);
    else
        launch_scan_variant<false, 1>(a, w, nullptr, En, fz, pp, df, stream, 0, false);
    return hipGetLastError();
}

long long scan_tile_count(int nx, int ny)
{
    return (long long)((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY);
}

template <bool WIDE, bool LERP32>
void launch_scan_batch_mode(const ScanArgs &proto, const DfWeights &w, const ppm_batch_mol *mols,
                            const ppm_batch_scan *jobs, int n_jobs, dim3 grid, int max_nz,
                            const float4 *arena, float *fz, float *df, hipStream_t stream)
{
    dim3 block(kTX, kTY, 1);
    const bool want_df = proto.m != 0 && df;
    const DfWeights sw = want_df ? sample_weights(w, proto.m) : w;
    float *dfo = want_df ? df : nullptr;
    if ((fz || want_df) && max_nz <= kMaxScanLdsHeights) {
        const size_t lds = (size_t)max_nz * kTX * kTY * sizeof(float);
        hipLaunchKernelGGL((relaxed_scan_batch_kernel<true, WIDE, LERP32>), grid, block, lds,
                           stream, proto, sw, mols, jobs, n_jobs, arena, fz, dfo);
    } else {
        hipLaunchKernelGGL((relaxed_scan_batch_kernel<false, WIDE, LERP32>), grid, block, 0,
                           stream, proto, sw, mols, jobs, n_jobs, arena, fz, dfo);
    }
}

hipError_t launch_relaxed_scan_batch(const ScanArgs &proto, const DfWeights &w,
                                     const ppm_batch_mol *mols_dev,
                                     const ppm_batch_scan *jobs_dev, int n_jobs,
                                     long long n_tiles, int max_nz, bool wide,
                                     const float4 *arena, float *fz_arena, float *df_arena,
                                     hipStream_t stream)
{
    if (n_tiles <= 0) return hipSuccess;
    const long long gx = n_tiles < 65536 ? n_tiles : 65536;
    const long long gy = (n_tiles + gx - 1) / gx;
    dim3 grid((unsigned)gx, (unsigned)gy, 1);
    if (wide) {
        if (proto.lerp32)
            launch_scan_batch_mode<true, true>(proto, w, mols_dev, jobs_dev, n_jobs, grid, max_nz,
                                               arena, fz_arena, df_arena, stream);
        else
            launch_scan_batch_mode<true, false>(proto, w, mols_dev, jobs_dev, n_jobs, grid, max_nz,
                                                arena, fz_arena, df_arena, stream);
    } else {
        if (proto.lerp32)
            launch_scan_batch_mode<false, true>(proto, w, mols_dev, jobs_dev, n_jobs, grid, max_nz,
                                                arena, fz_arena, df_arena, stream);
        else
            launch_scan_batch_mode<false, false>(proto, w, mols_dev, jobs_dev, n_jobs, grid,
                                                 max_nz, arena, fz_arena, df_arena, stream);
    }
    return hipGetLastError();
}

hipError_t launch_df(const float *fz, int nz, int ny, int nx, int m, const DfWeights &w,
                     float *df, hipStream_t stream)
{
    const size_t plane = (size_t)nx * ny;
    const int n_out = nz - 2 * m;
    if (plane == 0 || n_out <= 0) return hipSuccess;
    dim3 block(256, 1, 1);
    const int chunks = (n_out + kDfChunk - 1) / kDfChunk;
    dim3 grid((unsigned)((plane + 255) / 256), (unsigned)(chunks < 65535 ? chunks : 65535), 1);
    const DfWeights sw = sample_weights(w, m);   // zero beyond 2m
    if (m <= 8)
        hipLaunchKernelGGL((df_kernel<8>), grid, block, 0, stream, fz, nz, ny, nx, m, sw, df);
    else if (m <= 16)
        hipLaunchKernelGGL((df_kernel<16>), grid, block, 0, stream, fz, nz, ny, nx, m, sw, df);
    else
        hipLaunchKernelGGL((df_kernel<32>), grid, block, 0, stream, fz, nz, ny, nx, m, sw, df);
    return hipGetLastError();
}

}  // namespace ppm
