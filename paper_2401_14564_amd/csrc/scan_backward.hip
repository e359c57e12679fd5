// scan_backward.hip -- implicit adjoint of the relaxed scan + frequency shift.
//
// At every relaxed point the net force vanishes, G(r*, theta) = 0 (Eq. 1), so the
// equilibrium moves with the atom parameters theta as dr*/dtheta = -J^{-1} dG/dtheta
// with J = dG/dr.  The tip force Fz_tip = -F^T_z(r*) (text after Eq. 2) depends on
// theta only through r*, and the frequency shift (Eq. 3) is linear in Fz_tip.
// Hence, for L with dL/d(df) = grad_df:
//   gbar_k = dL/dFz_k   (transposed frequency-shift weights)
//   mu     = J^{-T} (gbar_k grad_r F^T_z)
//   dL/dtheta_i = sum_k mu . sum_corners w_c d f_i(v_c)/d theta_i
// where f_i(v) = phi(rho) (v - r_i) is atom i's pair force (Eq. 5 + Eq. 6) at a
// cell corner, recomputed here; the gradient of the grid is never stored.
//
// Kernels:
//  1. adjoint_solve: one lane per relaxed point (tip column and height) forms
//     its grad_df tap sum, gathers the eight corners of the point's cell,
//     builds J (trilinear cell Jacobian + spring Jacobian, FP64), solves the
//     3x3 transposed system and writes mu, the cell and its fractions.
//  2. atom_scatter: one lane per atom, one block of four waves per chunk of
//     relaxed points (a tile of 8 x 8 columns x 2 heights).  The chunk's corner
//     weights mu w_c are merged per distinct voxel in LDS (neighbouring points
//     share corners), then the four waves split the voxels, every lane evaluating
//     its own atom's pair-force derivatives once per voxel and accumulating in
//     FP64 registers, so no cross-lane reduction is needed.  Each block writes
//     its per-atom partial sums, scaled by the per-atom constant factors.
//  3. reduce: sums the partials of every (atom, component) in a fixed order ->
//     deterministic result.
#include "ppm_device.h"
#include "ppm_kernels.h"

namespace ppm {
namespace {

constexpr int kTX = 16, kTY = 16;

struct EqRecord {
    float4 mu_v;      // mu (3), valid flag
    float4 t;         // tx, ty, tz, unused
    int4 idx;         // ix, iy, iz (cell corner), unused
};

template <int M>
__global__ __launch_bounds__(kTX * kTY) void adjoint_solve_kernel(
    const BwdArgs A, const DfWeights wts, const float4 *__restrict__ ff,
    const float4 *__restrict__ pp, const float *__restrict__ grad_df, EqRecord *__restrict__ rec)
{
    const ScanArgs &a = A.s;
    const int ix = blockIdx.x * kTX + threadIdx.x;
    const int iy = blockIdx.y * kTY + threadIdx.y;
    if (ix >= a.snx || iy >= a.sny) return;
    const size_t plane = (size_t)a.snx * a.sny;
    const size_t col = (size_t)iy * a.snx + ix;
    const double ax = a.x0 + ix * a.sdx, ay = a.y0 + iy * a.sdy;

    // one point (column, height s) per lane; heights blockIdx.z, + gridDim.z, ...
    // gbar_s = sum_j wts.w[j] grad_df(s - (2M - j)) in j order, the terms of
    // outputs outside 0 .. ndf-1 and of zero weight (j < 2M - 2m) being zero
    for (int s = (int)blockIdx.z; s < a.snz; s += (int)gridDim.z) {
        float gbar = 0.0f;
#pragma unroll
        for (int j = 0; j < 2 * M + 1; ++j) {
            const int so = s - (2 * M - j);
            const float g = (j >= 2 * M - 2 * a.m && so >= 0 && so < a.ndf)
                                ? grad_df[(size_t)so * plane + col] : 0.0f;
            gbar = fmaf(wts.w[j], g, gbar);
        }

        const size_t o = (size_t)s * plane + col;
        const float4 st = pp[o];
        EqRecord r;
        r.mu_v = make_float4(0.f, 0.f, 0.f, 0.f);
        r.t = make_float4(0.f, 0.f, 0.f, 0.f);
        r.idx = make_int4(0, 0, 0, 0);
        if (gbar != 0.0f && st.w >= 0.0f) {
            const double az = a.z_top - s * a.sdz;
            const double dx = a.d0x + st.x, dy = a.d0y + st.y, dz = a.d0z + st.z;  // r - anchor
            const double x = ax + dx, y = ay + dy, z = az + dz;
            // cell
            const double ux = (x - a.ox) * a.ihx, uy = (y - a.oy) * a.ihy, uz = (z - a.oz) * a.ihz;
            double tx, ty, tz;
            bool xin = true, yin = true, zin;
            int cx, cy;
            if (a.periodic) {
                const double fx = floor(ux), fy = floor(uy);
                tx = ux - fx;
                ty = uy - fy;
                cx = wrap_index(fx, a.gnx, a.ignx);
                cy = wrap_index(fy, a.gny, a.igny);
            } else {
                cx = clamp_cell(ux, a.gnx, tx, xin);
                cy = clamp_cell(uy, a.gny, ty, yin);
            }
            const int cz = clamp_cell(uz, a.gnz, tz, zin);
            const int cx1 = (cx + 1 < a.gnx) ? cx + 1 : 0, cy1 = (cy + 1 < a.gny) ? cy + 1 : 0;
            const size_t pl = (size_t)a.gnx * a.gny;
            const size_t b0 = (size_t)cz * pl, b1 = b0 + pl;
            const float4 v000 = ff[b0 + (size_t)cy * a.gnx + cx];
            const float4 v100 = ff[b0 + (size_t)cy * a.gnx + cx1];
            const float4 v010 = ff[b0 + (size_t)cy1 * a.gnx + cx];
            const float4 v110 = ff[b0 + (size_t)cy1 * a.gnx + cx1];
            const float4 v001 = ff[b1 + (size_t)cy * a.gnx + cx];
            const float4 v101 = ff[b1 + (size_t)cy * a.gnx + cx1];
            const float4 v011 = ff[b1 + (size_t)cy1 * a.gnx + cx];
            const float4 v111 = ff[b1 + (size_t)cy1 * a.gnx + cx1];
            const double sx = 1.0 - tx, sy = 1.0 - ty, sz = 1.0 - tz;
            // d/dx, d/dy, d/dz of the trilinear weights (per unit length)
            const double ihx = xin ? a.ihx : 0.0, ihy = yin ? a.ihy : 0.0;
            const double ihz = zin ? a.ihz : 0.0;
            double J[9];
#define PPM_JROW(C, r)                                                                          \
    {                                                                                           \
        const double e00 = (double)v100.C - v000.C, e10 = (double)v110.C - v010.C;             \
        const double e01 = (double)v101.C - v001.C, e11 = (double)v111.C - v011.C;             \
        J[3 * r + 0] = ihx * (sy * sz * e00 + ty * sz * e10 + sy * tz * e01 + ty * tz * e11);   \
        const double f00 = (double)v010.C - v000.C, f10 = (double)v110.C - v100.C;             \
        const double f01 = (double)v011.C - v001.C, f11 = (double)v111.C - v101.C;             \
        J[3 * r + 1] = ihy * (sx * sz * f00 + tx * sz * f10 + sx * tz * f01 + tx * tz * f11);   \
        const double g00 = (double)v001.C - v000.C, g10 = (double)v101.C - v100.C;             \
        const double g01 = (double)v011.C - v010.C, g11 = (double)v111.C - v110.C;             \
        J[3 * r + 2] = ihz * (sx * sy * g00 + tx * sy * g10 + sx * ty * g01 + tx * ty * g11);   \
    }
            PPM_JROW(x, 0)
            PPM_JROW(y, 1)
            PPM_JROW(z, 2)
#undef PPM_JROW
            // spring Jacobian dF^T/dr = -k_R[(1 - R0/|d|) I + R0 d d^T/|d|^3] - diag(kx, ky, 0)
            const double dn = sqrt(dx * dx + dy * dy + dz * dz);
            const double c1 = 1.0 - a.R0 / dn, c2 = a.R0 / (dn * dn * dn);
            const double d[3] = {dx, dy, dz};
            double Jt[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Jt[3 * i + j] = -a.kR * ((i == j ? c1 : 0.0) + c2 * d[i] * d[j]);
            Jt[0] -= a.kx;
            Jt[4] -= a.ky;
            for (int i = 0; i < 9; ++i) J[i] += Jt[i];
            // solve J^T mu = gbar * (row z of Jt)
            const double g = (double)gbar;
            const double b[3] = {g * Jt[6], g * Jt[7], g * Jt[8]};
            // transpose: T[i][j] = J[j][i]
            const double T00 = J[0], T01 = J[3], T02 = J[6];
            const double T10 = J[1], T11 = J[4], T12 = J[7];
            const double T20 = J[2], T21 = J[5], T22 = J[8];
            const double k00 = T11 * T22 - T12 * T21, k01 = T12 * T20 - T10 * T22,
                         k02 = T10 * T21 - T11 * T20;
            const double det = T00 * k00 + T01 * k01 + T02 * k02;
            if (fabs(det) > 1e-300) {
                const double id = 1.0 / det;
                const double mu0 = (k00 * b[0] + (T02 * T21 - T01 * T22) * b[1] +
                                    (T01 * T12 - T02 * T11) * b[2]) * id;
                const double mu1 = (k01 * b[0] + (T00 * T22 - T02 * T20) * b[1] +
                                    (T02 * T10 - T00 * T12) * b[2]) * id;
                const double mu2 = (k02 * b[0] + (T01 * T20 - T00 * T21) * b[1] +
                                    (T00 * T11 - T01 * T10) * b[2]) * id;
                r.mu_v = make_float4((float)mu0, (float)mu1, (float)mu2, 1.0f);
                r.t = make_float4((float)tx, (float)ty, (float)tz, 0.0f);
                r.idx = make_int4(cx, cy, cz, 0);
            }
        }
        rec[o] = r;
    }
}

// Points of one scatter chunk: a tile of 8 x 8 tip columns x 2 heights.
// Neighbouring relaxed points share cell corners (adjacent columns an x or y
// face, adjacent heights a z face), so the chunk's corner weights are first
// merged per distinct voxel.
constexpr int kChX = 8, kChY = 8, kChZ = 2, kChPts = kChX * kChY * kChZ;
// Largest local box (voxels) the merge accumulates in LDS; larger chunks (a
// probe that moved far from its neighbours, a chunk across a periodic seam)
// take the per-point path.
constexpr int kCellCap = 1024;

// d(force of this lane's atom at v)/d(atom parameters), contracted with m:
// d = v - r_atom (FP32), m = sum of trilinear weight x mu over the relaxed
// points that have v as a cell corner.  Accumulates -(phi I + phi'/rho d d^T) m
// into (ax, ay, az) and the parameter factors into aq, aR, ae, aqq (scaled
// per atom at the end).  QUAD: the probe carries the d_z2 quadrupole q_zz,
// whose pair force is f = -kQ grad u with u = (3 dz^2 - rho^2)/rho^5 and
// grad u = a d + b e_z, a = 3 rho^-5 - 15 dz^2 rho^-7, b = 6 dz rho^-5; its
// derivatives are df/d(atom) = kQ hess u and df/dq = -k_e q_zz grad u.
// PERIODIC: minimum image and the shifted-force cutoff of the force-field
// build: phi gains -fc/rho (fc = -dU/drho at rc of the LJ + Coulomb pair), u
// gains Y (3 rho rc^-4 - 4 rc^-3) with Y = 3 dz^2/rho^2 - 1, and pairs beyond
// rc drop out.
struct AtomConsts {
    float R2, e12, kq, kQ, rc2;
    float fcm, irc2, aRc, aec;      // shifted-force terms (periodic)
    float c3, c9, c18, c24;         // shifted d_z2 terms (periodic)
};

template <bool QUAD, bool PERIODIC>
__device__ __forceinline__ void pair_jvp(const AtomConsts &k, float dx, float dy, float dz,
                                         float mx, float my, float mz, float &ax_, float &ay_,
                                         float &az_, float &aq, float &aR, float &ae, float &aqq)
{
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    float ir = __builtin_amdgcn_rsqf(r2);
    if (PERIODIC) ir = (r2 < k.rc2) ? ir : 0.0f;
    const float ir2 = ir * ir;
    const float ir3 = ir * ir2;
    const float s2 = k.R2 * ir2;
    const float s6 = s2 * s2 * s2;
    const float s12 = s6 * s6;
    const float ec = k.kq * ir;
    float phi = fmaf(k.e12, s12 - s6, ec) * ir2;
    // phi'(rho)/rho = ir2^2 [12 e (-14 s12 + 8 s6) - 3 kq/rho]
    float dphi = fmaf(k.e12, fmaf(-14.0f, s12, 8.0f * s6), -3.0f * ec) * ir2 * ir2;
    if (PERIODIC) {
        phi = fmaf(-k.fcm, ir, phi);
        dphi = fmaf(k.fcm, ir3, dphi);
    }
    const float md = fmaf(mx, dx, fmaf(my, dy, mz * dz));
    const float tq = dphi * md;
    ax_ -= fmaf(phi, mx, tq * dx);
    ay_ -= fmaf(phi, my, tq * dy);
    az_ -= fmaf(phi, mz, tq * dz);
    const float im = ir2 * md;
    if (PERIODIC) {
        const float jm = ir * md;
        aq = fmaf(fmaf(-k.irc2, ir, ir3), md, aq);
        aR = fmaf(fmaf(2.0f, s12, -s6), im, fmaf(-k.aRc, jm, aR));
        ae = fmaf(s12 - s6, im, fmaf(-k.aec, jm, ae));
    } else {
        aq = fmaf(ir3, md, aq);                       // x k_e q_pp
        aR = fmaf(fmaf(2.0f, s12, -s6), im, aR);      // x 72 e_iP / R_iP
        ae = fmaf(s12 - s6, im, ae);                  // x 12 de_iP/de_i
    }
    if (QUAD) {
        const float ir5 = ir3 * ir2, ir7 = ir5 * ir2, ir9 = ir7 * ir2;
        const float z2 = dz * dz;
        float ua = fmaf(-15.0f * z2, ir7, 3.0f * ir5);
        float ub = 6.0f * dz * ir5;
        // grad a . m and grad b . m
        float ga = fmaf(fmaf(105.0f * z2, ir9, -15.0f * ir7), md, -30.0f * dz * ir7 * mz);
        float gb = fmaf(6.0f * ir5, mz, -30.0f * dz * ir7 * md);
        if (PERIODIC) {
            // shifted d_z2 term: grad u gains ax d + bx e_z with
            // ax = -9 rc^-4 dz^2 rho^-3 + 24 rc^-3 dz^2 rho^-4 - 3 rc^-4 rho^-1,
            // bx = 18 rc^-4 dz rho^-1 - 24 rc^-3 dz rho^-2
            const float ir4 = ir2 * ir2, ir6 = ir4 * ir2;
            ua += fmaf(z2, fmaf(k.c24, ir4, -k.c9 * ir3), -k.c3 * ir);
            ub += dz * fmaf(k.c18, ir, -k.c24 * ir2);
            ga += fmaf(-k.c9, fmaf(2.0f * dz * ir3, mz, -3.0f * z2 * ir5 * md),
                       fmaf(k.c24, fmaf(2.0f * dz * ir4, mz, -4.0f * z2 * ir6 * md),
                            k.c3 * ir3 * md));
            gb += fmaf(k.c18, fmaf(ir, mz, -dz * ir3 * md),
                       -k.c24 * fmaf(ir2, mz, -2.0f * dz * ir4 * md));
        }
        ax_ = fmaf(k.kQ, fmaf(ua, mx, dx * ga), ax_);
        ay_ = fmaf(k.kQ, fmaf(ua, my, dy * ga), ay_);
        az_ = fmaf(k.kQ, fmaf(ua, mz, fmaf(dz, ga, gb)), az_);
        aqq = fmaf(ua, md, fmaf(ub, mz, aqq));    // x -k_e q_zz
    }
}

// Displacement component v - r_atom along a periodic or open axis, FP64, then FP32.
template <bool PERIODIC>
__device__ __forceinline__ float axis_disp(double v, double p, double L)
{
    double d = v - p;
    if (PERIODIC) d -= L * rint(d / L);
    return (float)d;
}

// One block of four waves per (chunk, block of 64 atoms); lane = atom, the
// same 64 atoms in every wave.  Wave 0 stages the chunk's records and merges
// their corner weights per voxel in LDS (in a fixed order, so the result is
// deterministic); the four waves then split the distinct voxels, every lane
// evaluating its atom's pair-force derivatives once per voxel (FP32 per batch of
// eight voxels, then FP64), and wave 0 adds the four waves' sums in order.
constexpr int kScatterWaves = 4;

template <bool QUAD, bool PERIODIC>
__global__ __launch_bounds__(64 * kScatterWaves) void atom_scatter_kernel(
    const BwdArgs A, const EqRecord *__restrict__ rec, const double *__restrict__ pos,
    const double *__restrict__ q, const double *__restrict__ R, const double *__restrict__ eps,
    double *__restrict__ partial)
{
    __shared__ float s_m[3][kCellCap];
    __shared__ float4 s_u[kCellCap];          // merged voxels: (m, packed local x, y, z)
    // The chunk's records and the merge tags share s_u's storage: wave 0 writes
    // s_u only after its merge has read them for the last time (a wave's LDS
    // operations complete in order), and the per-point path, which reads the
    // records after the barrier, writes no s_u.  (28.7 KB per block: five
    // blocks per CU instead of four.)
    EqRecord *const s_rec = reinterpret_cast<EqRecord *>(s_u);                // [kChPts]
    int *const s_tag = reinterpret_cast<int *>(s_rec + kChPts);               // [kCellCap]
    static_assert(kChPts * sizeof(EqRecord) + kCellCap * sizeof(int) <= sizeof(s_u),
                  "records and tags fit in s_u");
    __shared__ int s_box[8];                  // lo[3], bx, by, bz, n, flags
    const ScanArgs &a = A.s;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int atom = blockIdx.y * 64 + lane;
    const bool live = atom < A.n_atoms;
    const int ia = live ? atom : 0;
    const double px = pos[3 * ia], py = pos[3 * ia + 1], pz = pos[3 * ia + 2];
    const double RiP = R[ia] + A.R_pp;
    const double eiP = sqrt(eps[ia] * A.eps_pp);
    AtomConsts k;
    k.R2 = (float)(RiP * RiP);
    k.e12 = (float)(12.0 * eiP);
    k.kq = (float)(A.kq_pp * q[ia]);
    k.kQ = (float)(A.kQ_pp * q[ia]);
    k.rc2 = A.rc2;
    k.fcm = k.irc2 = k.aRc = k.aec = k.c3 = k.c9 = k.c18 = k.c24 = 0.f;
    if (PERIODIC) {
        const double irc = 1.0 / A.rc;
        const double sc2 = RiP * RiP * irc * irc, sc6 = sc2 * sc2 * sc2, sc12 = sc6 * sc6;
        k.fcm = (float)(12.0 * eiP * (sc12 - sc6) * irc + A.kq_pp * q[ia] * irc * irc);
        k.irc2 = (float)(irc * irc);
        k.aRc = (float)((2.0 * sc12 - sc6) * irc);
        k.aec = (float)((sc12 - sc6) * irc);
        const double irc3 = irc * irc * irc, irc4 = irc3 * irc;
        k.c3 = (float)(3.0 * irc4);
        k.c9 = (float)(9.0 * irc4);
        k.c18 = (float)(18.0 * irc4);
        k.c24 = (float)(24.0 * irc3);
    }

    // the chunk: tip columns (cx0 .. cx0+7, cy0 .. cy0+7), heights s0, s0+1
    const int ntx = (a.snx + kChX - 1) / kChX, nty = (a.sny + kChY - 1) / kChY;
    const int chunk = blockIdx.x;
    const int tzi = chunk / (ntx * nty), rest = chunk - tzi * ntx * nty;
    const int cx0 = (rest % ntx) * kChX, cy0 = (rest / ntx) * kChY, s0 = tzi * kChZ;
    const size_t plane = (size_t)a.snx * a.sny;

    if (wv == 0) {
        // stage the chunk's records (invalid or outside the lattice: mu_v.w = 0)
        // and reduce the local box of its valid cells (base corners)
        int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX};
        int hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
#pragma unroll
        for (int r = 0; r < kChPts / 64; ++r) {
            const int pnt = r * 64 + lane;
            const int ix = cx0 + (pnt % kChX), iy = cy0 + ((pnt / kChX) % kChY);
            const int sh = s0 + pnt / (kChX * kChY);
            EqRecord e;
            if (ix < a.snx && iy < a.sny && sh < a.snz) {
                e = rec[(size_t)sh * plane + (size_t)iy * a.snx + ix];
            } else {
                e.mu_v = make_float4(0.f, 0.f, 0.f, 0.f);
                e.t = e.mu_v;
                e.idx = make_int4(0, 0, 0, 0);
            }
            s_rec[pnt] = e;
            if (e.mu_v.w != 0.0f) {
                lo[0] = min(lo[0], e.idx.x); lo[1] = min(lo[1], e.idx.y);
                lo[2] = min(lo[2], e.idx.z);
                hi[0] = max(hi[0], e.idx.x); hi[1] = max(hi[1], e.idx.y);
                hi[2] = max(hi[2], e.idx.z);
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                lo[d] = min(lo[d], __shfl_xor(lo[d], off));
                hi[d] = max(hi[d], __shfl_xor(hi[d], off));
            }
        const bool any = lo[0] <= hi[0];
        const int bx = hi[0] - lo[0] + 2, by = hi[1] - lo[1] + 2, bz = hi[2] - lo[2] + 2;
        const bool merge = any && (long long)bx * by * bz <= kCellCap;
        int n = 0;
        if (merge) {
            const int nc = bx * by * bz;
            for (int c = lane; c < nc; c += 64) s_m[0][c] = s_m[1][c] = s_m[2][c] = 0.0f;
            // merge, in 16 groups of eight points taken in a fixed order: lane
            // 8 p + c holds corner c of the group's point p.  A group's points lie
            // at least two columns apart, so their cells rarely share a voxel; the
            // lanes tag the voxels they hit (a wave's LDS operations complete in
            // order) and, when no two lanes of the group hit the same voxel, the
            // group adds its 64 weights in one step, else point by point.  Each
            // voxel therefore sums its weights in a fixed order (deterministic).
            static_assert(kChX == 8 && kChY == 8 && kChZ == 2, "merge groups of an 8x8x2 chunk");
            const int ci = lane & 1, cj = (lane >> 1) & 1, ck = (lane >> 2) & 1;
            const int gp = lane >> 3;
            for (int g = 0; g < 16; ++g) {
                // group g: height g >> 3, columns (xo + 2 i, yo + 4 j) for i < 4,
                // j < 2, with xo = (g >> 2) & 1 and yo = g & 3
                const int px = ((g >> 2) & 1) + 2 * (gp & 3);
                const int py = (g & 3) + 4 * (gp >> 2);
                const EqRecord r = s_rec[(g >> 3) * (kChX * kChY) + py * kChX + px];
                const bool valid = r.mu_v.w != 0.0f;
                const float w = (ci ? r.t.x : 1.0f - r.t.x) * (cj ? r.t.y : 1.0f - r.t.y) *
                                (ck ? r.t.z : 1.0f - r.t.z);
                const int c = valid ? ((r.idx.z + ck - lo[2]) * by + (r.idx.y + cj - lo[1])) * bx +
                                          (r.idx.x + ci - lo[0])
                                    : 0;
                if (valid)
                    __hip_atomic_store(s_tag + c, lane, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_WORKGROUP);
                const bool clash =
                    valid && __hip_atomic_load(s_tag + c, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP) != lane;
                if (__ballot(clash) == 0ull) {
                    if (valid) {
                        s_m[0][c] += w * r.mu_v.x;
                        s_m[1][c] += w * r.mu_v.y;
                        s_m[2][c] += w * r.mu_v.z;
                    }
                } else {
                    for (int q = 0; q < 8; ++q) {
                        if (gp == q && valid) {
                            s_m[0][c] += w * r.mu_v.x;
                            s_m[1][c] += w * r.mu_v.y;
                            s_m[2][c] += w * r.mu_v.z;
                        }
                    }
                }
            }
            // the voxels that received weight, in cell order: (m, packed local x, y, z)
            int lx = lane % bx, ly = (lane / bx) % by, lz = lane / (bx * by);
            const int sx = 64 % bx, sy = (64 / bx) % by, sz = 64 / (bx * by);
            for (int c0 = 0; c0 < nc; c0 += 64) {
                const int c = c0 + lane;
                float4 m = make_float4(0.f, 0.f, 0.f, 0.f);
                if (c < nc) m = make_float4(s_m[0][c], s_m[1][c], s_m[2][c], 0.f);
                const bool hit = m.x != 0.0f || m.y != 0.0f || m.z != 0.0f;
                const unsigned long long bal = __ballot(hit);
                if (hit) {
                    m.w = __uint_as_float((uint32_t)lx | ((uint32_t)ly << 10) |
                                          ((uint32_t)lz << 20));
                    s_u[n + __popcll(bal & ((1ull << lane) - 1ull))] = m;
                }
                n += __popcll(bal);
                lx += sx;
                const int cxr = lx >= bx;
                lx -= cxr ? bx : 0;
                ly += sy + cxr;
                const int cyr = ly >= by;
                ly -= cyr ? by : 0;
                lz += sz + cyr;
            }
        }
        if (lane == 0) {
            s_box[0] = lo[0]; s_box[1] = lo[1]; s_box[2] = lo[2];
            s_box[3] = bx; s_box[4] = by; s_box[5] = bz;
            s_box[6] = n;
            s_box[7] = (any ? 1 : 0) | (merge ? 2 : 0);
        }
    }
    __syncthreads();
    const int flags = s_box[7];
    double gx = 0.0, gy = 0.0, gz = 0.0, gq = 0.0, gR = 0.0, ge = 0.0, gqq = 0.0;
    if (flags & 2) {
        const int n = s_box[6];
        // the box corner relative to the atom, FP64 then FP32 (minimum image on a
        // periodic grid); a voxel's offset is then one FP32 multiply-add per axis
        // (plus the wrap, the box being at most 1023 voxels wide)
        const float bdx = axis_disp<PERIODIC>(a.ox + s_box[0] * A.hx, px, A.Lx);
        const float bdy = axis_disp<PERIODIC>(a.oy + s_box[1] * A.hy, py, A.Ly);
        const float bdz = (float)(a.oz + s_box[2] * A.hz - pz);
        const float hxf = (float)A.hx, hyf = (float)A.hy, hzf = (float)A.hz;
        const float Lxf = (float)A.Lx, Lyf = (float)A.Ly;
        const float iLxf = PERIODIC ? (float)(1.0 / A.Lx) : 0.f;
        const float iLyf = PERIODIC ? (float)(1.0 / A.Ly) : 0.f;
        // wave wv takes the voxels [n wv / 4, n (wv+1) / 4)
        const int ub = (n * wv) / kScatterWaves, ue = (n * (wv + 1)) / kScatterWaves;
        for (int u0 = ub; u0 < ue; u0 += 8) {
            float ax_ = 0.f, ay_ = 0.f, az_ = 0.f, aq = 0.f, aR = 0.f, ae = 0.f, aqq = 0.f;
            const int u1 = min(ue, u0 + 8);
            for (int u = u0; u < u1; ++u) {
                const float4 e = s_u[u];
                const uint32_t pk = __float_as_uint(e.w);
                float dx = fmaf((float)(pk & 1023u), hxf, bdx);
                float dy = fmaf((float)((pk >> 10) & 1023u), hyf, bdy);
                const float dz = fmaf((float)(pk >> 20), hzf, bdz);
                if (PERIODIC) {
                    dx = fmaf(-Lxf, rintf(dx * iLxf), dx);
                    dy = fmaf(-Lyf, rintf(dy * iLyf), dy);
                }
                pair_jvp<QUAD, PERIODIC>(k, dx, dy, dz, e.x, e.y, e.z, ax_, ay_, az_, aq, aR,
                                         ae, aqq);
            }
            gx += ax_;
            gy += ay_;
            gz += az_;
            gq += aq;
            gR += aR;
            ge += ae;
            gqq += aqq;
        }
    } else if (flags & 1) {
        // per point (wave wv: points wv, wv + 4, ...): the eight corners of its cell
        for (int pnt = wv; pnt < kChPts; pnt += kScatterWaves) {
            const EqRecord r = s_rec[pnt];
            if (r.mu_v.w == 0.0f) continue;
            const int cx1 = (r.idx.x + 1 < a.gnx) ? r.idx.x + 1 : 0;
            const int cy1 = (r.idx.y + 1 < a.gny) ? r.idx.y + 1 : 0;
            const float dxs[2] = {axis_disp<PERIODIC>(a.ox + r.idx.x * A.hx, px, A.Lx),
                                  axis_disp<PERIODIC>(a.ox + cx1 * A.hx, px, A.Lx)};
            const float dys[2] = {axis_disp<PERIODIC>(a.oy + r.idx.y * A.hy, py, A.Ly),
                                  axis_disp<PERIODIC>(a.oy + cy1 * A.hy, py, A.Ly)};
            const float dzs[2] = {(float)(a.oz + r.idx.z * A.hz - pz),
                                  (float)(a.oz + (r.idx.z + 1) * A.hz - pz)};
            const float tx = r.t.x, ty = r.t.y, tz = r.t.z;
            const float wx[2] = {1.0f - tx, tx}, wy[2] = {1.0f - ty, ty}, wz[2] = {1.0f - tz, tz};
            float ax_ = 0.f, ay_ = 0.f, az_ = 0.f, aq = 0.f, aR = 0.f, ae = 0.f, aqq = 0.f;
#pragma unroll
            for (int cc = 0; cc < 8; ++cc) {
                const int i = cc & 1, j = (cc >> 1) & 1, kk = cc >> 2;
                const float w = wx[i] * wy[j] * wz[kk];
                pair_jvp<QUAD, PERIODIC>(k, dxs[i], dys[j], dzs[kk], w * r.mu_v.x,
                                         w * r.mu_v.y, w * r.mu_v.z, ax_, ay_, az_, aq, aR, ae,
                                         aqq);
            }
            gx += ax_;
            gy += ay_;
            gz += az_;
            gq += aq;
            gR += aR;
            ge += ae;
            gqq += aqq;
        }
    }
    // the four waves' sums, added by wave 0 in wave order (s_u is free again)
    __syncthreads();
    double *s_red = reinterpret_cast<double *>(s_u);          // [wave][7][64]
    if (wv > 0) {
        double *o = s_red + (size_t)(wv - 1) * 7 * 64 + lane;
        o[0] = gx; o[64] = gy; o[128] = gz; o[192] = gq; o[256] = gR; o[320] = ge;
        o[384] = gqq;
    }
    __syncthreads();
    if (wv == 0) {
        for (int w = 0; w < kScatterWaves - 1; ++w) {
            const double *o = s_red + (size_t)w * 7 * 64 + lane;
            gx += o[0]; gy += o[64]; gz += o[128]; gq += o[192]; gR += o[256]; ge += o[320];
            gqq += o[384];
        }
        if (live) {
            // partial[atom][component][chunk]: the sum over chunks reads rows
            const size_t nb = gridDim.x;
            double *out = partial + (size_t)atom * 6 * nb + blockIdx.x;
            out[0] = gx;
            out[nb] = gy;
            out[2 * nb] = gz;
            out[3 * nb] = gq * A.ke_qpp - (QUAD ? gqq * A.kQ_pp : 0.0);
            out[4 * nb] = gR * 72.0 * eiP / RiP;
            out[5 * nb] = (eiP > 0.0) ? ge * 12.0 * (A.eps_pp / (2.0 * eiP)) : 0.0;
        }
    }
}

// One block per (atom, component): fixed-order sum over the chunk partials, a
// contiguous row partial[atom][component][0 .. n_blocks) read by this block only.
__global__ __launch_bounds__(256) void reduce_kernel(const double *__restrict__ partial,
                                                     int n_blocks, int n_atoms,
                                                     double *__restrict__ g_pos,
                                                     double *__restrict__ g_q,
                                                     double *__restrict__ g_R,
                                                     double *__restrict__ g_eps)
{
    __shared__ double s[256];
    const int atom = blockIdx.x / 6, comp = blockIdx.x % 6;
    const double *rowp = partial + (size_t)blockIdx.x * n_blocks;
    double acc = 0.0;
    for (int b = threadIdx.x; b < n_blocks; b += 256) acc += rowp[b];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && atom < n_atoms) {
        const double v = s[0];
        if (comp < 3) g_pos[3 * atom + comp] = v;
        else if (comp == 3) g_q[atom] = v;
        else if (comp == 4) g_R[atom] = v;
        else g_eps[atom] = v;
    }
}

DfWeights repad_lag(const DfWeights &w, int m, int M)
{
    // input: forward layout of capacity K (W[2K - lag] = weight of lag);
    // output: V[j] = weight of lag 2m - (2M - j) for the grad_df taps.
    DfWeights o{};
    const int K = kMaxDfHalfWidth;
    for (int j = 2 * M - 2 * m; j <= 2 * M; ++j) {
        const int lag = 2 * m - (2 * M - j);
        o.w[j] = w.w[2 * K - lag];
    }
    return o;
}

}  // namespace

hipError_t launch_backward(const BwdArgs &A, const DfWeights &w, const float4 *ff,
                           const float4 *pp, const float *grad_df, const double *pos,
                           const double *q, const double *R, const double *eps, float4 *eq_ws,
                           double *partial_ws, double *g_pos, double *g_q, double *g_R,
                           double *g_eps, hipStream_t stream)
{
    EqRecord *rec = reinterpret_cast<EqRecord *>(eq_ws);
    dim3 blk(kTX, kTY, 1);
    dim3 grd((A.s.snx + kTX - 1) / kTX, (A.s.sny + kTY - 1) / kTY,
             (unsigned)(A.s.snz < 65535 ? A.s.snz : 65535));
    const int m = A.s.m;
    if (m <= 8)
        hipLaunchKernelGGL((adjoint_solve_kernel<8>), grd, blk, 0, stream, A, repad_lag(w, m, 8),
                           ff, pp, grad_df, rec);
    else if (m <= 16)
        hipLaunchKernelGGL((adjoint_solve_kernel<16>), grd, blk, 0, stream, A,
                           repad_lag(w, m, 16), ff, pp, grad_df, rec);
    else
        hipLaunchKernelGGL((adjoint_solve_kernel<32>), grd, blk, 0, stream, A,
                           repad_lag(w, m, 32), ff, pp, grad_df, rec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (A.n_atoms == 0) return hipSuccess;
    const int na_blocks = (A.n_atoms + 63) / 64;
    dim3 g2(A.n_eq_blocks, na_blocks, 1);
    const dim3 sblk(64 * kScatterWaves, 1, 1);
    if (A.kQ_pp != 0.0) {
        if (A.periodic)
            hipLaunchKernelGGL((atom_scatter_kernel<true, true>), g2, sblk, 0, stream, A, rec, pos,
                               q, R, eps, partial_ws);
        else
            hipLaunchKernelGGL((atom_scatter_kernel<true, false>), g2, sblk, 0, stream, A, rec,
                               pos, q, R, eps, partial_ws);
    } else {
        if (A.periodic)
            hipLaunchKernelGGL((atom_scatter_kernel<false, true>), g2, sblk, 0, stream, A, rec,
                               pos, q, R, eps, partial_ws);
        else
            hipLaunchKernelGGL((atom_scatter_kernel<false, false>), g2, sblk, 0, stream, A, rec,
                               pos, q, R, eps, partial_ws);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_kernel, dim3(A.n_atoms * 6, 1, 1), dim3(256, 1, 1), 0, stream,
                       partial_ws, A.n_eq_blocks, A.n_atoms, g_pos, g_q, g_R, g_eps);
    return hipGetLastError();
}

}  // namespace ppm
