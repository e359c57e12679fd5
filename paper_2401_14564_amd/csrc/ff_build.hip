// ff_build.hip -- force-field grid projection on gfx950.
//
// Every voxel sums the Lennard-Jones (Eq. 5) and point-charge Coulomb (Eq. 6)
// energy of the probe particle and the force F = -grad E over the sample's
// atoms (Sec. 2.2, Sec. 5.1.1 step 1).  A probe with a quadrupolar d_z2 charge
// q_zz (Sec. 2.2.3) adds, per atom, q_zz d^2 V_i/dz^2 with V_i the atom's
// Coulomb potential: kQ_i (3 dz^2 - rho^2) / rho^5, kQ_i = k_e q_i q_zz.  The
// work is O(n_atoms * n_voxels) and bound by the FP32 vector ALU; it is not a
// dense contraction, so no MFMA.
//
// Design:
//  * A block of BX x BY threads owns a brick of BX x BY x NZB voxels; each
//    thread owns NZB voxels of one z-column, so dx, dy and dx^2+dy^2 are shared
//    by NZB pairs (register blocking along z).  A wave covers 8 x 8 columns
//    (eight 128-byte runs of float4 stores), the most compact box for the
//    periodic per-wave atom lists below.
//  * Atoms are staged through LDS in chunks of BX*BY.  While staging, each atom's
//    mixing rules are applied once (R_iP = R_i + R_PP, e_iP = sqrt(e_i e_PP),
//    kq_i = k_e q_i q_PP) and folded, in FP64, into A_i = e_iP R_iP^12 and
//    B_i = 2 e_iP R_iP^6, so that a pair needs rho^-6 alone (its LJ energy is
//    rho^-6 (A_i rho^-6 - B_i)), and its position is made brick-local in FP64 before
//    rounding to FP32: FP32 differences of small local coordinates keep the
//    relative error of rho near 1e-7, which absolute FP32 coordinates (ulp of
//    24 A = 1.9e-6 A) would not.  The inner loop reads one atom per step with
//    wave-uniform LDS addresses (broadcast).
//  * Periodic samples: each atom takes, per brick, the image nearest to the
//    brick centre (exact minimum image for every voxel of the brick as long as
//    cutoff + brick half-diagonal < L/2, which the host checks), atoms beyond
//    cutoff + half-diagonal of the centre are dropped with a deterministic
//    ballot compaction (positions first; the FP64 per-atom constants are then
//    computed for the kept atoms only, one thread per kept slot), and each wave
//    sorts the kept atoms against its own 8 x 8 x NZB box into interior atoms
//    (no mask), shell atoms (each pair masked by rho^2 < cutoff^2) and close
//    interior atoms (summed last, into an energy accumulator of their own).  The
//    cutoff is a shifted-force truncation: along every ray from an atom each
//    pair term Y(direction) g(rho) becomes g - g(rc) - (rho - rc) g'(rc), so
//    energy and force vanish on the cutoff sphere (a plain truncation leaves a
//    force step k_e q_i q_PP / rc^2 on every charged atom's sphere, which makes
//    the grid rough at the voxel scale and stalls the relaxation).  For the
//    LJ + Coulomb pair this is E += fc rho - C, F -= fc d / rho with per-atom
//    constants fc = -dU/drho(rc), C = U(rc) + rc fc; the radial part of the
//    d_z2 term folds into the same two constants, its angular part adds
//    kQ dz^2 (9 rho^-1 rc^-4 - 12 rho^-2 rc^-3) to E.
#include <type_traits>

#include "ppm.h"
#include "ppm_kernels.h"

namespace ppm {
namespace {

// Interior atoms within this distance (A) of a wave's box are summed last.
constexpr float kCloseA = 3.0f;

template <int BX, int BY, int NZB>
__device__ __host__ __forceinline__ double ff_brick_half_diagonal_dev(double hx, double hy,
                                                                      double hz)
{
    const double ex = 0.5 * (BX - 1) * hx, ey = 0.5 * (BY - 1) * hy, ez = 0.5 * (NZB - 1) * hz;
    return sqrt(ex * ex + ey * ey + ez * ez);
}

// LDS of one brick: staged atoms and per-wave counts of the compaction.
template <int NT>
struct BrickLds {
    float4 geo[NT];   // brick-local (x, y, z) and A_i = e_iP R_iP^12
    float4 par[NT];   // 12 A_i, -6 B_i, kq_i, -B_i  (B_i = 2 e_iP R_iP^6)
    float4 aux[NT];   // shifted-force constants fc, C (periodic), kQ_i (quadrupole)
    int wcnt[NT / 64];
    int idx[NT];      // periodic: atom index of each staged slot
    // periodic: per wave, the staged atoms whose cutoff sphere holds the whole
    // wave box (interior: [0] beyond kCloseA of the box, [2] within it) and
    // those it only cuts (shell, [1]), in staging order, as byte offsets into
    // geo (the same offsets address par and aux)
    uint16_t list[NT / 64][3][NT];
};

// An atom's auxiliary constants: all four with a quadrupolar probe, else
// only the shifted-force pair (fc, C).
template <bool QUAD>
__device__ __forceinline__ float4 lds_aux(const float4 *s_aux, int t)
{
    if (QUAD) return s_aux[t];
    const float2 v = *reinterpret_cast<const float2 *>(&s_aux[t]);
    return make_float4(v.x, v.y, 0.f, 0.f);
}

// One atom's terms at the NZB voxels of a thread's z-column.  MASKED: the pair
// enters only inside the cutoff sphere (rho^2 < rc^2 in FP32), and the
// shifted-force constant -C with it; unmasked periodic pairs (every voxel of
// the wave inside the sphere) leave -C to the caller, which adds it once per
// atom for the whole wave.
template <int NZB, bool PERIODIC, bool MASKED, bool EONLY, bool QUAD>
__device__ __forceinline__ void ff_pair(const float4 g, const float4 p, const float4 aux, float vx,
                                        float vy, const float (&vz)[NZB], float rc2, float c9,
                                        float c12, float c18, float c24, float (&Fx)[NZB],
                                        float (&Fy)[NZB], float (&Fz)[NZB], float (&E)[NZB])
{
    const float dx = vx - g.x, dy = vy - g.y;
    const float dxy2 = fmaf(dx, dx, dy * dy);
#pragma unroll
    for (int k = 0; k < NZB; ++k) {
        const float dz = vz[k] - g.z;
        const float r2 = fmaf(dz, dz, dxy2);
        float ir = __builtin_amdgcn_rsqf(r2);
        const bool in = !MASKED || r2 < rc2;
        if (MASKED) ir = in ? ir : 0.0f;
        const float ir2 = ir * ir;
        const float ir4 = ir2 * ir2;
        const float ir6 = ir4 * ir2;
        const float ec = p.z * ir;
        // E: e (s12 - 2 s6) = rho^-6 (A rho^-6 - B), plus kq/rho; on periodic
        // samples the shifted-force terms + fc rho (- C inside the sphere),
        // folded as (fc rho^2 + kq)/rho
        float e = fmaf(fmaf(g.w, ir6, p.w), ir6, E[k]);
        if (PERIODIC) {
            if (MASKED)     // one rounding for the pair's Coulomb + shift terms
                e += fmaf(fmaf(aux.x, r2, p.z), ir, in ? -aux.y : 0.0f);   // ir = 0 outside
            else            // (-C is summed per wave for interior atoms)
                e = fmaf(fmaf(aux.x, r2, p.z), ir, e);
        } else {
            e += ec;
        }
        E[k] = e;
        float f = 0.0f;
        // F/rho: 12 e (s12 - s6)/rho^2 = rho^-8 (12 A rho^-6 - 6 B), plus kq/rho^3
        if (!EONLY) f = fmaf(fmaf(p.x, ir6, p.y), ir6, ec) * ir2;
        if (PERIODIC && !EONLY) f = fmaf(-aux.x, ir, f);
        if (QUAD) {
            // u = (3 dz^2 - rho^2)/rho^5,
            // -grad u = rho^-5 [(15 dz^2/rho^2 - 3) d - 6 dz e_z]
            const float z2 = dz * dz;
            const float q5 = aux.z * (ir4 * ir);               // kQ_i / rho^5
            E[k] = fmaf(q5, fmaf(3.0f, z2, -r2), E[k]);
            if (!EONLY) {
                f = fmaf(q5, fmaf(15.0f * z2, ir2, -3.0f), f);
                Fz[k] = fmaf(-6.0f * q5, dz, Fz[k]);
            }
            if (PERIODIC) {
                // angular part of the shift: kQ dz^2 (9 rc^-4/rho - 12 rc^-3/rho^2),
                // its -grad: -kQ [dz^2 rho^-3 (24 rc^-3/rho - 9 rc^-4) d
                //                 + dz rho^-1 (18 rc^-4 - 24 rc^-3/rho) e_z]
                const float qz2 = aux.z * z2;
                E[k] = fmaf(qz2, fmaf(c9, ir, -c12 * ir2), E[k]);
                if (!EONLY) {
                    f = fmaf(-qz2 * ir2 * ir, fmaf(c24, ir, -c9), f);
                    Fz[k] = fmaf(-aux.z * dz * ir, fmaf(-c24, ir, c18), Fz[k]);
                }
            }
        }
        if (!EONLY) {
            Fx[k] = fmaf(f, dx, Fx[k]);
            Fy[k] = fmaf(f, dy, Fy[k]);
            Fz[k] = fmaf(f, dz, Fz[k]);
        }
    }
}

// One brick of BX x BY x NZB voxels with corner voxel (ix0, iy0, iz0).
// EONLY: only the energy is accumulated and stored (one float per voxel, the
// input of the tricubic scan); `ff` then points at floats.  QUAD: the probe
// carries a quadrupole moment (kQ_pp != 0).
template <int BX, int BY, int NZB, bool PERIODIC, bool EONLY, bool QUAD>
__device__ __forceinline__ void ff_brick(const FFArgs &a, int ix0, int iy0, int iz0,
                                         const double *__restrict__ pos,
                                         const double *__restrict__ q,
                                         const double *__restrict__ R,
                                         const double *__restrict__ eps,
                                         float4 *__restrict__ ff, BrickLds<BX * BY> &lds)
{
    constexpr int NT = BX * BY;
    constexpr int NW = NT / 64;
    float4 *s_geo = lds.geo;
    float4 *s_par = lds.par;
    float4 *s_aux = lds.aux;
    int *s_wcnt = lds.wcnt;
    static_assert(BX % 8 == 0 && BY % 8 == 0 && NT <= 256,
                  "8 x 8-column waves; list offsets 16 * (NT - 1) fit in 16 bits");
    // angular part of the shifted d_z2 term: 9 rc^-4, 12 rc^-3, 18 rc^-4, 24 rc^-3
    float c9 = 0.f, c12 = 0.f, c18 = 0.f, c24 = 0.f;
    if (PERIODIC && QUAD) {
        const double irc3 = 1.0 / (a.rc * a.rc * a.rc), irc4 = irc3 / a.rc;
        c9 = (float)(9.0 * irc4);
        c12 = (float)(12.0 * irc3);
        c18 = (float)(18.0 * irc4);
        c24 = (float)(24.0 * irc3);
    }

    // each wave owns an 8 x 8 patch of the brick's columns (a compact box for
    // the periodic cull); tid stages atoms, (tx, ty) is the thread's column
    const int tid = (int)threadIdx.y * BX + (int)threadIdx.x;
    constexpr int WPX = BX / 8;                                 // waves per brick row
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
    const int tx = 8 * (wv % WPX) + (tid & 7), ty = 8 * (wv / WPX) + ((tid >> 3) & 7);
    // a wave whose columns all lie beyond the grid's x or y edge (bricks of a
    // ragged grid) stages atoms with the others but computes no pairs
    const bool live = ix0 + 8 * (wv % WPX) < a.nx && iy0 + 8 * (wv / WPX) < a.ny;

    // brick centre in FP64
    const double hcx = 0.5 * (BX - 1), hcy = 0.5 * (BY - 1), hcz = 0.5 * (NZB - 1);
    const double cx = a.ox + (ix0 + hcx) * a.hx;
    const double cy = a.oy + (iy0 + hcy) * a.hy;
    const double cz = a.oz + (iz0 + hcz) * a.hz;
    // this thread's voxels relative to the brick centre, exactly rounded
    const float vx = (float)((tx - hcx) * a.hx);
    const float vy = (float)((ty - hcy) * a.hy);
    float vz[NZB];
#pragma unroll
    for (int k = 0; k < NZB; ++k) vz[k] = (float)((k - hcz) * a.hz);

    // E_cl: the energy of the close interior atoms (periodic), kept apart so
    // that the small terms of later chunks are not rounded against it
    float Fx[NZB], Fy[NZB], Fz[NZB], E[NZB], E_cl[NZB];
#pragma unroll
    for (int k = 0; k < NZB; ++k) Fx[k] = Fy[k] = Fz[k] = E[k] = E_cl[k] = 0.0f;
    // this wave's box (periodic culling): its 8 x 8 columns, all NZB heights
    const float wex = (float)(3.5 * a.hx), wey = (float)(3.5 * a.hy), wez = (float)(hcz * a.hz);
    const float wcx = (float)((8 * (wv % WPX) + 3.5 - hcx) * a.hx);
    const float wcy = (float)((8 * (wv / WPX) + 3.5 - hcy) * a.hy);
    float rc2_in = 0.f, rc2_out = 0.f;
    if (PERIODIC) {
        rc2_in = (float)((a.rc - 1e-3) * (a.rc - 1e-3));
        rc2_out = (float)((a.rc + 1e-3) * (a.rc + 1e-3));
    }

    // periods and cutoff as reciprocals, once per brick (the minimum image
    // rounds dx / Lx to an integer; a product with 1/Lx can round the other
    // way only at half a period, where both images lie beyond the cull radius)
    const double iLx = PERIODIC ? 1.0 / a.Lx : 0.0, iLy = PERIODIC ? 1.0 / a.Ly : 0.0;
    const double irc = PERIODIC ? 1.0 / a.rc : 0.0;
    // an atom's staged record: mixing (R_iP, e_iP, kq_i) folded into A_i, B_i,
    // and on periodic samples its shifted-force constants, all in FP64
    auto atom_record = [&](int ia, float4 &geo, float4 &par, float4 &aux) {
        const double RiP = R[ia] + a.R_pp;
        const double eiP = sqrt(eps[ia] * a.eps_pp);
        const double R6 = RiP * RiP * RiP * RiP * RiP * RiP;
        const double A = eiP * R6 * R6, B = 2.0 * eiP * R6;
        geo.w = (float)A;
        par = make_float4((float)(12.0 * A), (float)(-6.0 * B), (float)(a.kq_pp * q[ia]),
                          (float)(-B));
        aux = make_float4(0.f, 0.f, (float)(a.kQ_pp * q[ia]), 0.f);
        if (PERIODIC) {
            // U(rc) and fc = -dU/drho(rc) of the LJ + Coulomb pair, in FP64
            const double rc = a.rc;
            const double sc2 = RiP * RiP * irc * irc, sc6 = sc2 * sc2 * sc2;
            const double sc12 = sc6 * sc6, kq = a.kq_pp * q[ia];
            const double Uc = eiP * (sc12 - 2.0 * sc6) + kq * irc;
            double fc = 12.0 * eiP * (sc12 - sc6) * irc + kq * irc * irc;
            double C = Uc + rc * fc;
            if (QUAD) {    // radial part of the shifted d_z2 term
                const double kQ = a.kQ_pp * q[ia], irc3 = irc * irc * irc;
                fc -= 3.0 * kQ * irc3 * irc;
                C -= 4.0 * kQ * irc3;
            }
            aux.x = (float)fc;
            aux.y = (float)C;
        }
    };

    for (int base = 0; base < a.n_atoms; base += NT) {
        const int i = base + tid;
        int cnt;
        if (PERIODIC) {
            // (1) minimum image and cull of atom i; deterministic compaction of
            // the kept atoms (wave ballot + per-wave offsets) with their
            // brick-local positions and indices
            bool keep = false;
            float4 geo = make_float4(0.f, 0.f, 0.f, 0.f);
            if (i < a.n_atoms) {
                double dx = pos[3 * i] - cx, dy = pos[3 * i + 1] - cy, dz = pos[3 * i + 2] - cz;
                dx -= a.Lx * rint(dx * iLx);
                dy -= a.Ly * rint(dy * iLy);
                keep = dx * dx + dy * dy + dz * dz < a.cull2;
                geo = make_float4((float)dx, (float)dy, (float)dz, 0.f);
            }
            const int lane = tid & 63;
            const unsigned long long m = __ballot(keep);
            const int before = __popcll(m & ((1ull << lane) - 1ull));
            if (lane == 0) s_wcnt[wv] = __popcll(m);
            __syncthreads();
            int off = 0;
            cnt = 0;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                off += (w < wv) ? s_wcnt[w] : 0;
                cnt += s_wcnt[w];
            }
            if (keep) {
                s_geo[off + before] = geo;
                lds.idx[off + before] = i;
            }
            __syncthreads();
            // (2) the records of the kept atoms only (about a third of the atoms
            // on the large sample): one thread per slot
            if (tid < cnt) {
                float4 g = s_geo[tid], pr, ax;
                atom_record(lds.idx[tid], g, pr, ax);
                s_geo[tid].w = g.w;
                s_par[tid] = pr;
                s_aux[tid] = ax;
            }
        } else {
            // open samples: every atom of the chunk is staged, in its own slot
            bool keep = false;
            float4 geo = make_float4(0.f, 0.f, 0.f, 0.f), par = geo, aux = geo;
            if (i < a.n_atoms) {
                const double dx = pos[3 * i] - cx, dy = pos[3 * i + 1] - cy,
                             dz = pos[3 * i + 2] - cz;
                keep = true;
                geo = make_float4((float)dx, (float)dy, (float)dz, 0.f);
                atom_record(i, geo, par, aux);
            }
            cnt = __builtin_amdgcn_readfirstlane(min(NT, a.n_atoms - base));
            if (keep) {
                s_geo[tid] = geo;
                s_par[tid] = par;
                if (QUAD) s_aux[tid] = aux;
            }
        }
        __syncthreads();

        if (PERIODIC) {
            // Per-wave lists: the wave's 8 x 8 x NZB voxels span a box (brick-
            // local, FP32) of centre (wcx, wcy, 0) and half extents (wex, wey, wez).
            // An atom enters the shell list if the box comes within rc (+1e-3 A,
            // so that no pair the FP32 mask would admit is dropped) and an
            // interior list if the whole box is within rc - 1e-3 A (every pair
            // inside the sphere, so no mask is needed).  Interior atoms within
            // kCloseA of the box go to a list of their own, summed last and into
            // an energy accumulator of their own: their terms reach thousands of
            // eV at the voxels next to them, and in the common accumulator they
            // would leave the many small terms of the other atoms (those of later
            // chunks too) to be rounded against that magnitude.
            const int lane = tid & 63;
            int n_in = 0, n_sh = 0, n_cl = 0;
            // rounds of 64 staged atoms, as many as the chunk kept (cnt and
            // live are wave-uniform)
            const int cnt_w = live ? cnt : 0;
            for (int r = 0; r * 64 < cnt_w; ++r) {
                const int j = r * 64 + lane;
                bool is_in = false, is_sh = false, is_cl = false;
                if (j < cnt_w) {
                    const float4 g = s_geo[j];
                    const float ax = fabsf(g.x - wcx), ay = fabsf(g.y - wcy), az = fabsf(g.z);
                    const float nx_ = fmaxf(ax - wex, 0.f), ny_ = fmaxf(ay - wey, 0.f),
                                nz_ = fmaxf(az - wez, 0.f);
                    const float near2 = fmaf(nx_, nx_, fmaf(ny_, ny_, nz_ * nz_));
                    const float fx_ = ax + wex, fy_ = ay + wey, fz_ = az + wez;
                    const float far2 = fmaf(fx_, fx_, fmaf(fy_, fy_, fz_ * fz_));
                    const bool inner = far2 < rc2_in;
                    is_cl = inner && near2 < kCloseA * kCloseA;
                    is_in = inner && !is_cl;
                    is_sh = !inner && near2 < rc2_out;
                }
                const unsigned long long mi = __ballot(is_in), ms = __ballot(is_sh),
                                         mc = __ballot(is_cl);
                const unsigned long long below = (1ull << lane) - 1ull;
                if (is_in) lds.list[wv][0][n_in + __popcll(mi & below)] = (uint16_t)(16 * j);
                if (is_sh) lds.list[wv][1][n_sh + __popcll(ms & below)] = (uint16_t)(16 * j);
                if (is_cl) lds.list[wv][2][n_cl + __popcll(mc & below)] = (uint16_t)(16 * j);
                n_in += __popcll(mi);
                n_sh += __popcll(ms);
                n_cl += __popcll(mc);
            }
            __syncthreads();
            // the next atom's list entry and data are read before the current
            // atom's pairs, so the LDS latency overlaps them
            auto rec = [&](int off, float4 &g, float4 &p, float4 &x) {
                g = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_geo) + off);
                p = *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_par) + off);
                x = lds_aux<QUAD>(
                    reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(s_aux) + off), 0);
            };
            // the pairs of one list; unmasked (interior) atoms return their -C
            // for the caller to subtract once per wave
            auto pairs = [&](auto masked, const uint16_t *L, int n, float(&Eacc)[NZB]) {
                constexpr bool M = decltype(masked)::value;
                float sc = 0.0f;
                if (n == 0) return sc;
                float4 g, pa, ax;
                rec(L[0], g, pa, ax);
                for (int j = 0; j < n; ++j) {
                    float4 gn, pn, xn;
                    rec(L[min(j + 1, n - 1)], gn, pn, xn);
                    ff_pair<NZB, true, M, EONLY, QUAD>(g, pa, ax, vx, vy, vz, a.rc2, c9, c12,
                                                       c18, c24, Fx, Fy, Fz, Eacc);
                    if (!M) sc += ax.y;
                    g = gn;
                    pa = pn;
                    ax = xn;
                }
                return sc;
            };
            // interior, shell, then the close interior atoms
            float sumC = pairs(std::false_type{}, lds.list[wv][0], n_in, E);
            pairs(std::true_type{}, lds.list[wv][1], n_sh, E);
            sumC += pairs(std::false_type{}, lds.list[wv][2], n_cl, E_cl);
#pragma unroll
            for (int k = 0; k < NZB; ++k) E[k] -= sumC;
        } else {
            const int cnt_w = live ? cnt : 0;
            for (int j = 0; j < cnt_w; ++j)
                ff_pair<NZB, false, false, EONLY, QUAD>(
                    s_geo[j], s_par[j],
                    QUAD ? s_aux[j] : make_float4(0.f, 0.f, 0.f, 0.f), vx, vy, vz, a.rc2, c9,
                    c12, c18, c24, Fx, Fy, Fz, E);
        }
        __syncthreads();
    }

    const int ix = ix0 + tx, iy = iy0 + ty;
    if (ix < a.nx && iy < a.ny) {
#pragma unroll
        for (int k = 0; k < NZB; ++k) {
            const int iz = iz0 + k;
            if (iz < a.nz) {
                const size_t o = ((size_t)iz * a.ny + iy) * a.nx + ix;
                const float e = PERIODIC ? E[k] + E_cl[k] : E[k];
                if (EONLY) reinterpret_cast<float *>(ff)[o] = e;
                else ff[o] = make_float4(Fx[k], Fy[k], Fz[k], e);
            }
        }
    }
}

// At most four waves per SIMD: the register budget (up to 128 VGPRs) lets the
// compiler put independent work after each v_rsq_f32 instead of its consumer,
// which on gfx950 costs a wait state per pair (72 VGPRs, seven waves per SIMD:
// 0.35 ms at 240^3; four: 0.32 ms).  Periodic bricks of depth 8 get three
// (up to 168 VGPRs): within 128 the compiler evaluates their eight voxels one
// after another, each a dependent chain, instead of interleaving them (large
// periodic build at depth 8: 5.2 ms with four waves, 4.2 ms with three).
template <int BX, int BY, int NZB, bool PERIODIC, bool EONLY, bool QUAD>
__global__ __launch_bounds__(BX * BY) __attribute__((amdgpu_waves_per_eu(1, (PERIODIC && NZB > 6) ? 3 : 4))) void ff_build_kernel(
    const FFArgs a, const double *__restrict__ pos, const double *__restrict__ q,
    const double *__restrict__ R, const double *__restrict__ eps, float4 *__restrict__ ff)
{
    __shared__ BrickLds<BX * BY> lds;
    ff_brick<BX, BY, NZB, PERIODIC, EONLY, QUAD>(a, blockIdx.x * BX, blockIdx.y * BY,
                                                 blockIdx.z * NZB, pos, q, R, eps, ff, lds);
}

// Batched build: one block per brick of any molecule of the batch.  The
// molecule of a brick is found by a binary search over the table's
// brick_begin (wave-uniform, scalar loads); its grid, atom range, arena
// offset and brick depth (ff_nzb, 6 or 8 voxels per thread) come from the
// table.  The probe (mixing parameters) is shared.
template <int BX, int BY, int NZB, bool QUAD>
__device__ __forceinline__ void ff_batch_brick(FFArgs a, const ppm_batch_mol &M, long long local,
                                               const double *__restrict__ pos,
                                               const double *__restrict__ q,
                                               const double *__restrict__ R,
                                               const double *__restrict__ eps,
                                               float4 *__restrict__ arena, BrickLds<BX * BY> &lds)
{
    const int nbx = (M.grid.n[0] + BX - 1) / BX, nby = (M.grid.n[1] + BY - 1) / BY;
    const int bz = (int)(local / ((long long)nbx * nby));
    if (bz * NZB >= M.grid.n[2]) return;      // past the last brick of the batch
    const int rest = (int)(local - (long long)bz * nbx * nby);
    const int off = M.atom_begin;
    float4 *ff = arena + M.ff_offset;
    if (M.grid.periodic_xy) {
        const double hd = ff_brick_half_diagonal_dev<BX, BY, NZB>(a.hx, a.hy, a.hz);
        a.Lx = a.nx * a.hx;
        a.Ly = a.ny * a.hy;
        a.rc2 = (float)(M.grid.cutoff * M.grid.cutoff);
        a.cull2 = (M.grid.cutoff + hd) * (M.grid.cutoff + hd);
        a.rc = M.grid.cutoff;
        ff_brick<BX, BY, NZB, true, false, QUAD>(a, (rest % nbx) * BX, (rest / nbx) * BY,
                                                 bz * NZB, pos + 3 * (size_t)off, q + off,
                                                 R + off, eps + off, ff, lds);
    } else {
        ff_brick<BX, BY, NZB, false, false, QUAD>(a, (rest % nbx) * BX, (rest / nbx) * BY,
                                                  bz * NZB, pos + 3 * (size_t)off, q + off,
                                                  R + off, eps + off, ff, lds);
    }
}

template <int BX, int BY, bool QUAD>
__global__ __launch_bounds__(BX * BY) void ff_build_batch_kernel(
    const FFArgs probe_args, const ppm_batch_mol *__restrict__ mols, int n_mol,
    const double *__restrict__ pos, const double *__restrict__ q, const double *__restrict__ R,
    const double *__restrict__ eps, float4 *__restrict__ arena)
{
    __shared__ BrickLds<BX * BY> lds;
    const long long b = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    int lo = 0, hi = n_mol - 1;               // last molecule with brick_begin <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (mols[mid].brick_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const ppm_batch_mol &M = mols[lo];
    FFArgs a = probe_args;
    a.ox = M.grid.origin[0];
    a.oy = M.grid.origin[1];
    a.oz = M.grid.origin[2];
    a.hx = M.grid.step[0];
    a.hy = M.grid.step[1];
    a.hz = M.grid.step[2];
    a.nx = M.grid.n[0];
    a.ny = M.grid.n[1];
    a.nz = M.grid.n[2];
    a.n_atoms = M.n_atoms;
    const long long local = b - M.brick_begin;
    if (M.ff_nzb == 6)
        ff_batch_brick<BX, BY, 6, QUAD>(a, M, local, pos, q, R, eps, arena, lds);
    else
        ff_batch_brick<BX, BY, 8, QUAD>(a, M, local, pos, q, R, eps, arena, lds);
}

// 16 x 16-column bricks, 8 voxels per thread along z unless the autotuner
// chose 6.  Grid extents are usually multiples of 16 voxels (240 at the
// paper's scale) or close to one, so few threads of the last brick of a row
// idle (64-wide bricks left a quarter of them idle on a 240-voxel row: 0.38
// against 0.35 ms); the small half-diagonal keeps a periodic brick's cull
// sphere (cutoff + half-diagonal) close to the cutoff sphere and the
// brick-local coordinates small.
constexpr int kBX = 16, kBY = 16, kNZB = 8;

int brick_depth(int nzb) { return nzb == 6 ? 6 : kNZB; }

}  // namespace

// Brick geometry used by the launcher (the host validates the periodic cutoff
// against its half-diagonal).
double ff_brick_half_diagonal(double hx, double hy, double hz, int nzb)
{
    return brick_depth(nzb) == 6 ? ff_brick_half_diagonal_dev<kBX, kBY, 6>(hx, hy, hz)
                                 : ff_brick_half_diagonal_dev<kBX, kBY, kNZB>(hx, hy, hz);
}

long long ff_brick_count(int nx, int ny, int nz, int nzb)
{
    const int d = brick_depth(nzb);
    return (long long)((nx + kBX - 1) / kBX) * ((ny + kBY - 1) / kBY) * ((nz + d - 1) / d);
}

template <int NZB, bool EONLY, bool QUAD>
void launch_build(const FFArgs &a, const double *pos, const double *q, const double *R,
                  const double *eps, float4 *out, hipStream_t stream)
{
    dim3 block(kBX, kBY, 1);
    dim3 grid((a.nx + kBX - 1) / kBX, (a.ny + kBY - 1) / kBY, (a.nz + NZB - 1) / NZB);
    if (a.Lx > 0.0)
        hipLaunchKernelGGL((ff_build_kernel<kBX, kBY, NZB, true, EONLY, QUAD>), grid, block, 0,
                           stream, a, pos, q, R, eps, out);
    else
        hipLaunchKernelGGL((ff_build_kernel<kBX, kBY, NZB, false, EONLY, QUAD>), grid, block, 0,
                           stream, a, pos, q, R, eps, out);
}

hipError_t launch_build_ff(const FFArgs &a, const double *pos, const double *q,
                           const double *R, const double *eps, float4 *ff, hipStream_t stream,
                           int nzb)
{
    if (brick_depth(nzb) == 6) {
        if (a.kQ_pp != 0.0) launch_build<6, false, true>(a, pos, q, R, eps, ff, stream);
        else launch_build<6, false, false>(a, pos, q, R, eps, ff, stream);
    } else {
        if (a.kQ_pp != 0.0) launch_build<kNZB, false, true>(a, pos, q, R, eps, ff, stream);
        else launch_build<kNZB, false, false>(a, pos, q, R, eps, ff, stream);
    }
    return hipGetLastError();
}

hipError_t launch_build_energy(const FFArgs &a, const double *pos, const double *q,
                               const double *R, const double *eps, float *E, hipStream_t stream)
{
    float4 *out = reinterpret_cast<float4 *>(E);   // EONLY kernels store floats
    if (a.kQ_pp != 0.0) launch_build<kNZB, true, true>(a, pos, q, R, eps, out, stream);
    else launch_build<kNZB, true, false>(a, pos, q, R, eps, out, stream);
    return hipGetLastError();
}

hipError_t launch_build_ff_batch(const FFArgs &probe_args, const ppm_batch_mol *mols_dev,
                                 int n_mol, long long n_bricks, const double *pos,
                                 const double *q, const double *R, const double *eps,
                                 float4 *arena, hipStream_t stream)
{
    if (n_bricks <= 0) return hipSuccess;
    // 2-D grid: x up to 65536 blocks per row, as many rows as needed
    const long long gx = n_bricks < 65536 ? n_bricks : 65536;
    const long long gy = (n_bricks + gx - 1) / gx;
    if (probe_args.kQ_pp != 0.0)
        hipLaunchKernelGGL((ff_build_batch_kernel<kBX, kBY, true>),
                           dim3((unsigned)gx, (unsigned)gy, 1), dim3(kBX, kBY, 1), 0, stream,
                           probe_args, mols_dev, n_mol, pos, q, R, eps, arena);
    else
        hipLaunchKernelGGL((ff_build_batch_kernel<kBX, kBY, false>),
                           dim3((unsigned)gx, (unsigned)gy, 1), dim3(kBX, kBY, 1), 0, stream,
                           probe_args, mols_dev, n_mol, pos, q, R, eps, arena);
    return hipGetLastError();
}

}  // namespace ppm
