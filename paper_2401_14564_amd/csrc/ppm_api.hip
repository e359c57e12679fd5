// ppm_api.hip -- host side of the C ABI declared in include/ppm.h: argument
// validation, derived constants, and kernel launches.  Nothing here computes
// per-voxel or per-point results; every step of the path runs in the kernels.
#include <math.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "ppm.h"
#include "ppm_kernels.h"

using namespace ppm;

// Workspace of ppm_relaxed_scan_backward_noalloc: one copy in every GPU's
// memory that the library runs on, held until the process ends.  In host code
// `scratch` is only a symbol: its device address (different on each GPU) comes
// from hipGetSymbolAddress, taken once per device in noalloc_scratch().
static __device__ __align__(256) unsigned char scratch[PPM_NOALLOC_SCRATCH_BYTES];

namespace {

thread_local int32_t g_last_hip_error = 0;

constexpr int kMaxScratchDevices = 64;
std::atomic<void *> g_scratch_ptr[kMaxScratchDevices];
std::mutex g_scratch_mutex;

ppm_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return PPM_OK;
    g_last_hip_error = (int32_t)e;
    return PPM_EHIP;
}

// Device address of `scratch` on the current device (looked up on the first
// call per device, with that device current, then cached).
ppm_status noalloc_scratch(void **out)
{
    int dev = 0;
    ppm_status st = hip_status(hipGetDevice(&dev));
    if (st != PPM_OK) return st;
    if (dev < 0 || dev >= kMaxScratchDevices) return PPM_EUNSUPPORTED;
    void *p = g_scratch_ptr[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mutex);
        p = g_scratch_ptr[dev].load(std::memory_order_acquire);
        if (!p) {
            st = hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
            if (st != PPM_OK) return st;
            if (!p) return PPM_EHIP;
            g_scratch_ptr[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return PPM_OK;
}

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

ppm_status check_grid(const ppm_grid *g)
{
    if (!g) return PPM_EINVAL;
    for (int i = 0; i < 3; ++i) {
        if (g->n[i] < 2) return PPM_EINVAL;
        if (!finite_pos(g->step[i]) || !isfinite(g->origin[i])) return PPM_EINVAL;
    }
    const double nv = (double)g->n[0] * g->n[1] * g->n[2];
    if (nv >= 2147483648.0) return PPM_ERANGE;
    if (g->periodic_xy != 0 && g->periodic_xy != 1) return PPM_EINVAL;
    return PPM_OK;
}

ppm_status check_probe(const ppm_probe *p)
{
    if (!p) return PPM_EINVAL;
    if (!isfinite(p->R_pp) || !(p->eps_pp >= 0.0) || !isfinite(p->eps_pp) || !isfinite(p->q_pp) ||
        !isfinite(p->q_zz))
        return PPM_EINVAL;
    if (!(p->k_lat[0] >= 0.0) || !(p->k_lat[1] >= 0.0) || !(p->k_rad >= 0.0)) return PPM_EINVAL;
    if (!isfinite(p->k_lat[0]) || !isfinite(p->k_lat[1]) || !isfinite(p->k_rad)) return PPM_EINVAL;
    const double R0 = sqrt(p->d0[0] * p->d0[0] + p->d0[1] * p->d0[1] + p->d0[2] * p->d0[2]);
    if (!finite_pos(R0)) return PPM_EINVAL;
    return PPM_OK;
}

ppm_status check_fire(const ppm_fire *f)
{
    if (!f) return PPM_EINVAL;
    if (!finite_pos(f->dt0) || !finite_pos(f->dt_max) || !finite_pos(f->mass) ||
        !finite_pos(f->f_conv))
        return PPM_EINVAL;
    if (!finite_pos(f->f_inc) || !finite_pos(f->f_dec) || !isfinite(f->alpha0) ||
        !isfinite(f->f_alpha))
        return PPM_EINVAL;
    if (f->alpha0 < 0.0 || f->alpha0 > 1.0 || f->f_alpha < 0.0 || f->f_alpha > 1.0)
        return PPM_EINVAL;
    if (f->n_min < 0 || f->max_iter < 1) return PPM_EINVAL;
    return PPM_OK;
}

ppm_status check_scan(const ppm_scan *s)
{
    if (!s) return PPM_EINVAL;
    if (s->nx < 1 || s->ny < 1 || s->nz < 1) return PPM_EINVAL;
    if (!isfinite(s->x0) || !isfinite(s->y0) || !isfinite(s->dx) || !isfinite(s->dy) ||
        !isfinite(s->z_top) || !isfinite(s->dz))
        return PPM_EINVAL;
    if (s->nz > 1 && !finite_pos(s->dz)) return PPM_EINVAL;
    const double n = (double)s->nx * s->ny * s->nz;
    if (n >= 1099511627776.0) return PPM_ERANGE;   // 2^40 points
    return PPM_OK;
}

int32_t df_half_width(double A, double dz)
{
    if (!finite_pos(A) || !finite_pos(dz)) return -1;
    const double m = ceil(A / (2.0 * dz) - 1e-9);
    if (m > 1e6) return -1;
    return (int32_t)m;
}

// Exact weights of Eq. 3 for the piecewise-linear interpolant of the samples
// (integrals of z/sqrt(a^2-z^2) and z^2/sqrt(a^2-z^2) on each segment), with the
// prefactor -(f0/2k)(8/(pi A^2)) (N/m per eV/A^2) folded in, laid out for the
// ring buffer: W[2K - lag] multiplies the sample `lag` heights before the newest,
// i.e. the sample at physical offset j = lag - m from the centre.
ppm_status df_weights(const ppm_df_params *p, double dz, int m, DfWeights *W)
{
    if (!p || !finite_pos(p->A) || !finite_pos(p->k_cant) || !isfinite(p->f0))
        return PPM_EINVAL;
    if (m > kMaxDfHalfWidth) return PPM_EUNSUPPORTED;
    memset(W, 0, sizeof(*W));
    const double a = 0.5 * p->A;
    double w[2 * kMaxDfHalfWidth + 1] = {0};
    for (int j = -m; j < m; ++j) {
        const double z0 = j * dz, z1 = (j + 1) * dz;
        const double lo = fmax(z0, -a), hi = fmin(z1, a);
        if (!(lo < hi)) continue;
        const double rl = sqrt(fmax(a * a - lo * lo, 0.0)), rh = sqrt(fmax(a * a - hi * hi, 0.0));
        const double I1 = rl - rh;   // int z / sqrt(a^2 - z^2)
        const double I2 = 0.5 * a * a * (asin(fmin(hi / a, 1.0)) - asin(fmax(lo / a, -1.0))) -
                          0.5 * (hi * rh - lo * rl);   // int z^2 / sqrt(a^2 - z^2)
        w[j + m] += (z1 * I1 - I2) / dz;
        w[j + 1 + m] += (I2 - z0 * I1) / dz;
    }
    const double C = -(p->f0 / (2.0 * p->k_cant)) * (8.0 / (M_PI * p->A * p->A)) *
                     kEvPerA2InNewtonPerM;
    const int K = kMaxDfHalfWidth;
    for (int lag = 0; lag <= 2 * m; ++lag) W->w[2 * K - lag] = (float)(C * w[lag]);
    // lag = m + j  ->  w index j + m = lag
    return PPM_OK;
}

ScanArgs make_scan_args(const ppm_grid *g, const ppm_probe *p, const ppm_fire *f,
                        const ppm_scan *s)
{
    ScanArgs a;
    memset(&a, 0, sizeof(a));
    fill_scan_geometry(a, *g, *p, *s);
    if (f) {
        a.dt0 = f->dt0;
        a.dt_max = f->dt_max;
        a.f_inc = f->f_inc;
        a.f_dec = f->f_dec;
        a.alpha0 = f->alpha0;
        a.f_alpha = f->f_alpha;
        a.inv_mass = 1.0 / f->mass;
        a.f_conv2 = f->f_conv * f->f_conv;
        a.n_min = f->n_min;
        a.max_iter = f->max_iter;
        a.lerp32 = f->f_conv >= kLerp32MinFconv ? 1 : 0;
    }
    return a;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Chunks of relaxed points for the atom scatter of the backward pass: tiles of
// 8 x 8 tip columns x 2 heights (the scatter kernel's layout).
void backward_chunks(const ppm_scan *s, int *n_blocks, int *per_block)
{
    const long long nb = (long long)((s->nx + 7) / 8) * ((s->ny + 7) / 8) * ((s->nz + 1) / 2);
    *n_blocks = (int)(nb < 1 ? 1 : nb);
    *per_block = 128;
}

size_t backward_record_bytes(const ppm_scan *s)
{
    return align256((size_t)s->nx * s->ny * s->nz * 48);
}

// Median time (ms) of three launches of `run` after one untimed launch, with
// HIP events on `stream`; negative if an event call failed.
template <typename Run>
float time_median3(hipStream_t stream, Run run, ppm_status *st)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.0f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.0f;
    }
    float t[3] = {0.f, 0.f, 0.f};
    *st = run();
    for (int r = 0; r < 3 && *st == PPM_OK; ++r) {
        if (hipEventRecord(e0, stream) != hipSuccess) { *st = PPM_EHIP; break; }
        *st = run();
        if (*st != PPM_OK) break;
        if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t[r], e0, e1) != hipSuccess)
            *st = PPM_EHIP;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (*st != PPM_OK) return -1.0f;
    const float lo = fminf(t[0], fminf(t[1], t[2])), hi = fmaxf(t[0], fmaxf(t[1], t[2]));
    return t[0] + t[1] + t[2] - lo - hi;
}

}  // namespace

extern "C" {

const char *ppm_status_string(ppm_status s)
{
    switch (s) {
    case PPM_OK: return "ok";
    case PPM_EINVAL: return "invalid argument";
    case PPM_ERANGE: return "size out of range";
    case PPM_EHIP: return "HIP runtime error";
    case PPM_EUNSUPPORTED: return "unsupported by this build";
    default: return "unknown status";
    }
}

int32_t ppm_last_hip_error(void) { return g_last_hip_error; }

int32_t ppm_df_half_width(double A, double dz) { return df_half_width(A, dz); }

static bool valid_nzb(int nzb) { return nzb == 0 || nzb == 6 || nzb == 8; }
static bool valid_tile(int tile) { return tile == 0 || tile == 8 || tile == 16; }

static ppm_status ff_setup(const ppm_grid *grid, const ppm_probe *probe, int32_t n_atoms,
                           const double *pos, const double *q, const double *R,
                           const double *eps, const void *out, FFArgs *a, int nzb = 0)
{
    ppm_status st = check_grid(grid);
    if (st != PPM_OK) return st;
    if ((st = check_probe(probe)) != PPM_OK) return st;
    if (n_atoms < 0 || !out) return PPM_EINVAL;
    if (n_atoms > 0 && (!pos || !q || !R || !eps)) return PPM_EINVAL;
    memset(a, 0, sizeof(*a));
    a->ox = grid->origin[0];
    a->oy = grid->origin[1];
    a->oz = grid->origin[2];
    a->hx = grid->step[0];
    a->hy = grid->step[1];
    a->hz = grid->step[2];
    a->nx = grid->n[0];
    a->ny = grid->n[1];
    a->nz = grid->n[2];
    a->n_atoms = n_atoms;
    a->R_pp = probe->R_pp;
    a->eps_pp = probe->eps_pp;
    a->kq_pp = kCoulomb * probe->q_pp;
    a->kQ_pp = kCoulomb * probe->q_zz;
    if (grid->periodic_xy) {
        const double Lx = grid->n[0] * grid->step[0], Ly = grid->n[1] * grid->step[1];
        const double hd =
            ff_brick_half_diagonal(grid->step[0], grid->step[1], grid->step[2], nzb);
        if (!finite_pos(grid->cutoff) || grid->cutoff + hd >= 0.5 * fmin(Lx, Ly))
            return PPM_EINVAL;
        a->Lx = Lx;
        a->Ly = Ly;
        a->rc2 = (float)(grid->cutoff * grid->cutoff);
        a->cull2 = (grid->cutoff + hd) * (grid->cutoff + hd);
        a->rc = grid->cutoff;
    }
    return PPM_OK;
}

ppm_status ppm_build_ff_tuned(const ppm_grid *grid, const ppm_probe *probe,
                              const ppm_tuning *tuning, int32_t n_atoms, const double *pos,
                              const double *q, const double *R, const double *eps, float *ff,
                              void *stream)
{
    const int nzb = tuning ? tuning->ff_nzb : 0;
    if (!valid_nzb(nzb)) return PPM_EINVAL;
    FFArgs a;
    ppm_status st = ff_setup(grid, probe, n_atoms, pos, q, R, eps, ff, &a, nzb);
    if (st != PPM_OK) return st;
    return hip_status(launch_build_ff(a, pos, q, R, eps, reinterpret_cast<float4 *>(ff),
                                      (hipStream_t)stream, nzb));
}

ppm_status ppm_build_ff(const ppm_grid *grid, const ppm_probe *probe, int32_t n_atoms,
                        const double *pos, const double *q, const double *R,
                        const double *eps, float *ff, void *stream)
{
    return ppm_build_ff_tuned(grid, probe, nullptr, n_atoms, pos, q, R, eps, ff, stream);
}

ppm_status ppm_tune_build_ff(const ppm_grid *grid, const ppm_probe *probe, int32_t n_atoms,
                             const double *pos, const double *q, const double *R,
                             const double *eps, float *ff, void *stream, ppm_tuning *tuning,
                             float *ms)
{
    if (!tuning) return PPM_EINVAL;
    FFArgs a;
    ppm_status st = ff_setup(grid, probe, n_atoms, pos, q, R, eps, ff, &a, 8);
    if (st != PPM_OK) return st;
    const int cand[2] = {8, 6};
    float t[2];
    for (int c = 0; c < 2; ++c) {
        ppm_tuning tt = *tuning;
        tt.ff_nzb = cand[c];
        t[c] = time_median3((hipStream_t)stream, [&]() {
            return ppm_build_ff_tuned(grid, probe, &tt, n_atoms, pos, q, R, eps, ff, stream);
        }, &st);
        if (st != PPM_OK) return st;
    }
    tuning->ff_nzb = t[1] < t[0] ? 6 : 8;
    if (ms) { ms[0] = t[0]; ms[1] = t[1]; }
    return PPM_OK;
}

ppm_status ppm_build_energy(const ppm_grid *grid, const ppm_probe *probe, int32_t n_atoms,
                            const double *pos, const double *q, const double *R,
                            const double *eps, float *E, void *stream)
{
    FFArgs a;
    ppm_status st = ff_setup(grid, probe, n_atoms, pos, q, R, eps, E, &a);
    if (st != PPM_OK) return st;
    return hip_status(launch_build_energy(a, pos, q, R, eps, E, (hipStream_t)stream));
}

static ppm_status scan_setup(const ppm_grid *grid, const void *field, const ppm_probe *probe,
                             const ppm_fire *fire, const ppm_scan *scan, float *fz, float *pp,
                             const ppm_df_params *dfp, float *df, ScanArgs *a, DfWeights *W)
{
    ppm_status st;
    if ((st = check_grid(grid)) != PPM_OK) return st;
    if ((st = check_probe(probe)) != PPM_OK) return st;
    if ((st = check_fire(fire)) != PPM_OK) return st;
    if ((st = check_scan(scan)) != PPM_OK) return st;
    if (!field || (!fz && !pp && !df)) return PPM_EINVAL;
    *a = make_scan_args(grid, probe, fire, scan);
    memset(W, 0, sizeof(*W));
    a->m = 0;
    if (df) {
        if (!dfp) return PPM_EINVAL;
        const int m = df_half_width(dfp->A, scan->dz);
        if (m < 1) return PPM_EINVAL;
        if (m > kMaxDfHalfWidth) return PPM_EUNSUPPORTED;
        if (scan->nz < 2 * m + 1) return PPM_EINVAL;
        if (scan->nz > kMaxScanLdsHeights && !fz) return PPM_EUNSUPPORTED;
        if ((st = df_weights(dfp, scan->dz, m, W)) != PPM_OK) return st;
        a->m = m;
        a->ndf = scan->nz - 2 * m;
    }
    return PPM_OK;
}

ppm_status ppm_relaxed_scan_tuned(const ppm_grid *grid, const float *ff,
                                  const ppm_probe *probe, const ppm_fire *fire,
                                  const ppm_scan *scan, const ppm_tuning *tuning, float *fz,
                                  float *pp, const ppm_df_params *dfp, float *df, void *stream)
{
    const int tile = tuning ? tuning->scan_tile : 0;
    const int direct = tuning ? tuning->scan_fz_direct : 0;
    if (!valid_tile(tile) || (direct != 0 && direct != 1)) return PPM_EINVAL;
    ScanArgs a;
    DfWeights W;
    ppm_status st = scan_setup(grid, ff, probe, fire, scan, fz, pp, dfp, df, &a, &W);
    if (st != PPM_OK) return st;
    return hip_status(launch_relaxed_scan(a, W, reinterpret_cast<const float4 *>(ff), fz,
                                          reinterpret_cast<float4 *>(pp), df,
                                          (hipStream_t)stream, tile, direct != 0));
}

ppm_status ppm_relaxed_scan(const ppm_grid *grid, const float *ff, const ppm_probe *probe,
                            const ppm_fire *fire, const ppm_scan *scan, float *fz, float *pp,
                            const ppm_df_params *dfp, float *df, void *stream)
{
    return ppm_relaxed_scan_tuned(grid, ff, probe, fire, scan, nullptr, fz, pp, dfp, df, stream);
}

ppm_status ppm_tune_relaxed_scan(const ppm_grid *grid, const float *ff, const ppm_probe *probe,
                                 const ppm_fire *fire, const ppm_scan *scan, float *fz,
                                 float *pp, const ppm_df_params *dfp, float *df, void *stream,
                                 ppm_tuning *tuning, float *ms)
{
    if (!tuning) return PPM_EINVAL;
    ScanArgs a;
    DfWeights W;
    ppm_status st = scan_setup(grid, ff, probe, fire, scan, fz, pp, dfp, df, &a, &W);
    if (st != PPM_OK) return st;
    // (scan_tile, scan_fz_direct); the direct route only with an fz output
    const int cand[3][2] = {{16, 0}, {8, 0}, {8, 1}};
    const int n_cand = fz ? 3 : 2;
    float t[3] = {0.0f, 0.0f, 0.0f};
    int best = 0;
    for (int c = 0; c < n_cand; ++c) {
        ppm_tuning tt = *tuning;
        tt.scan_tile = cand[c][0];
        tt.scan_fz_direct = cand[c][1];
        t[c] = time_median3((hipStream_t)stream, [&]() {
            return ppm_relaxed_scan_tuned(grid, ff, probe, fire, scan, &tt, fz, pp, dfp, df,
                                          stream);
        }, &st);
        if (st != PPM_OK) return st;
        if (t[c] < t[best]) best = c;
    }
    tuning->scan_tile = cand[best][0];
    tuning->scan_fz_direct = cand[best][1];
    if (ms) { ms[0] = t[0]; ms[1] = t[1]; ms[2] = t[2]; }
    return PPM_OK;
}

ppm_status ppm_relaxed_scan_tricubic(const ppm_grid *grid, const float *E,
                                     const ppm_probe *probe, const ppm_fire *fire,
                                     const ppm_scan *scan, float *fz, float *pp,
                                     const ppm_df_params *dfp, float *df, void *stream)
{
    ScanArgs a;
    DfWeights W;
    ppm_status st = scan_setup(grid, E, probe, fire, scan, fz, pp, dfp, df, &a, &W);
    if (st != PPM_OK) return st;
    if (grid->n[2] < 2) return PPM_EINVAL;
    return hip_status(launch_relaxed_scan_tricubic(a, W, E, fz, reinterpret_cast<float4 *>(pp),
                                                   df, (hipStream_t)stream));
}

ppm_status ppm_df(const float *fz, int32_t nz, int32_t ny, int32_t nx, double dz,
                  const ppm_df_params *dfp, float *df, void *stream)
{
    if (!fz || !df || !dfp || ny < 1 || nx < 1 || !finite_pos(dz)) return PPM_EINVAL;
    const int m = df_half_width(dfp->A, dz);
    if (m < 1) return PPM_EINVAL;
    if (m > kMaxDfHalfWidth) return PPM_EUNSUPPORTED;
    if (nz < 2 * m + 1) return PPM_EINVAL;
    if ((double)nx * ny * nz >= 2147483648.0 * 4.0) return PPM_ERANGE;
    DfWeights W;
    ppm_status st = df_weights(dfp, dz, m, &W);
    if (st != PPM_OK) return st;
    return hip_status(launch_df(fz, nz, ny, nx, m, W, df, (hipStream_t)stream));
}

size_t ppm_backward_workspace_bytes(const ppm_scan *scan, int32_t n_atoms)
{
    if (check_scan(scan) != PPM_OK || n_atoms < 0) return 0;
    int nb, per;
    backward_chunks(scan, &nb, &per);
    const size_t na_pad = (size_t)((n_atoms + 63) / 64) * 64;
    return backward_record_bytes(scan) + align256((size_t)nb * na_pad * 6 * sizeof(double));
}

ppm_status ppm_relaxed_scan_backward(const ppm_grid *grid, const float *ff,
                                     const ppm_probe *probe, const ppm_scan *scan,
                                     const ppm_df_params *dfp, int32_t n_atoms,
                                     const double *pos, const double *q, const double *R,
                                     const double *eps, const float *pp,
                                     const float *grad_df, double *g_pos, double *g_q,
                                     double *g_R, double *g_eps, void *workspace,
                                     size_t workspace_bytes, void *stream)
{
    ppm_status st;
    if ((st = check_grid(grid)) != PPM_OK) return st;
    if ((st = check_probe(probe)) != PPM_OK) return st;
    if ((st = check_scan(scan)) != PPM_OK) return st;
    if (!ff || !pp || !grad_df || !dfp || n_atoms < 0) return PPM_EINVAL;
    if (n_atoms > 0 && (!pos || !q || !R || !eps || !g_pos || !g_q || !g_R || !g_eps))
        return PPM_EINVAL;
    const int m = df_half_width(dfp->A, scan->dz);
    if (m < 1) return PPM_EINVAL;
    if (m > kMaxDfHalfWidth) return PPM_EUNSUPPORTED;
    if (scan->nz < 2 * m + 1) return PPM_EINVAL;
    if (!workspace || workspace_bytes < ppm_backward_workspace_bytes(scan, n_atoms))
        return PPM_EINVAL;
    if (grid->periodic_xy && !finite_pos(grid->cutoff)) return PPM_EINVAL;
    DfWeights W;
    if ((st = df_weights(dfp, scan->dz, m, &W)) != PPM_OK) return st;
    BwdArgs A;
    memset(&A, 0, sizeof(A));
    A.s = make_scan_args(grid, probe, nullptr, scan);
    A.s.m = m;
    A.s.ndf = scan->nz - 2 * m;
    A.hx = grid->step[0];
    A.hy = grid->step[1];
    A.hz = grid->step[2];
    A.periodic = grid->periodic_xy;
    A.Lx = grid->n[0] * grid->step[0];
    A.Ly = grid->n[1] * grid->step[1];
    A.rc2 = (float)(grid->cutoff * grid->cutoff);
    A.rc = grid->cutoff;
    A.n_atoms = n_atoms;
    A.R_pp = probe->R_pp;
    A.eps_pp = probe->eps_pp;
    A.kq_pp = kCoulomb * probe->q_pp;
    A.ke_qpp = kCoulomb * probe->q_pp;
    A.kQ_pp = kCoulomb * probe->q_zz;
    backward_chunks(scan, &A.n_eq_blocks, &A.eq_per_block);
    char *ws = static_cast<char *>(workspace);
    float4 *rec = reinterpret_cast<float4 *>(ws);
    double *partial = reinterpret_cast<double *>(ws + backward_record_bytes(scan));
    return hip_status(launch_backward(A, W, reinterpret_cast<const float4 *>(ff),
                                      reinterpret_cast<const float4 *>(pp), grad_df, pos, q, R,
                                      eps, rec, partial, g_pos, g_q, g_R, g_eps,
                                      (hipStream_t)stream));
}

ppm_status ppm_relaxed_scan_backward_noalloc(const ppm_grid *grid, const float *ff,
                                             const ppm_probe *probe, const ppm_scan *scan,
                                             const ppm_df_params *dfp, int32_t n_atoms,
                                             const double *pos, const double *q,
                                             const double *R, const double *eps, const float *pp,
                                             const float *grad_df, double *g_pos, double *g_q,
                                             double *g_R, double *g_eps, void *stream)
{
    if (check_scan(scan) != PPM_OK || n_atoms < 0) return PPM_EINVAL;
    if (ppm_backward_workspace_bytes(scan, n_atoms) > (size_t)PPM_NOALLOC_SCRATCH_BYTES)
        return PPM_ERANGE;
    void *ws = nullptr;
    ppm_status st = noalloc_scratch(&ws);
    if (st != PPM_OK) return st;
    // the kernels write every record and partial they read: nothing to clear
    return ppm_relaxed_scan_backward(grid, ff, probe, scan, dfp, n_atoms, pos, q, R, eps, pp,
                                     grad_df, g_pos, g_q, g_R, g_eps, ws,
                                     (size_t)PPM_NOALLOC_SCRATCH_BYTES, stream);
}

static bool same_probe_lj(const ppm_probe &a, const ppm_probe &b)
{
    return a.R_pp == b.R_pp && a.eps_pp == b.eps_pp && a.q_pp == b.q_pp && a.q_zz == b.q_zz;
}

ppm_status ppm_batch_plan(int32_t n_mol, ppm_batch_mol *mols, int32_t n_jobs,
                          ppm_batch_scan *jobs, const ppm_df_params *dfp, int64_t *totals)
{
    if (n_mol < 1 || n_jobs < 0 || !mols || (n_jobs > 0 && !jobs) || !totals) return PPM_EINVAL;
    ppm_status st;
    long long vox = 0, bricks = 0;
    for (int i = 0; i < n_mol; ++i) {
        ppm_batch_mol &M = mols[i];
        if ((st = check_grid(&M.grid)) != PPM_OK) return st;
        if (M.n_atoms < 0 || M.atom_begin < 0 || !valid_nzb(M.ff_nzb)) return PPM_EINVAL;
        if (M.grid.periodic_xy) {
            const double Lx = M.grid.n[0] * M.grid.step[0], Ly = M.grid.n[1] * M.grid.step[1];
            const double hd = ff_brick_half_diagonal(M.grid.step[0], M.grid.step[1],
                                                     M.grid.step[2], M.ff_nzb);
            if (!finite_pos(M.grid.cutoff) || M.grid.cutoff + hd >= 0.5 * fmin(Lx, Ly))
                return PPM_EINVAL;
        }
        M.ff_offset = vox;
        M.brick_begin = bricks;
        vox += (long long)M.grid.n[0] * M.grid.n[1] * M.grid.n[2];
        bricks += ff_brick_count(M.grid.n[0], M.grid.n[1], M.grid.n[2], M.ff_nzb);
    }
    long long nfz = 0, ndf = 0, tiles = 0;
    int m = 0;
    if (dfp) {
        if (n_jobs > 0) {
            m = df_half_width(dfp->A, jobs[0].scan.dz);
            if (m < 1) return PPM_EINVAL;
            if (m > kMaxDfHalfWidth) return PPM_EUNSUPPORTED;
        }
    }
    for (int j = 0; j < n_jobs; ++j) {
        ppm_batch_scan &J = jobs[j];
        if (J.mol < 0 || J.mol >= n_mol) return PPM_EINVAL;
        if ((st = check_probe(&J.probe)) != PPM_OK) return st;
        if (!same_probe_lj(J.probe, jobs[0].probe)) return PPM_EINVAL;
        if ((st = check_scan(&J.scan)) != PPM_OK) return st;
        if (dfp) {
            if (J.scan.dz != jobs[0].scan.dz) return PPM_EUNSUPPORTED;
            if (J.scan.nz < 2 * m + 1) return PPM_EINVAL;
        }
        J.fz_offset = nfz;
        J.df_offset = ndf;
        J.tile_begin = tiles;
        nfz += (long long)J.scan.nx * J.scan.ny * J.scan.nz;
        if (dfp) ndf += (long long)J.scan.nx * J.scan.ny * (J.scan.nz - 2 * m);
        tiles += scan_tile_count(J.scan.nx, J.scan.ny);
    }
    totals[0] = vox;
    totals[1] = bricks;
    totals[2] = nfz;
    totals[3] = ndf;
    totals[4] = tiles;
    return PPM_OK;
}

ppm_status ppm_batch_build_ff(int32_t n_mol, const ppm_batch_mol *mols_host,
                              const ppm_batch_mol *mols_dev, const ppm_probe *probe,
                              const double *pos, const double *q, const double *R,
                              const double *eps, float *ff_arena, void *stream)
{
    if (n_mol < 1 || !mols_host || !mols_dev || !ff_arena) return PPM_EINVAL;
    ppm_status st;
    if ((st = check_probe(probe)) != PPM_OK) return st;
    long long total_atoms = 0, bricks = 0, vox = 0;
    for (int i = 0; i < n_mol; ++i) {
        const ppm_batch_mol &M = mols_host[i];
        if ((st = check_grid(&M.grid)) != PPM_OK) return st;
        if (M.n_atoms < 0 || M.atom_begin < 0 || !valid_nzb(M.ff_nzb)) return PPM_EINVAL;
        if (M.ff_offset != vox || M.brick_begin != bricks) return PPM_EINVAL;   // not planned
        if (M.grid.periodic_xy) {
            const double Lx = M.grid.n[0] * M.grid.step[0], Ly = M.grid.n[1] * M.grid.step[1];
            const double hd = ff_brick_half_diagonal(M.grid.step[0], M.grid.step[1],
                                                     M.grid.step[2], M.ff_nzb);
            if (!finite_pos(M.grid.cutoff) || M.grid.cutoff + hd >= 0.5 * fmin(Lx, Ly))
                return PPM_EINVAL;
        }
        const long long end = (long long)M.atom_begin + M.n_atoms;
        if (end > total_atoms) total_atoms = end;
        vox += (long long)M.grid.n[0] * M.grid.n[1] * M.grid.n[2];
        bricks += ff_brick_count(M.grid.n[0], M.grid.n[1], M.grid.n[2], M.ff_nzb);
    }
    if (total_atoms > 0 && (!pos || !q || !R || !eps)) return PPM_EINVAL;
    FFArgs a;
    memset(&a, 0, sizeof(a));
    a.R_pp = probe->R_pp;
    a.eps_pp = probe->eps_pp;
    a.kq_pp = kCoulomb * probe->q_pp;
    a.kQ_pp = kCoulomb * probe->q_zz;
    return hip_status(launch_build_ff_batch(a, mols_dev, n_mol, bricks, pos, q, R, eps,
                                            reinterpret_cast<float4 *>(ff_arena),
                                            (hipStream_t)stream));
}

ppm_status ppm_batch_relaxed_scan(int32_t n_mol, const ppm_batch_mol *mols_host,
                                  const ppm_batch_mol *mols_dev, int32_t n_jobs,
                                  const ppm_batch_scan *jobs_host,
                                  const ppm_batch_scan *jobs_dev, const ppm_fire *fire,
                                  const ppm_df_params *dfp, const float *ff_arena,
                                  float *fz_arena, float *df_arena, void *stream)
{
    if (n_mol < 1 || n_jobs < 1 || !mols_host || !mols_dev || !jobs_host || !jobs_dev ||
        !ff_arena)
        return PPM_EINVAL;
    ppm_status st;
    if ((st = check_fire(fire)) != PPM_OK) return st;
    if (!fz_arena && !df_arena) return PPM_EINVAL;
    if (df_arena && !dfp) return PPM_EINVAL;
    int m = 0;
    if (df_arena) {
        m = df_half_width(dfp->A, jobs_host[0].scan.dz);
        if (m < 1) return PPM_EINVAL;
        if (m > kMaxDfHalfWidth) return PPM_EUNSUPPORTED;
    }
    bool wide = false;
    for (int i = 0; i < n_mol; ++i) {
        if ((st = check_grid(&mols_host[i].grid)) != PPM_OK) return st;
        if (scan_grid_wide(mols_host[i].grid.n[0], mols_host[i].grid.n[1], mols_host[i].grid.n[2],
                           16.0))
            wide = true;
    }
    long long nfz = 0, ndf = 0, tiles = 0;
    int max_nz = 0;
    for (int j = 0; j < n_jobs; ++j) {
        const ppm_batch_scan &J = jobs_host[j];
        if (J.mol < 0 || J.mol >= n_mol) return PPM_EINVAL;
        if ((st = check_probe(&J.probe)) != PPM_OK) return st;
        if (!same_probe_lj(J.probe, jobs_host[0].probe)) return PPM_EINVAL;
        if ((st = check_scan(&J.scan)) != PPM_OK) return st;
        if (J.fz_offset != nfz || J.tile_begin != tiles) return PPM_EINVAL;   // not planned
        if (df_arena) {
            if (J.scan.dz != jobs_host[0].scan.dz) return PPM_EUNSUPPORTED;
            if (J.scan.nz < 2 * m + 1) return PPM_EINVAL;
            if (J.df_offset != ndf) return PPM_EINVAL;
            ndf += (long long)J.scan.nx * J.scan.ny * (J.scan.nz - 2 * m);
        }
        if (J.scan.nz > max_nz) max_nz = J.scan.nz;
        nfz += (long long)J.scan.nx * J.scan.ny * J.scan.nz;
        tiles += scan_tile_count(J.scan.nx, J.scan.ny);
    }
    if (df_arena && max_nz > kMaxScanLdsHeights && !fz_arena) return PPM_EUNSUPPORTED;
    ScanArgs proto = make_scan_args(&mols_host[jobs_host[0].mol].grid, &jobs_host[0].probe, fire,
                                    &jobs_host[0].scan);
    DfWeights W;
    memset(&W, 0, sizeof(W));
    proto.m = 0;
    if (df_arena) {
        if ((st = df_weights(dfp, jobs_host[0].scan.dz, m, &W)) != PPM_OK) return st;
        proto.m = m;
    }
    return hip_status(launch_relaxed_scan_batch(proto, W, mols_dev, jobs_dev, n_jobs, tiles,
                                                max_nz, wide,
                                                reinterpret_cast<const float4 *>(ff_arena),
                                                fz_arena, df_arena, (hipStream_t)stream));
}

ppm_status ppm_lateral_stiffness(const ppm_grid *grid, const float *ff, const ppm_probe *probe,
                                 const ppm_scan *scan, const float *pp, float *k_out,
                                 void *stream)
{
    ppm_status st;
    if ((st = check_grid(grid)) != PPM_OK) return st;
    if ((st = check_probe(probe)) != PPM_OK) return st;
    if ((st = check_scan(scan)) != PPM_OK) return st;
    if (!ff || !pp || !k_out) return PPM_EINVAL;
    ScanArgs a = make_scan_args(grid, probe, nullptr, scan);
    return hip_status(launch_lateral_stiffness(a, reinterpret_cast<const float4 *>(ff),
                                               reinterpret_cast<const float4 *>(pp), k_out,
                                               (hipStream_t)stream));
}

static ppm_status hartree_plans(const ppm_grid *grid, FftPlan plans[3])
{
    ppm_status st;
    if ((st = check_grid(grid)) != PPM_OK) return st;
    for (int i = 0; i < 3; ++i)
        if (!fft_plan(grid->n[i], &plans[i])) return PPM_EUNSUPPORTED;
    return PPM_OK;
}

size_t ppm_hartree_workspace_bytes(const ppm_grid *grid)
{
    FftPlan plans[3];
    if (hartree_plans(grid, plans) != PPM_OK) return 0;
    const size_t N = (size_t)grid->n[0] * grid->n[1] * grid->n[2];
    return 3 * align256(N * 16) + align256(hartree_scratch_bytes());
}

ppm_status ppm_tip_density(const ppm_grid *grid, double q_pp, double q_zz, double sigma,
                           float *rho, void *stream)
{
    ppm_status st;
    if ((st = check_grid(grid)) != PPM_OK) return st;
    if (!rho || !(sigma > 0.0) || !isfinite(sigma) || !isfinite(q_pp) || !isfinite(q_zz))
        return PPM_EINVAL;
    return hip_status(launch_tip_density(grid->n[0], grid->n[1], grid->n[2], grid->step[0],
                                         grid->step[1], grid->step[2], q_pp, q_zz, sigma, rho,
                                         (hipStream_t)stream));
}

ppm_status ppm_hartree_ff(const ppm_grid *grid, const float *V, const float *rho,
                          int32_t accumulate, float *ff, void *workspace,
                          size_t workspace_bytes, void *stream)
{
    FftPlan plans[3];
    ppm_status st;
    if ((st = hartree_plans(grid, plans)) != PPM_OK) return st;
    if (!V || !rho || !ff || !workspace) return PPM_EINVAL;
    if (accumulate != 0 && accumulate != 1) return PPM_EINVAL;
    const size_t N = (size_t)grid->n[0] * grid->n[1] * grid->n[2];
    const size_t one = align256(N * 16);
    if (workspace_bytes < 3 * one + align256(hartree_scratch_bytes())) return PPM_EINVAL;
    char *ws = static_cast<char *>(workspace);
    return hip_status(launch_hartree(plans, grid->n[0], grid->n[1], grid->n[2], grid->step[0],
                                     grid->step[1], grid->step[2], V, rho, accumulate,
                                     reinterpret_cast<float4 *>(ff),
                                     reinterpret_cast<double2 *>(ws),
                                     reinterpret_cast<double2 *>(ws + one),
                                     reinterpret_cast<double2 *>(ws + 2 * one), ws + 3 * one,
                                     (hipStream_t)stream));
}

}  // extern "C"
