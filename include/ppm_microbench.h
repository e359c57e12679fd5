/*
 * ppm_microbench.h -- measurement kernels for the rooflines of the two hot
 * kernels (libppm_microbench.so).  Not part of the probe-particle library.
 *
 * ppm_mb_gather_band_bytes: size of the band the gather benchmark reads (a
 *   float4 array [32][64][64], 2 MiB: resident in each XCD's 4 MiB L2).
 * ppm_mb_gather: `blocks` blocks of 256 lanes; every lane performs `iters`
 *   steps, each loading the eight float4 corners of one trilinear cell of the
 *   band (128 bytes per lane-step), at cell positions drawn from a
 *   counter-based hash of (seed, lane, step).  coherent != 0: a wave's lanes
 *   are 16 x 4 neighbouring columns that drift in z (the relaxed scan's
 *   pattern); 0: uniformly random cells.  band: device, initialised by the
 *   caller; out: device, blocks * 256 float4 (sums of the loads, written so
 *   that no load is dead).  Returns 0, -1 for bad arguments, -3 if the launch
 *   failed.  Enqueued on `stream`.
 * ppm_mb_pair: `blocks` blocks of 256 threads, each thread evaluating the
 *   force-field build's LJ + Coulomb pair body (periodic != 0: with the cutoff
 *   mask and shifted-force terms) for `reps` x 256 atoms at 8 voxels, with the
 *   atoms in LDS and no global traffic.  out: device, blocks * 256 floats.
 *   Returns as ppm_mb_gather.
 * ppm_mb_issue: `blocks` blocks of 256 lanes, each lane running `iters` steps
 *   of eight independent chains of one instruction kind: 0 = FP32 FMA with
 *   vector-register operands only, 1 = FP32 FMA with one scalar-register
 *   (wave-uniform) factor, 2 = FP64 FMA with vector-register operands, 3 = FP32
 *   reciprocal square root (8 x iters instructions per lane).  out: device,
 *   blocks * 256 floats.  Returns as ppm_mb_gather (-1 also for an unknown kind).
 */
#ifndef PPM_MICROBENCH_H
#define PPM_MICROBENCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

size_t ppm_mb_gather_band_bytes(void);
int ppm_mb_gather(const float *band, int coherent, int blocks, int iters, uint32_t seed,
                  float *out, void *stream);
int ppm_mb_pair(int periodic, int blocks, int reps, float *out, void *stream);
int ppm_mb_issue(int kind, int blocks, int iters, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PPM_MICROBENCH_H */
