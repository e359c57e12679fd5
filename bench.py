"""Benchmark of the probe-particle hot path on one MI355X.

One step = one pass of the forward hot path over the paper-scale workload
(60-atom molecule, 240^3 force-field grid, 240x240 tip columns x 100 heights):
force-field build -> relaxed scan with the fused frequency shift.  Inputs are
resident in device memory before timing starts.  The reported value is relaxed
probe positions (pixel x height) per second of the whole step.

Also reported, each timed separately after the main loop:
  * per-kernel durations (HIP events on the launch stream) and the roofline of
    the dominant kernel;
  * the backward/forward time ratio on the differentiation workload (128x128
    tips x 30 heights over the same molecule and grid);
  * the FP64 CPU oracle on the host cores running the same step (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3       # MI355X vector FP32 (packed), published
FLOP_PER_PAIR = 31             # algorithmic FLOP per voxel-atom pair (FMA = 2)
BYTES_PER_EVAL = 96            # 8 corners x (Fx, Fy, Fz) FP32 per force evaluation


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the backward measurement")
    return ap.parse_args()


def _sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel_key, src, launches_bytes_key):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    e = t.get(kernel_key)
    if not e or e.get("source_sha") != _sha(src):
        return None
    return e.get(launches_bytes_key)


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2401_14564_amd as ppm
    from paper_2401_14564_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    w = W.config1()
    atoms = ppm.atoms_to_device(w.atoms)
    nx, ny, nz = w.grid.n
    ff = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=dev)
    m = ppm.df_half_width(w.df.A, w.scan.dz)
    out = dict(fz=torch.empty((w.scan.nz, w.scan.ny, w.scan.nx), dtype=torch.float32, device=dev),
               df=torch.empty((w.scan.nz - 2 * m, w.scan.ny, w.scan.nx), dtype=torch.float32,
                              device=dev))
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        ppm.build_ff(w.grid, w.probe, atoms, out=ff)
        if ev is not None:
            ev[1].record(stream)
        ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=False, pp=False,
                         out=out)
        if ev is not None:
            ev[2].record(stream)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    ff_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    scan_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))

    # FIRE evaluations per launch (deterministic: same inputs, same iterations)
    res = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=True, pp=True)
    iters = res["pp"][..., 3]
    n_eq = w.scan.n_eq
    evals = float(iters.abs().sum().item()) + n_eq
    nonconv = int((iters < 0).sum().item())
    scan_bytes = evals * BYTES_PER_EVAL + n_eq * 4 + (w.scan.nz - 2 * m) * w.scan.nx * w.scan.ny * 4
    scan_gbs = scan_bytes / (scan_ms * 1e-3) / 1e9
    pairs = w.grid.nvox * w.atoms.n
    ff_tflops = pairs * FLOP_PER_PAIR / (ff_ms * 1e-3) / 1e12
    scan_src = ["paper_2401_14564_amd/csrc/relaxed_scan.hip", "paper_2401_14564_amd/csrc/ppm_kernels.h"]
    ff_src = ["paper_2401_14564_amd/csrc/ff_build.hip", "paper_2401_14564_amd/csrc/ppm_kernels.h"]
    dominant = "relaxed_scan" if scan_ms >= ff_ms else "ff_build"
    if dominant == "relaxed_scan":
        roof = {"kernel": "relaxed_scan_kernel", "bound": "hbm", "achieved": round(scan_gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(scan_gbs / HBM_PEAK_GBS, 4),
                "traffic": _traffic("relaxed_scan_c1", scan_src, "hbm_bytes_per_launch")}
    else:
        roof = {"kernel": "ff_build_kernel", "bound": "alu", "achieved": round(ff_tflops, 2),
                "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ff_tflops / FP32_PEAK_TFLOPS, 4),
                "traffic": _traffic("ff_build_c1", ff_src, "hbm_bytes_per_launch")}

    result = {
        "metric": "relaxed-scan PP relaxations/s (force-field build + relaxed scan + fused df)",
        "value": round(n_eq / (ms_per_step * 1e-3), 1),
        "unit": "relaxations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 grid / f64 relaxation",
        "data": "synthetic (seeded 60-atom molecule, random-free tip lattice)",
        "config": {"workload": "paper-scale plain method: 60 atoms, grid 240^3 at 0.1 A, "
                               "scan 240x240 tips x 100 heights, FIRE f_conv 1e-4 eV/A, "
                               "df A=1 A f0=30300 Hz k=1800 N/m",
                   "relaxations_per_step": n_eq, "voxels": w.grid.nvox, "atoms": w.atoms.n},
        "roofline": roof,
        "kernels": {
            "ff_build": {"ms": round(ff_ms, 4), "tflops": round(ff_tflops, 2),
                         "frac_of_fp32_peak": round(ff_tflops / FP32_PEAK_TFLOPS, 4),
                         "traffic": _traffic("ff_build_c1", ff_src, "hbm_bytes_per_launch")},
            "relaxed_scan": {"ms": round(scan_ms, 4), "gather_gbs": round(scan_gbs, 1),
                             "fire_evals_per_relaxation": round(evals / n_eq, 3),
                             "mean_fire_steps": round(float(iters.abs().mean().item()), 3),
                             "not_converged": nonconv,
                             "algorithmic_bytes": int(scan_bytes)},
        },
    }

    if not a.no_extra:
        result["backward"] = _bench_backward(ppm, W, torch)

    if not a.no_cpu:
        result["cpu_baseline"] = _cpu_baseline(w, n_eq)
    print(json.dumps(result), flush=True)


def _bench_backward(ppm, W, torch):
    """bwd/fwd time on the differentiation workload (loss ||df - df_t||^2)."""
    w, target = W.config4()
    dev = torch.device("cuda:0")
    atoms = ppm.atoms_to_device(w.atoms)
    nx, ny, nz = w.grid.n
    ff = torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=dev)
    ppm.build_ff(w.grid, w.probe, target, out=ff)
    df_t = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=False)["df"].clone()
    out = {}

    def fwd():
        ppm.build_ff(w.grid, w.probe, atoms, out=ff)
        return ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=False, out=out)

    res = fwd()
    gdf = 2.0 * (res["df"] - df_t)
    ws = torch.empty(int(ppm._lib.lib().ppm_backward_workspace_bytes(
        ppm._lib.scan_struct(w.scan), w.atoms.n)), dtype=torch.uint8, device=dev)

    def bwd():
        return ppm.relaxed_scan_backward(w.grid, ff, w.probe, w.scan, w.df, atoms, res["pp"], gdf,
                                         workspace=ws)

    for _ in range(3):
        fwd()
        bwd()
    torch.cuda.synchronize()
    n = 10
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    tf, tb = [], []
    for _ in range(n):
        e[0].record()
        fwd()
        e[1].record()
        bwd()
        e[2].record()
        torch.cuda.synchronize()
        tf.append(e[0].elapsed_time(e[1]))
        tb.append(e[1].elapsed_time(e[2]))
    import numpy as np
    fwd_ms, bwd_ms = float(np.median(tf)), float(np.median(tb))
    return {"workload": "differentiation: 60 atoms, grid 240^3, scan 128x128 x 30 heights "
                        "(20 df outputs), loss ||df - df_target||^2",
            "fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4),
            "bwd_over_fwd": round(bwd_ms / fwd_ms, 4)}


def _cpu_baseline(w, n_eq):
    """The FP64 oracle, as it stands, on the host cores: the same step (full
    force-field grid, then a sampled set of tip columns at the same FIRE
    settings, no Newton polish), scaled to relaxations/s of the whole step."""
    import numpy as np
    import oracle as orc
    threads = orc.num_threads()
    t0 = time.perf_counter()
    ffo = orc.build_ff(w.grid, w.probe, w.atoms)
    t1 = time.perf_counter()
    rng = np.random.default_rng(12345)
    ncol = w.scan.nx * w.scan.ny
    nsamp = 5760                                   # 10% of the tip columns
    sel = rng.choice(ncol, size=nsamp, replace=False)
    cols = np.stack([sel % w.scan.nx, sel // w.scan.nx], axis=1).astype(np.int32)
    t2 = time.perf_counter()
    res = orc.relaxed_scan(w.grid, ffo, w.probe, w.fire, w.scan, cols=cols)
    fzs = res["fz"].T
    orc.df(fzs, w.scan.dz, w.df)
    t3 = time.perf_counter()
    t_step = (t1 - t0) + (t3 - t2) * (ncol / nsamp)
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(n_eq / t_step, 1), "unit": "relaxations/s", "cores": threads,
            "kind": "oracle",
            "sample": f"full force-field grid ({t1 - t0:.2f} s) + relaxed scan of {nsamp} of "
                      f"{ncol} tip columns ({t3 - t2:.2f} s), scaled to the whole step "
                      f"({t_step:.2f} s); FP64, no polish; cpu: {cpu}, os.cpu_count() "
                      f"{os.cpu_count()}"}


if __name__ == "__main__":
    main()
