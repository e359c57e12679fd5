"""Benchmark of the probe-particle hot path on one MI355X.

One step = one pass of the forward hot path over the large periodic sample
(400-atom flake on a 1,200-atom two-layer slab, periodic in x and y with a
12 A shifted-force cutoff, 400x400x300 force-field grid, 400x400 tip columns x
120 heights): force-field build -> relaxed scan with the Fz readout and the
frequency shift.  Inputs are resident in device memory before timing starts.  The
reported value is relaxed probe positions (pixel x height) per second of the
whole job.  By default the two stages run in order on one stream; --pipeline
overlaps the force-field build of step i+1 with the scan of step i on a second
stream.

Also reported, each timed separately after the main loop:
  * per-kernel durations (HIP events on the launch stream), the roofline of the
    dominant kernel against the published peak, and each hot kernel against a
    ceiling measured on this GPU by the microbenchmarks of
    libppm_microbench.so (8-corner gathers from an L2-resident band; the
    force-field pair body without memory traffic);
  * the paper-scale open workload (60 atoms, 240^3 grid, 240x240 x 100), in
    order and pipelined;
  * the backward/forward time ratio on the differentiation workload (128x128
    tips x 30 heights over the paper-scale molecule and grid);
  * 256 molecules x 3 probe stiffnesses batched against per-molecule loops;
  * the quadrupolar probe, grid-electrostatics, lateral-stiffness and tricubic
    rows on the paper-scale workload;
  * the FP64 CPU oracle on the host cores on a bounded sample of the headline
    step (cpu_baseline).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extra]
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3       # MI355X vector FP32 (packed), published
FLOP_PER_PAIR = 31             # algorithmic FLOP per voxel-atom pair (FMA = 2), open sample
FLOP_PER_PAIR_SF = 37          # periodic sample: + rho = r2/rho (1), ec - C (1), fc rho + . (2),
                               # the force's -fc/rho (2) of the shifted-force cutoff
BYTES_PER_EVAL = 96            # 8 corners x (Fx, Fy, Fz) FP32 per force evaluation


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the backward measurement")
    ap.add_argument("--pipeline", action="store_true",
                    help="overlap step i+1's force-field build with step i's scan on a second "
                         "stream (double-buffered grid)")
    ap.add_argument("--kernels-once", action="store_true",
                    help="for rocprofv3 --pmc: a 1 GiB copy (counter calibration), then one "
                         "launch of each hot kernel on the large periodic workload (tuned "
                         "shapes) and on the paper-scale one")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc output folders (FETCH_SIZE, WRITE_SIZE) "
                         "into profiles/traffic.json")
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR",
                    help="print the mean per-dispatch counters of the force-field and scan "
                         "kernels in rocprofv3 --pmc output folders as a markdown table")
    return ap.parse_args()


_FF_SRC = ["paper_2401_14564_amd/csrc/ff_build.hip", "paper_2401_14564_amd/csrc/ppm_kernels.h"]
_SCAN_SRC = ["paper_2401_14564_amd/csrc/relaxed_scan.hip",
             "paper_2401_14564_amd/csrc/ppm_kernels.h", "paper_2401_14564_amd/csrc/ppm_device.h"]
CALIB_BYTES = 1 << 30


def _ff_kernel(tuning, periodic):
    """rocprofv3 name (template part) of the force-field kernel a build launches."""
    nzb = getattr(tuning, "ff_nzb", 0) or 8
    return f"ff_build_kernel<16, 16, {nzb}, {'true' if periodic else 'false'}, false, false>"


def _scan_kernel(tuning, periodic):
    """Name prefix of the scan kernel of a launch with a frequency shift and an
    fz output, the work-group shape of `tuning` (Fz staged in LDS, or
    with 8 x 8 work-groups and scan_fz_direct written straight to fz)."""
    t = getattr(tuning, "scan_tile", 0) or 16
    stage = "false" if t == 8 and getattr(tuning, "scan_fz_direct", 0) else "true"
    return f"relaxed_scan_kernel<{t}, {t}, {stage}, false, 0, {1 if periodic else 0},"


def kernels_once():
    """For rocprofv3 --pmc: a 1 GiB copy (counter calibration), then the
    autotuner and one launch of the force-field build and of the scan with its
    choice (as the timed steps run them) on the large periodic workload, one of
    each at the default shapes on the paper-scale workload, and one forward and
    backward on the differentiation workload."""
    import torch
    import paper_2401_14564_amd as ppm
    from paper_2401_14564_amd import workloads as W
    dev = torch.device("cuda:0")
    a = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)                        # reads and writes CALIB_BYTES
    torch.cuda.synchronize()
    del a, b
    for w, tune in ((W.config2(), True), (W.config1(), False)):
        ff = ppm.build_ff(w.grid, w.probe, w.atoms)
        t = None
        if tune:
            t, _ = ppm.tune_build_ff(w.grid, w.probe, w.atoms, out=ff)
            t, _, _ = ppm.tune_relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df,
                                            fz=True, pp=False, tuning=t)
        torch.cuda.synchronize()
        ppm.build_ff(w.grid, w.probe, w.atoms, out=ff, tuning=t)
        torch.cuda.synchronize()
        ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=True, pp=False,
                         tuning=t)
        torch.cuda.synchronize()
        print(w.name, "shapes", t, flush=True)
        del ff
    # one backward on the differentiation workload (loss ||df - df_target||^2)
    w, target = W.config4()
    atoms = ppm.atoms_to_device(w.atoms)
    # (its forward at other launch shapes than the paper-scale launches above,
    # so that every kernel name in the counter tables covers one workload)
    t4 = ppm.Tuning(6, 8)
    ff = ppm.build_ff(w.grid, w.probe, target, tuning=t4)
    df_t = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=False,
                            tuning=t4)["df"].clone()
    ppm.build_ff(w.grid, w.probe, atoms, out=ff, tuning=t4)
    res = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df, fz=False, tuning=t4)
    torch.cuda.synchronize()
    ppm.relaxed_scan_backward(w.grid, ff, w.probe, w.scan, w.df, atoms, res["pp"],
                              2.0 * (res["df"] - df_t))
    torch.cuda.synchronize()
    print(w.name, "backward", flush=True)
    print("kernels-once done", flush=True)


def _read_pmc(folder, counter):
    """{kernel name: [values per dispatch]} from a rocprofv3 counter-collection csv."""
    import csv
    import glob
    rows = {}
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {folder}")
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                rows.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return rows


# the library's kernels in rocprofv3 kernel names (template arguments kept)
KERNEL_NAME_RE = (r"((ff_build_kernel|relaxed_scan_kernel|atom_scatter_kernel|"
                  r"adjoint_solve_kernel)<[^>]*>|reduce_kernel\(double)")


def summarize_pmc(fetch_dir, write_dir):
    """profiles/traffic.json: HBM bytes per launch of every force-field, scan and
    backward kernel in the two counter runs, scaled by what the counters read for the
    known copy, with the hashes of the sources they were taken on."""
    import re
    out = {"calibration": f"torch copy of {CALIB_BYTES} bytes (reads and writes that many)",
           "units": "bytes per launch, counter KiB x 1024 x (known copy bytes / copy reading)",
           "ff_source_sha": _sha(_FF_SRC), "scan_source_sha": _sha(_SCAN_SRC), "kernels": {}}
    for counter, folder in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _read_pmc(folder, counter)
        copy = [v for k, v in rows.items() if "copy" in k.lower() or "elementwise" in k.lower()]
        calib_kib = max(max(v) for v in copy) if copy else None
        factor = (CALIB_BYTES / 1024.0) / calib_kib if calib_kib else 1.0
        out[f"{counter}_copy_reading_kib"] = calib_kib
        out[f"{counter}_scale"] = factor
        for k, vs in rows.items():
            m = re.search(KERNEL_NAME_RE, k)
            if not m:
                continue
            e = out["kernels"].setdefault(m.group(1), {"dispatches": len(vs)})
            e[counter.lower() + "_bytes"] = float(np.mean(vs)) * 1024.0 * factor
    for e in out["kernels"].values():
        if "fetch_size_bytes" in e and "write_size_bytes" in e:
            e["hbm_bytes_per_launch"] = e["fetch_size_bytes"] + e["write_size_bytes"]
    out["commands"] = [
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d $REPO/{fetch_dir.rstrip('/')} -o pmc "
        "-- python3 $REPO/bench.py --kernels-once",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d $REPO/{write_dir.rstrip('/')} -o pmc "
        "-- python3 $REPO/bench.py --kernels-once",
        f"python3 bench.py --summarize-pmc {fetch_dir} {write_dir}"]
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def summarize_counters(folders):
    """Markdown table of the mean per-dispatch value of every counter in the
    given rocprofv3 --pmc output folders, for the force-field, scan and
    backward kernels."""
    import csv
    import glob
    import re
    table = {}
    for folder in folders:
        for fn in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as f:
                for r in csv.DictReader(f):
                    m = re.search(KERNEL_NAME_RE, r["Kernel_Name"])
                    if not m:
                        continue
                    table.setdefault(m.group(1), {}).setdefault(r["Counter_Name"], []).append(
                        float(r["Counter_Value"]))
    counters = sorted({c for v in table.values() for c in v})
    lines = ["| kernel | " + " | ".join(counters) + " |",
             "|---|" + "---|" * len(counters)]
    for k, v in table.items():
        lines.append(f"| `{k}` | " + " | ".join(
            f"{np.mean(v[c]):.4g}" if c in v else "" for c in counters) + " |")
    print("\n".join(lines))


def _sha(paths):
    """Hash of the code in the given sources, comments and whitespace removed
    (a counter summary stays valid across comment-only edits)."""
    import re
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def _traffic(name_prefix, src_key, src):
    """HBM bytes per launch of the kernel whose name starts with name_prefix,
    from the committed rocprofv3 counter summary, if it was taken on the
    current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get(src_key) != _sha(src):
        return None
    for name, e in t.get("kernels", {}).items():
        if name.startswith(name_prefix):
            return e.get("hbm_bytes_per_launch")
    return None


def _run_steps(ppm, torch, w, atoms, ffs, outs, pipeline, steps, warmup, tuning=None):
    """Time `steps` forward steps (force-field build -> relaxed scan with the Fz
    readout and the frequency shift) after `warmup` untimed ones.  Returns (ms per step, mean
    build ms, mean scan ms), the kernel times from HIP events on the streams
    the kernels run on."""
    if pipeline:
        s_ff, s_scan = torch.cuda.Stream(), torch.cuda.Stream()
    else:
        s_ff = s_scan = torch.cuda.current_stream()
    nbuf = len(ffs)
    ff_done = [torch.cuda.Event() for _ in range(nbuf)]
    scan_done = [torch.cuda.Event() for _ in range(nbuf)]
    for e in scan_done:
        e.record(s_scan)

    def step(i, ev=None):
        b = i % nbuf
        with torch.cuda.stream(s_ff):
            s_ff.wait_event(scan_done[b])          # buffer b is free again
            if ev is not None:
                ev[0].record(s_ff)
            ppm.build_ff(w.grid, w.probe, atoms, out=ffs[b], tuning=tuning)
            if ev is not None:
                ev[1].record(s_ff)
            ff_done[b].record(s_ff)
        with torch.cuda.stream(s_scan):
            s_scan.wait_event(ff_done[b])
            if ev is not None:
                ev[2].record(s_scan)
            ppm.relaxed_scan(w.grid, ffs[b], w.probe, w.fire, w.scan, dfp=w.df, fz=True,
                             pp=False, out=outs[b], tuning=tuning)
            if ev is not None:
                ev[3].record(s_scan)
            scan_done[b].record(s_scan)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(i, evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return ((t1 - t0) * 1e3 / steps,
            float(np.mean([e[0].elapsed_time(e[1]) for e in evs])),
            float(np.mean([e[2].elapsed_time(e[3]) for e in evs])))


def _buffers(ppm, torch, w, nbuf):
    dev = torch.device("cuda:0")
    nx, ny, nz = w.grid.n
    m = ppm.df_half_width(w.df.A, w.scan.dz)
    ffs = [torch.empty((nz, ny, nx, 4), dtype=torch.float32, device=dev) for _ in range(nbuf)]
    outs = [dict(df=torch.empty((w.scan.nz - 2 * m, w.scan.ny, w.scan.nx), dtype=torch.float32,
                                device=dev),
                 fz=torch.empty((w.scan.nz, w.scan.ny, w.scan.nx), dtype=torch.float32,
                                device=dev)) for _ in range(nbuf)]
    return ffs, outs, m


def _scan_stats(ppm, torch, w, ff, tile=16):
    """FIRE evaluations of one scan launch (deterministic: same inputs, same
    iterations, the same for every launch shape) and the critical path: a
    64-lane wave covers 4 rows of 16 columns in 16 x 16-column blocks and
    8 x 8 columns in 8 x 8 blocks, and lasts as long as its slowest column."""
    res = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=None, fz=False, pp=True)
    it = res["pp"][..., 3]
    n_eq = w.scan.n_eq
    evals = float(it.abs().sum().item()) + n_eq
    per_col = (it.abs().sum(0) + w.scan.nz).cpu().numpy()            # [ny, nx]
    ny, nx = per_col.shape
    wy, wx = (8, 8) if tile == 8 else (4, 16)
    pc = np.zeros(((ny + wy - 1) // wy * wy, (nx + wx - 1) // wx * wx))
    pc[:ny, :nx] = per_col
    wave = pc.reshape(pc.shape[0] // wy, wy, pc.shape[1] // wx, wx).max(axis=(1, 3))
    out = dict(evals=evals, not_converged=int((it < 0).sum().item()),
               mean_steps=float(it.abs().mean().item()), max_steps=int(it.abs().max().item()),
               slowest_wave_evals=float(wave.max()), mean_wave_evals=float(wave.mean()))
    del res
    return out


def main():
    a = _args()
    if a.summarize_pmc:
        summarize_pmc(*a.summarize_pmc)
        return
    if a.summarize_counters:
        summarize_counters(a.summarize_counters)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if a.kernels_once:
        kernels_once()
        return
    import torch

    import paper_2401_14564_amd as ppm
    from paper_2401_14564_amd import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # headline: the large periodic sample (the largest single-GPU workload)
    w = W.config2()
    atoms = ppm.atoms_to_device(w.atoms)
    ffs, outs, m = _buffers(ppm, torch, w, 2 if a.pipeline else 1)
    # launch shapes from the autotuner, on these inputs, before the timed steps
    tuning, ff_tune_ms = ppm.tune_build_ff(w.grid, w.probe, atoms, out=ffs[0])
    tuning, scan_tune_ms, _ = ppm.tune_relaxed_scan(w.grid, ffs[0], w.probe, w.fire, w.scan,
                                                    dfp=w.df, fz=True, pp=False, out=outs[0],
                                                    tuning=tuning)
    ms_per_step, ff_ms, scan_ms = _run_steps(ppm, torch, w, atoms, ffs, outs, a.pipeline,
                                             a.steps, a.warmup, tuning)
    n_eq = w.scan.n_eq
    st = _scan_stats(ppm, torch, w, ffs[0], tuning.scan_tile)
    pairs = _pairs_within_cutoff(w)
    ff_tflops = pairs * FLOP_PER_PAIR_SF / (ff_ms * 1e-3) / 1e12
    n_df = (w.scan.nz - 2 * m) * w.scan.nx * w.scan.ny
    # algorithmic bytes of the scan launch as timed: 96 B per force evaluation
    # plus the Fz and frequency-shift outputs (the probe state is not written)
    scan_bytes = st["evals"] * BYTES_PER_EVAL + (n_eq + n_df) * 4
    scan_gbs = scan_bytes / (scan_ms * 1e-3) / 1e9
    mb = _microbench(torch)
    ff_name, scan_name = _ff_kernel(tuning, True), _scan_kernel(tuning, True)
    ff_roof = {"kernel": ff_name, "bound": "alu",
               "achieved": round(ff_tflops, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
               "frac": round(ff_tflops / FP32_PEAK_TFLOPS, 4),
               "traffic": _traffic(ff_name, "ff_source_sha", _FF_SRC)}
    scan_l2 = mb["gather_coherent_gbs"] * BYTES_PER_EVAL / MB_BYTES_PER_GATHER
    scan_roof = {"kernel": scan_name + "...>", "bound": "hbm", "achieved": round(scan_gbs, 1),
                 "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(scan_gbs / HBM_PEAK_GBS, 4),
                 "traffic": _traffic(scan_name, "scan_source_sha", _SCAN_SRC)}
    roof = ff_roof if ff_ms >= scan_ms else scan_roof

    result = {
        "metric": "relaxed-scan PP relaxations/s (force-field build + relaxed scan + df)",
        "value": round(n_eq / (ms_per_step * 1e-3), 1),
        "unit": "relaxations/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 grid and interpolation / f64 relaxation",
        "data": "synthetic (seeded 400-atom flake on a 1,200-atom slab, random-free tip lattice)",
        "config": {"workload": "large periodic sample: 1,600 atoms, periodic xy, 12 A "
                               "shifted-force cutoff, grid 400x400x300 at 0.1 A, scan 400x400 "
                               "tips x 120 heights, FIRE f_conv 1e-4 eV/A, df A=1 A f0=30300 Hz "
                               "k=1800 N/m",
                   "pipelining": ("step i+1's force-field build overlaps step i's scan on a "
                                  "second stream (double-buffered grid)") if a.pipeline else
                                 "none: build then scan, in order, on one stream",
                   "outputs": "Fz (the tip-force readout) at every relaxed point and the frequency "
                              "shift; probe state not written",
                   "relaxations_per_step": n_eq, "voxels": w.grid.nvox, "atoms": w.atoms.n,
                   "launch_shapes": {"ff_voxels_per_thread": tuning.ff_nzb,
                                     "scan_tile": f"{tuning.scan_tile}x{tuning.scan_tile}",
                                     "scan_fz_direct": tuning.scan_fz_direct,
                                     "autotuner_ms": {"ff_build": ff_tune_ms,
                                                      "relaxed_scan": scan_tune_ms}}},
        "roofline": roof,
        "kernels": {
            "ff_build": {"ms": round(ff_ms, 4), "pairs_within_cutoff": pairs,
                         "flop_per_pair": FLOP_PER_PAIR_SF, "tflops": round(ff_tflops, 2),
                         "frac_of_fp32_peak": round(ff_tflops / FP32_PEAK_TFLOPS, 4),
                         "measured_pair_ceiling_tflops": mb["pair_periodic_tflops"],
                         "frac_of_measured_ceiling": round(ff_tflops / mb["pair_periodic_tflops"],
                                                           4),
                         "roofline": ff_roof},
            "relaxed_scan": {"ms": round(scan_ms, 4),
                             "fire_evals_per_relaxation": round(st["evals"] / n_eq, 3),
                             "mean_fire_steps": round(st["mean_steps"], 3),
                             "max_fire_steps": st["max_steps"],
                             "not_converged": st["not_converged"],
                             "algorithmic_bytes": int(scan_bytes),
                             "gather_gbs": round(scan_gbs, 1),
                             "measured_gather_ceiling_gbs": round(scan_l2, 1),
                             "frac_of_measured_gather_ceiling": round(scan_gbs / scan_l2, 4),
                             "bound_note": "latency: one wave per column group; the kernel "
                                           "lasts as long as its slowest wave",
                             "slowest_wave_evals": int(st["slowest_wave_evals"]),
                             "mean_wave_evals": round(st["mean_wave_evals"], 1),
                             "us_per_eval_on_critical_path": round(
                                 scan_ms * 1e3 / st["slowest_wave_evals"], 4),
                             "roofline": scan_roof},
        },
        "microbench": mb,
    }
    del ffs, outs
    torch.cuda.empty_cache()

    if not a.no_extra:
        other = not a.pipeline
        ffs, outs, _ = _buffers(ppm, torch, w, 2 if other else 1)
        o_ms, o_ff, o_scan = _run_steps(ppm, torch, w, atoms, ffs, outs, other, a.steps, a.warmup,
                                        tuning)
        result["pipelined" if other else "sequential"] = {
            "pipelining": ("step i+1's force-field build overlaps step i's scan on a second "
                           "stream (double-buffered grid)") if other else
                          "none: build then scan, in order, on one stream",
            "ms_per_step": round(o_ms, 4),
            "relaxations_per_s": round(n_eq / (o_ms * 1e-3), 1),
            "ff_ms": round(o_ff, 4), "scan_ms": round(o_scan, 4)}
        del ffs, outs
        torch.cuda.empty_cache()
        result["paper_scale"] = _bench_paper_scale(ppm, W, torch, a)
        result["backward"] = _bench_backward(ppm, W, torch)
        result["batched"] = _bench_batch(ppm, W, torch, mb=mb)
        result["next_rows"] = _bench_next_rows(ppm, W, torch)

    if not a.no_cpu:
        result["cpu_baseline"] = _cpu_baseline(w, n_eq)
    print(json.dumps(result), flush=True)


MB_BYTES_PER_GATHER = 128      # the gather microbenchmark loads 8 float4 corners


def _microbench(torch):
    """Ceilings measured on this GPU (libppm_microbench.so): 8-corner float4
    gathers from an L2-resident band (the scan's access pattern, coherent and
    random), and the force-field pair body with no memory traffic (open and
    periodic/shifted-force).  Median of 5 launches each."""
    import ctypes as ct
    path = os.path.join(ROOT, "paper_2401_14564_amd", "libppm_microbench.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build with `python -m paper_2401_14564_amd.build`")
    L = ct.CDLL(path)
    L.ppm_mb_gather_band_bytes.restype = ct.c_size_t
    L.ppm_mb_gather.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_uint32,
                                ct.c_void_p, ct.c_void_p]
    L.ppm_mb_pair.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p]
    L.ppm_mb_issue.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p]
    dev = torch.device("cuda:0")
    band = torch.rand(int(L.ppm_mb_gather_band_bytes()) // 4, device=dev)
    gb, gi = 8192, 64
    gout = torch.empty(gb * 256 * 4, device=dev)
    pb, pr = 2048, 4
    pout = torch.empty(pb * 256, device=dev)
    stream = torch.cuda.current_stream().cuda_stream

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        ts = []
        for _ in range(5):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    out = {"gather_band_bytes": int(band.numel() * 4)}
    for coh, key in ((1, "coherent"), (0, "random")):
        ms = timed(lambda: L.ppm_mb_gather(ct.c_void_p(band.data_ptr()), coh, gb, gi, 12345,
                                            ct.c_void_p(gout.data_ptr()), ct.c_void_p(stream)))
        out[f"gather_{key}_gbs"] = round(gb * 256 * gi * MB_BYTES_PER_GATHER / (ms * 1e-3) / 1e9, 1)
    pairs = pb * 256 * 8 * 256 * pr
    for per, key, flop in ((0, "open", FLOP_PER_PAIR), (1, "periodic", FLOP_PER_PAIR_SF)):
        ms = timed(lambda: L.ppm_mb_pair(per, pb, pr, ct.c_void_p(pout.data_ptr()),
                                          ct.c_void_p(stream)))
        out[f"pair_{key}_tflops"] = round(pairs * flop / (ms * 1e-3) / 1e12, 2)
    # VALU issue rate per instruction kind, in lanes per SIMD and cycle at the
    # 2.4 GHz the published peaks assume (16 = one wave64 instruction per 4 cycles)
    ib, ii = 2048, 4096
    lanes = ib * 256 * ii * 8
    issue = {}
    for kind, key in ((0, "fp32_fma_vector_operands"), (1, "fp32_fma_scalar_factor"),
                      (2, "fp64_fma_vector_operands"), (3, "fp32_rsq")):
        ms = timed(lambda: L.ppm_mb_issue(kind, ib, ii, ct.c_void_p(pout.data_ptr()),
                                           ct.c_void_p(stream)))
        issue[key] = round(lanes / (ms * 1e-3) / (1024 * 2.4e9), 1)
    out["valu_issue_lanes_per_simd_cycle"] = issue
    out["fp32_fma_vector_tflops"] = round(issue["fp32_fma_vector_operands"] * 2 * 1024 * 2.4e9
                                          / 1e12, 1)
    out["note"] = ("gather: 128 B per lane-step (8 float4 corners), 2 MiB band; pair: "
                   f"{FLOP_PER_PAIR} (open) / {FLOP_PER_PAIR_SF} (periodic) algorithmic FLOP per "
                   "pair, 8 voxels per thread, atoms in LDS, no global traffic")
    return out


def _bench_paper_scale(ppm, W, torch, a):
    """The paper-scale open workload (60 atoms, 240^3 grid, 240x240 x 100
    heights), sequential and pipelined."""
    w = W.config1()
    atoms = ppm.atoms_to_device(w.atoms)
    ffs, outs, m = _buffers(ppm, torch, w, 2)
    seq = _run_steps(ppm, torch, w, atoms, ffs[:1], outs[:1], False, a.steps, a.warmup)
    pip = _run_steps(ppm, torch, w, atoms, ffs, outs, True, a.steps, a.warmup)
    st = _scan_stats(ppm, torch, w, ffs[0])
    n_eq = w.scan.n_eq
    n_df = (w.scan.nz - 2 * m) * w.scan.nx * w.scan.ny
    pairs = w.grid.nvox * w.atoms.n
    scan_bytes = st["evals"] * BYTES_PER_EVAL + (n_eq + n_df) * 4
    return {"workload": "paper-scale plain method: 60 atoms, grid 240^3 at 0.1 A (open), scan "
                        "240x240 tips x 100 heights",
            "ms_per_step": round(seq[0], 4), "relaxations_per_s": round(n_eq / (seq[0] * 1e-3), 1),
            "ff_ms": round(seq[1], 4), "scan_ms": round(seq[2], 4),
            "ff_tflops": round(pairs * FLOP_PER_PAIR / (seq[1] * 1e-3) / 1e12, 2),
            "scan_gather_gbs": round(scan_bytes / (seq[2] * 1e-3) / 1e9, 1),
            "fire_evals_per_relaxation": round(st["evals"] / n_eq, 3),
            "mean_fire_steps": round(st["mean_steps"], 3),
            "slowest_wave_evals": int(st["slowest_wave_evals"]),
            "pipelined": {"ms_per_step": round(pip[0], 4),
                          "relaxations_per_s": round(n_eq / (pip[0] * 1e-3), 1),
                          "ff_ms": round(pip[1], 4), "scan_ms": round(pip[2], 4)}}


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
    fwd_ms, bwd_ms = float(np.median(tf)), float(np.median(tb))
    return {"workload": "differentiation: 60 atoms, grid 240^3, scan 128x128 x 30 heights "
                        "(20 df outputs), loss ||df - df_target||^2",
            "fwd_ms": round(fwd_ms, 4), "bwd_ms": round(bwd_ms, 4),
            "bwd_over_fwd": round(bwd_ms / fwd_ms, 4)}


def _bench_batch(ppm, W, torch, n_mol=256, mb=None):
    """Frequency-shift stacks per second for 256 molecules x 3 lateral
    stiffnesses: one captured HIP graph (batched force-field launch + batched
    scan launch) against a plain per-molecule loop of build_ff + 3 scans on one
    stream (no per-molecule synchronisation)."""
    dev = torch.device("cuda:0")
    ws = W.config3(n_mol)
    mols = [(w.atoms, w.grid) for w in ws]
    jobs = []
    for i, w in enumerate(ws):
        for k in W.C3_K_LAT_N_PER_M:
            jobs.append((i, dataclasses.replace(w.probe, k_lat=(k * W.N_PER_M, k * W.N_PER_M)),
                         w.scan))
    bp = ppm.BatchPipeline.tuned(mols, jobs, ws[0].probe, ws[0].fire, ws[0].df)
    # eager stage times
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    bp.run()
    torch.cuda.synchronize()
    e[0].record()
    bp.build_ff()
    e[1].record()
    bp.scan()
    e[2].record()
    torch.cuda.synchronize()
    ff_ms, scan_ms = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    bp.capture()
    tb = []
    for _ in range(3):
        torch.cuda.synchronize()
        e[0].record()
        bp.replay()
        e[1].record()
        torch.cuda.synchronize()
        tb.append(e[0].elapsed_time(e[1]))
    batched_ms = float(np.median(tb))
    # plain loop
    maxvox = max(w.grid.nvox for w in ws)
    ffbuf = torch.empty(maxvox * 4, dtype=torch.float32, device=dev)
    atoms_dev = [ppm.atoms_to_device(w.atoms) for w in ws]
    m = ppm.df_half_width(ws[0].df.A, ws[0].scan.dz)
    outs = [torch.empty((sc.nz - 2 * m, sc.ny, sc.nx), dtype=torch.float32, device=dev)
            for (_, _, sc) in jobs]

    # the per-molecule loop builds with the batch's tuned depth (same bits) and
    # scans 128 x 128 lattices with the shape the autotuner picks for them
    tune = ppm.Tuning(ff_nzb=bp.ff_nzb)
    ff0 = ffbuf[:ws[0].grid.nvox * 4].view(ws[0].grid.n[2], ws[0].grid.n[1], ws[0].grid.n[0], 4)
    ppm.build_ff(ws[0].grid, ws[0].probe, atoms_dev[0], out=ff0, tuning=tune)
    tune, plain_scan_tune_ms, _ = ppm.tune_relaxed_scan(ws[0].grid, ff0, jobs[0][1], ws[0].fire,
                                                        jobs[0][2], dfp=ws[0].df, fz=False,
                                                        pp=False, out={"df": outs[0]},
                                                        tuning=tune)

    def plain():
        j = 0
        for i, w in enumerate(ws):
            nx, ny, nz = w.grid.n
            ff = ffbuf[:w.grid.nvox * 4].view(nz, ny, nx, 4)
            ppm.build_ff(w.grid, w.probe, atoms_dev[i], out=ff, tuning=tune)
            for _ in W.C3_K_LAT_N_PER_M:
                _, pr, sc = jobs[j]
                ppm.relaxed_scan(w.grid, ff, pr, w.fire, sc, dfp=w.df, fz=False, pp=False,
                                 out={"df": outs[j]}, tuning=tune)
                j += 1

    plain()
    tp = []
    for _ in range(2):
        torch.cuda.synchronize()
        e[0].record()
        plain()
        e[1].record()
        torch.cuda.synchronize()
        tp.append(e[0].elapsed_time(e[1]))
    plain_ms = float(np.median(tp))
    same = all(torch.equal(bp.df_stack(j), outs[j]) for j in range(len(jobs)))
    # the same per-molecule loop recorded once into a HIP graph (no launch
    # overhead left), to separate batching from launch cost
    pg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(pg):
        plain()
    tg = []
    for _ in range(3):
        torch.cuda.synchronize()
        e[0].record()
        pg.replay()
        e[1].record()
        torch.cuda.synchronize()
        tg.append(e[0].elapsed_time(e[1]))
    plain_graph_ms = float(np.median(tg))
    same_graph = all(torch.equal(bp.df_stack(j), outs[j]) for j in range(len(jobs)))
    del pg
    # FIRE evaluations of the batched scan, from the single scans (same bits) of
    # every 16th job with the probe state kept
    evals = pts = 0.0
    for j in range(0, len(jobs), 16):
        mi, pr, sc = jobs[j]
        r = ppm.relaxed_scan(ws[mi].grid, bp.ff_grid(mi), pr, ws[mi].fire, sc, fz=False, pp=True)
        it = r["pp"][..., 3]
        evals += float(it.abs().sum().item()) + sc.n_eq
        pts += sc.n_eq
    total_pts = float(sum(sc.n_eq for (_, _, sc) in jobs))
    scan_bytes = evals / pts * total_pts * BYTES_PER_EVAL
    scan_gbs = scan_bytes / (scan_ms * 1e-3) / 1e9
    gather_ceiling = (mb["gather_coherent_gbs"] * BYTES_PER_EVAL / MB_BYTES_PER_GATHER
                      if mb else None)
    voxels = sum(w.grid.nvox for w in ws)
    pairs = sum(w.grid.nvox * w.atoms.n for w in ws)
    return {"workload": f"{n_mol} seeded molecules, 10-120 atoms, cells with 5 A margins at "
                        "0.1 A, 128x128 tips x 20 heights, 3 lateral stiffnesses "
                        "(0.15, 0.25, 0.5 N/m)",
            "voxels": voxels, "pairs": pairs, "jobs": len(jobs),
            "batched_ms": round(batched_ms, 3), "plain_ms": round(plain_ms, 3),
            "batched_stacks_per_s": round(len(jobs) / (batched_ms * 1e-3), 1),
            "plain_stacks_per_s": round(len(jobs) / (plain_ms * 1e-3), 1),
            "batched_molecules_per_s": round(n_mol / (batched_ms * 1e-3), 1),
            "plain_molecules_per_s": round(n_mol / (plain_ms * 1e-3), 1),
            "plain_graph_ms": round(plain_graph_ms, 3),
            "speedup": round(plain_ms / batched_ms, 3),
            "speedup_vs_plain_graph": round(plain_graph_ms / batched_ms, 3),
            "speedup_baseline": "speedup: the per-molecule loop as issued from Python (one "
                                "build + 3 scans per molecule, one stream, no synchronisation); "
                                "speedup_vs_plain_graph: the same loop replayed as one graph",
            "batched_stage_ms": {"ff_build": round(ff_ms, 3), "scan": round(scan_ms, 3)},
            "batched_ff_tflops": round(pairs * FLOP_PER_PAIR / (ff_ms * 1e-3) / 1e12, 2),
            "batched_scan": {"note": "gather rate in algorithmic bytes (96 B per force "
                                     "evaluation); evaluations that reuse a lane's cached "
                                     "cell issue no load, so the rate can exceed the "
                                     "measured ceiling of real 8-corner gathers",
                             "fire_evals_per_point": round(evals / pts, 3),
                             "evals_sample": f"single scans of {len(range(0, len(jobs), 16))} "
                                             "of the jobs (every 16th)",
                             "gather_gbs": round(scan_gbs, 1),
                             "frac_of_measured_gather_ceiling":
                                 round(scan_gbs / gather_ceiling, 4) if gather_ceiling else None},
            "launch_shapes": {"ff_voxels_per_thread": bp.ff_nzb,
                              "ff_autotuner_ms": bp.tuning_ms,
                              "batched_scan_tile": "8x8",
                              "plain_scan_tile": f"{tune.scan_tile}x{tune.scan_tile}",
                              "plain_scan_autotuner_ms": plain_scan_tune_ms},
            "outputs_identical": bool(same and same_graph)}


def _pairs_within_cutoff(w):
    """Exact number of (voxel, atom) pairs with rho < cutoff for a grid periodic
    in x,y (minimum image; cutoff < L/2): per atom and z-layer, lattice rows
    crossing the disc, and per row the integers inside the chord."""
    g, at = w.grid, w.atoms
    hx, hy, hz = g.step
    nx, ny, nz = g.n
    rc = g.cutoff
    iz = np.arange(nz)
    iy = np.arange(ny)
    total = 0
    for a in at.pos:
        dz = g.origin[2] + iz * hz - a[2]
        dz = dz[np.abs(dz) < rc]
        r2 = rc * rc - dz * dz                                   # disc radius^2 per layer
        # minimum-image y offsets of every lattice row
        dy = g.origin[1] + iy * hy - a[1]
        dy -= ny * hy * np.rint(dy / (ny * hy))
        w2 = r2[:, None] - dy[None, :] ** 2                      # chord half-width^2
        ok = w2 > 0
        hw = np.sqrt(np.where(ok, w2, 0.0))
        x0 = (g.origin[0] - a[0]) % hx                           # lattice offset in x
        # integers k with |x0 + k hx| < hw
        cnt = np.ceil((hw - x0) / hx) - np.floor((-hw - x0) / hx) - 1
        total += int(np.sum(np.where(ok, cnt, 0)))
    return total


FLOP_PER_PAIR_QUAD = 47       # 31 of the point-charge probe + d_z2 term: dz^2 1, kQ/rho^5 3,
                              # E 4, force factor 5, Fz 3
# per grid point of the FFT route: max reduction (8), first x pass reading V and rho (8 + 16),
# seven axis passes (16 + 16), spectral product (16 read + 32 written), last z pass reading
# Fx + i Fy and E + i Fz and adding to the grid (32 + 16 read + 16 written)
HARTREE_BYTES_PER_POINT = 8 + 24 + 7 * 32 + 48 + 64
FLOP_PER_PAIR_ENERGY = 20     # energy only: d 3, r^2 5, rsq 1, 1/r^2 1, s^2 1, s^6 2,
                              # s^12 1, E_LJ 3, E_C 1, E sum 2


def _bench_next_rows(ppm, W, torch):
    """Paper-scale workload: lateral-mode stiffness post-pass over every relaxed
    point, and the tricubic variant (energy-only grid + scan on its tricubic
    interpolant)."""
    w = W.config1()
    atoms = ppm.atoms_to_device(w.atoms)
    ff = ppm.build_ff(w.grid, w.probe, atoms)
    res = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, w.scan, dfp=w.df)
    kbuf = ppm.lateral_stiffness(w.grid, ff, w.probe, w.scan, res["pp"])
    E = ppm.build_energy(w.grid, w.probe, atoms)
    tri = ppm.relaxed_scan_tricubic(w.grid, E, w.probe, w.fire, w.scan, dfp=w.df)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    tk, te, ts = [], [], []
    for _ in range(4):
        e[0].record()
        ppm.lateral_stiffness(w.grid, ff, w.probe, w.scan, res["pp"], out=kbuf)
        e[1].record()
        ppm.build_energy(w.grid, w.probe, atoms, out=E)
        e[2].record()
        ppm.relaxed_scan_tricubic(w.grid, E, w.probe, w.fire, w.scan, dfp=w.df, out=tri)
        e[3].record()
        torch.cuda.synchronize()
        tk.append(e[0].elapsed_time(e[1]))
        te.append(e[1].elapsed_time(e[2]))
        ts.append(e[2].elapsed_time(e[3]))
    n_eq = w.scan.n_eq
    pairs = w.grid.nvox * w.atoms.n
    k_ms, e_ms, s_ms = (float(np.median(x[1:])) for x in (tk, te, ts))
    it = tri["pp"][..., 3]
    # quadrupolar probe (d_z2, -0.05 e A^2, no monopole): the point-charge force field
    qprobe = dataclasses.replace(w.probe, q_pp=0.0, q_zz=-0.05)
    ffq = ppm.build_ff(w.grid, qprobe, atoms)
    qtune, qtune_ms = ppm.tune_build_ff(w.grid, qprobe, atoms, out=ffq)
    # grid electrostatics: LJ-only grid + FFT cross-correlation with the tip density
    V = torch.as_tensor(W.hartree_potential(w.atoms, w.grid).astype(np.float32), device="cuda")
    rho = ppm.tip_density(w.grid, 0.0, -0.05, W.TIP_SIGMA)
    ws = ppm.hartree_workspace(w.grid)
    lj_probe = dataclasses.replace(w.probe, q_pp=0.0, q_zz=0.0)
    ffh = ppm.build_ff(w.grid, lj_probe, atoms)
    ppm.hartree_ff(w.grid, V, rho, out=ffh, accumulate=True, workspace=ws)
    hres = ppm.relaxed_scan(w.grid, ffh, lj_probe, w.fire, w.scan, dfp=w.df, pp=False)
    tq, tl, th, tsc = [], [], [], []
    for _ in range(4):
        e[0].record()
        ppm.build_ff(w.grid, qprobe, atoms, out=ffq, tuning=qtune)
        e[1].record()
        ppm.build_ff(w.grid, lj_probe, atoms, out=ffh)
        e[2].record()
        ppm.hartree_ff(w.grid, V, rho, out=ffh, accumulate=True, workspace=ws)
        e[3].record()
        ppm.relaxed_scan(w.grid, ffh, lj_probe, w.fire, w.scan, dfp=w.df, pp=False, out=hres)
        e[4].record()
        torch.cuda.synchronize()
        tq.append(e[0].elapsed_time(e[1]))
        tl.append(e[1].elapsed_time(e[2]))
        th.append(e[2].elapsed_time(e[3]))
        tsc.append(e[3].elapsed_time(e[4]))
    q_ms, l_ms, h_ms, hs_ms = (float(np.median(x[1:])) for x in (tq, tl, th, tsc))
    nvox = w.grid.nvox
    return {"workload": "paper-scale (60 atoms, 240^3 grid, 240x240x100 scan)",
            "quadrupole_probe": {"ff_ms": round(q_ms, 3),
                                 "ff_tflops": round(pairs * FLOP_PER_PAIR_QUAD /
                                                    (q_ms * 1e-3) / 1e12, 2),
                                 "ff_voxels_per_thread": qtune.ff_nzb,
                                 "ff_autotuner_ms": qtune_ms},
            "hartree": {"note": "LJ grid + FFT cross-correlation of the d_z2 tip density "
                                "(-0.05 e A^2, sigma 0.7 A) with a synthetic periodic potential",
                        "lj_ff_ms": round(l_ms, 3),
                        "hartree_ms": round(h_ms, 3),
                        "hartree_algorithmic_gb": round(nvox * HARTREE_BYTES_PER_POINT / 1e9, 3),
                        "hartree_gbs": round(nvox * HARTREE_BYTES_PER_POINT / (h_ms * 1e-3) / 1e9,
                                             1),
                        "scan_ms": round(hs_ms, 3),
                        "relaxations_per_s": round(n_eq / ((l_ms + h_ms + hs_ms) * 1e-3), 1)},
            "lateral_stiffness": {"ms": round(k_ms, 3),
                                  "points_per_s": round(n_eq / (k_ms * 1e-3), 1),
                                  "gather_gbs": round(n_eq * (BYTES_PER_EVAL + 16 + 8) /
                                                      (k_ms * 1e-3) / 1e9, 1)},
            "tricubic": {"energy_grid_ms": round(e_ms, 3),
                         "energy_grid_tflops": round(pairs * FLOP_PER_PAIR_ENERGY /
                                                     (e_ms * 1e-3) / 1e12, 2),
                         "scan_ms": round(s_ms, 3),
                         "relaxations_per_s": round(n_eq / ((e_ms + s_ms) * 1e-3), 1),
                         "mean_fire_steps": round(float(it.abs().mean().item()), 3),
                         "not_converged": int((it < 0).sum().item()),
                         "grid_bytes": int(w.grid.nvox * 4)}}


def _cpu_baseline(w, n_eq):
    """The FP64 oracle, as it stands, on the host cores, on a bounded sample of
    the headline step, scaled to relaxations/s of the whole step:
      * force field: 4 of the 300 z-layers (full 400 x 400 planes, every atom
        tested against the cutoff), scaled by 300/4;
      * relaxed scan: a 40 x 40-column window over the flake (all 120 heights,
        the benchmark's FIRE settings, no Newton polish) on the oracle's own
        grid over the voxels those columns reach (built beforehand, untimed),
        scaled to the 160,000 columns.
    Each part: median of 3 timed runs after one warm-up, on every host core;
    then once more on one thread.  Also one molecule of the batched set (force
    field + 3 stiffness scans on 10% of the columns, scaled) as molecules/s."""
    import oracle as orc
    from paper_2401_14564_amd import workloads as W
    cores = orc.num_threads()
    nx, ny, nz = w.grid.n
    P = 4

    def ff_part():
        orc.build_ff(w.grid, w.probe, w.atoms, iz0=150, iz1=150 + P)

    # scan window: tips (180..219, 180..219); voxels the probes reach
    NW = 40
    scan = W.Scan(w.scan.x0 + 180 * w.scan.dx, w.scan.y0 + 180 * w.scan.dy, w.scan.dx,
                  w.scan.dy, NW, NW, w.scan.z_top, w.scan.dz, w.scan.nz)
    ix = np.arange(160, 241) % nx
    iy = np.arange(160, 241) % ny
    iz = np.arange(100, 240)
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    idx = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.int32)
    vals = orc.ff_voxels(w.grid, w.probe, w.atoms, idx, with_scale=False)
    ff = np.zeros((nz, ny, nx, 4))
    ff[idx[:, 2], idx[:, 1], idx[:, 0]] = vals.astype(np.float32)

    def scan_part():
        orc.relaxed_scan(w.grid, ff, w.probe, w.fire, scan)

    def med3(fn):
        fn()
        ts = []
        for _ in range(3):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    t_ff, t_scan = med3(ff_part), med3(scan_part)
    ncol = w.scan.nx * w.scan.ny
    t_step = t_ff * (nz / P) + t_scan * (ncol / NW ** 2)
    # one batched-set molecule: force field + three stiffness scans
    m0 = W.config3_molecule(0)
    rng = np.random.default_rng(12345)
    mcols = rng.choice(m0.scan.nx * m0.scan.ny, size=m0.scan.nx * m0.scan.ny // 10, replace=False)
    mcols = np.stack([mcols % m0.scan.nx, mcols // m0.scan.nx], axis=1).astype(np.int32)

    tm0 = time.perf_counter()
    fm = orc.build_ff(m0.grid, m0.probe, m0.atoms)
    tm1 = time.perf_counter()
    for k in W.C3_K_LAT_N_PER_M:
        pr = dataclasses.replace(m0.probe, k_lat=(k * W.N_PER_M, k * W.N_PER_M))
        r = orc.relaxed_scan(m0.grid, fm, pr, m0.fire, m0.scan, cols=mcols)
        orc.df(r["fz"].T, m0.scan.dz, m0.df)
    tm2 = time.perf_counter()
    t_mol = (tm1 - tm0) + (tm2 - tm1) * (m0.scan.nx * m0.scan.ny / len(mcols))
    # one thread
    orc.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        orc.build_ff(w.grid, w.probe, w.atoms, iz0=150, iz1=151)
        t_ff1 = (time.perf_counter() - t0) * P
        t0 = time.perf_counter()
        scan_part()
        t_scan1 = time.perf_counter() - t0
    finally:
        orc.set_num_threads(cores)
    t_step1 = t_ff1 * (nz / P) + t_scan1 * (ncol / NW ** 2)
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(n_eq / t_step, 1), "unit": "relaxations/s", "cores": cores,
            "kind": "oracle",
            "sample": f"large periodic step: force field on {P} of {nz} z-layers "
                      f"({t_ff:.3f} s, x{nz / P:.0f}) + relaxed scan of a {NW}x{NW}-column window "
                      f"x {w.scan.nz} heights ({t_scan:.3f} s, x{ncol / NW ** 2:.0f}) = "
                      f"{t_step:.1f} s "
                      f"per step; median of 3 after a warm-up; FP64, no polish; cpu: {cpu}, "
                      f"os.cpu_count() {os.cpu_count()}",
            "one_thread": {"value": round(n_eq / t_step1, 1), "step_s": round(t_step1, 1),
                           "note": "force field on one z-layer, the same scan window, one run"},
            "pairs_per_s": round(P * nx * ny * w.atoms.n / t_ff, 1),
            "equilibria_per_s": round(NW * NW * w.scan.nz / t_scan, 1),
            "batched_set_molecule": {
                "molecules_per_s": round(1.0 / t_mol, 3),
                "note": f"molecule 0 ({m0.atoms.n} atoms, grid {m0.grid.n}): full force field "
                        f"({tm1 - tm0:.2f} s) + 3 stiffness scans of {len(mcols)} of "
                        f"{m0.scan.nx * m0.scan.ny} columns ({tm2 - tm1:.2f} s, scaled), one run"}}


if __name__ == "__main__":
    main()
