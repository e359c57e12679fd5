"""Host-side checks of the C ABI (no GPU needed): the built library exports every
function include/ppm.h declares, the ctypes structs match the C layout, and
invalid arguments are rejected before anything is enqueued."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2401_14564_amd import _lib, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppm.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ppm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = _lib.lib()
    names = _declared_functions()
    assert "ppm_build_ff" in names and "ppm_relaxed_scan_backward" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(_lib.EXPORTED)


def test_struct_layout_matches_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "ppm.h"\n'
        "int main(void){\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(ppm_grid), sizeof(ppm_probe), sizeof(ppm_fire),'
        " sizeof(ppm_scan), sizeof(ppm_df_params));\n"
        'printf("%zu %zu %zu %zu %zu\\n", offsetof(ppm_grid, cutoff), offsetof(ppm_probe, d0),'
        " offsetof(ppm_fire, max_iter), offsetof(ppm_scan, nz), offsetof(ppm_scan, z_top));\n"
        'printf("%zu %zu %zu %zu %zu\\n", sizeof(ppm_tuning), sizeof(ppm_batch_mol),'
        " offsetof(ppm_batch_mol, ff_nzb), offsetof(ppm_batch_mol, ff_offset),"
        " sizeof(ppm_batch_scan));\n"
        "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(prog), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    sizes = [int(v) for v in out]
    assert sizes[:5] == [ct.sizeof(_lib.Grid), ct.sizeof(_lib.Probe), ct.sizeof(_lib.Fire),
                         ct.sizeof(_lib.Scan), ct.sizeof(_lib.DfParams)]
    assert sizes[5:10] == [_lib.Grid.cutoff.offset, _lib.Probe.d0.offset,
                           _lib.Fire.max_iter.offset, _lib.Scan.nz.offset, _lib.Scan.z_top.offset]
    assert sizes[10:] == [ct.sizeof(_lib.Tuning), ct.sizeof(_lib.BatchMol),
                          _lib.BatchMol.ff_nzb.offset, _lib.BatchMol.ff_offset.offset,
                          ct.sizeof(_lib.BatchScan)]


def test_status_strings():
    assert _lib.string(_lib.PPM_OK) == "ok"
    assert "invalid" in _lib.string(_lib.PPM_EINVAL)
    assert _lib.string(12345) == "unknown status"


def test_df_half_width():
    L = _lib.lib()
    assert L.ppm_df_half_width(1.0, 0.1) == 5
    assert L.ppm_df_half_width(0.7, 0.1) == 4
    assert L.ppm_df_half_width(2.0, 0.05) == 20
    assert L.ppm_df_half_width(0.0, 0.1) == -1
    assert L.ppm_df_half_width(1.0, -0.1) == -1


FAKE = ct.c_void_p(0x1000)   # never dereferenced: every call below fails validation


def _args():
    w = W.config0()
    return (_lib.grid_struct(w.grid), _lib.probe_struct(w.probe), _lib.fire_struct(w.fire),
            _lib.scan_struct(w.scan), _lib.df_struct(w.df))


def test_c_program_links_the_library_and_gets_its_errors(tmp_path):
    """A C99 program (strict, warnings as errors) includes the public headers,
    links libppm.so and receives the host-side validation results: a zero-sized
    grid, a missing output and a workspace query for an invalid scan (no launch
    is reached, so no GPU is needed)."""
    prog = tmp_path / "client.c"
    prog.write_text(r"""
#include <stdio.h>
#include <string.h>
#include "ppm.h"
int main(void) {
    ppm_grid g; ppm_probe p; ppm_scan s;
    memset(&g, 0, sizeof g); memset(&p, 0, sizeof p); memset(&s, 0, sizeof s);
    double x = 0.0;
    float out = 0.0f;
    ppm_status a = ppm_build_ff(&g, &p, 1, &x, &x, &x, &x, &out, NULL);
    g.n[0] = g.n[1] = g.n[2] = 8;
    g.step[0] = g.step[1] = g.step[2] = 0.1;
    p.d0[2] = -4.0; p.k_rad = 1.0; p.R_pp = 1.66; p.eps_pp = 0.0091;
    ppm_status b = ppm_build_ff(&g, &p, 1, &x, &x, &x, &x, NULL, NULL);
    size_t ws = ppm_backward_workspace_bytes(&s, 10);
    printf("%d %d %zu %s\n", (int)a, (int)b, ws, ppm_status_string(a));
    return 0;
}
""")
    exe = tmp_path / "client"
    pkg = os.path.dirname(_lib.LIB_PATH)
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                    os.path.dirname(HEADER), str(prog), "-o", str(exe), "-L", pkg, "-lppm",
                    f"-Wl,-rpath,{pkg}"], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert int(out[0]) == _lib.PPM_EINVAL and int(out[1]) == _lib.PPM_EINVAL
    assert int(out[2]) == 0
    assert " ".join(out[3:]) == _status_string(_lib.PPM_EINVAL)


def _status_string(code):
    return _lib.lib().ppm_status_string(code).decode()


def test_build_ff_rejects_bad_arguments():
    L = _lib.lib()
    g, p, f, s, d = _args()
    assert L.ppm_build_ff(None, p, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL
    assert L.ppm_build_ff(g, p, 1, None, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL
    assert L.ppm_build_ff(g, p, -1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL
    assert L.ppm_build_ff(g, p, 1, FAKE, FAKE, FAKE, FAKE, None, None) == _lib.PPM_EINVAL
    bad = _lib.grid_struct(W.Grid((0, 0, 0), (0.1, 0.1, 0.1), (1, 10, 10)))
    assert L.ppm_build_ff(bad, p, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL
    bad = _lib.grid_struct(W.Grid((0, 0, 0), (0.1, 0.0, 0.1), (10, 10, 10)))
    assert L.ppm_build_ff(bad, p, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL
    huge = _lib.grid_struct(W.Grid((0, 0, 0), (0.1, 0.1, 0.1), (2048, 2048, 1024)))
    assert L.ppm_build_ff(huge, p, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_ERANGE
    # periodic: cutoff must leave room for the brick half-diagonal below L/2
    per = _lib.grid_struct(W.Grid((0, 0, 0), (0.1, 0.1, 0.1), (100, 100, 10), 1, 4.9))
    assert L.ppm_build_ff(per, p, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL
    per = _lib.grid_struct(W.Grid((0, 0, 0), (0.1, 0.1, 0.1), (100, 100, 10), 1, 0.0))
    assert L.ppm_build_ff(per, p, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL
    badp = _lib.probe_struct(W.Probe(d0=(0.0, 0.0, 0.0)))
    assert L.ppm_build_ff(g, badp, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL
    badp = _lib.probe_struct(W.Probe(k_rad=-1.0))
    assert L.ppm_build_ff(g, badp, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None) == _lib.PPM_EINVAL


def test_relaxed_scan_rejects_bad_arguments():
    L = _lib.lib()
    g, p, f, s, d = _args()
    E = _lib.PPM_EINVAL
    assert L.ppm_relaxed_scan(g, FAKE, p, f, s, None, None, None, None, None) == E  # no output
    assert L.ppm_relaxed_scan(g, None, p, f, s, FAKE, None, None, None, None) == E  # no ff
    assert L.ppm_relaxed_scan(g, FAKE, p, f, s, None, None, None, FAKE, None) == E  # df w/o dfp
    for bad in (dict(f_conv=0.0), dict(dt0=-1.0), dict(mass=0.0), dict(max_iter=0),
                dict(alpha0=1.5), dict(n_min=-1)):
        bf = _lib.fire_struct(W.Fire(**bad))
        assert L.ppm_relaxed_scan(g, FAKE, p, bf, s, FAKE, None, None, None, None) == E, bad
    short = _lib.scan_struct(W.Scan(0, 0, 0.1, 0.1, 4, 4, 10.0, 0.1, 10))   # < 2m+1 = 11
    assert L.ppm_relaxed_scan(g, FAKE, p, f, short, None, None, d, FAKE, None) == E
    empty = _lib.scan_struct(W.Scan(0, 0, 0.1, 0.1, 0, 4, 10.0, 0.1, 20))
    assert L.ppm_relaxed_scan(g, FAKE, p, f, empty, FAKE, None, None, None, None) == E
    wide = _lib.df_struct(W.DfParams(A=7.0))                                # m = 35 > 32
    tall = _lib.scan_struct(W.Scan(0, 0, 0.1, 0.1, 4, 4, 10.0, 0.1, 80))
    assert L.ppm_relaxed_scan(g, FAKE, p, f, tall, None, None, wide, FAKE, None) == \
        _lib.PPM_EUNSUPPORTED


def test_df_and_backward_reject_bad_arguments():
    L = _lib.lib()
    g, p, f, s, d = _args()
    E = _lib.PPM_EINVAL
    assert L.ppm_df(None, 20, 4, 4, 0.1, d, FAKE, None) == E
    assert L.ppm_df(FAKE, 10, 4, 4, 0.1, d, FAKE, None) == E          # nz < 2m+1
    assert L.ppm_df(FAKE, 20, 0, 4, 0.1, d, FAKE, None) == E
    assert L.ppm_df(FAKE, 20, 4, 4, 0.0, d, FAKE, None) == E
    assert L.ppm_df(FAKE, 20, 4, 4, 0.1, _lib.df_struct(W.DfParams(k_cant=0.0)), FAKE, None) == E
    ws = L.ppm_backward_workspace_bytes(s, 12)
    assert ws > 0 and ws % 256 == 0
    args = [g, FAKE, p, s, d, 12, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE,
            FAKE, ws - 1, None]
    assert L.ppm_relaxed_scan_backward(*args) == E                     # workspace too small
    args[-2] = ws
    args[10] = None                                                    # no saved probe state
    assert L.ppm_relaxed_scan_backward(*args) == E


def test_batch_plan_offsets_on_host():
    """ppm_batch_plan fills the table offsets and totals on the host (no GPU)."""
    L = _lib.lib()
    ws = [W.config3_molecule(i) for i in range(3)]
    mols = (_lib.BatchMol * 3)()
    begin = 0
    for i, w in enumerate(ws):
        mols[i].grid = _lib.grid_struct(w.grid)
        mols[i].atom_begin = begin
        mols[i].n_atoms = w.atoms.n
        begin += w.atoms.n
    jobs = (_lib.BatchScan * 6)()
    for j in range(6):
        w = ws[j // 2]
        jobs[j].probe = _lib.probe_struct(w.probe)
        jobs[j].scan = _lib.scan_struct(w.scan)
        jobs[j].mol = j // 2
    totals = (ct.c_int64 * 5)()
    assert L.ppm_batch_plan(3, mols, 6, jobs, _lib.df_struct(W.DfParams()), totals) == _lib.PPM_OK
    vox = [w.grid.nvox for w in ws]
    assert [m.ff_offset for m in mols] == [0, vox[0], vox[0] + vox[1]]
    assert totals[0] == sum(vox)
    bricks = [((w.grid.n[0] + 15) // 16) * ((w.grid.n[1] + 15) // 16) * ((w.grid.n[2] + 7) // 8)
              for w in ws]
    assert [m.brick_begin for m in mols] == [0, bricks[0], bricks[0] + bricks[1]]
    assert totals[1] == sum(bricks)
    per_fz = [w.scan.nx * w.scan.ny * w.scan.nz for w in ws]
    assert [j.fz_offset for j in jobs] == list(np.cumsum([0] + [per_fz[k // 2] for k in range(5)]))
    assert totals[2] == 2 * sum(per_fz)
    assert totals[3] == 2 * sum(w.scan.nx * w.scan.ny * (w.scan.nz - 10) for w in ws)
    assert totals[4] == 6 * 256                     # 128x128 tips = 256 tiles of 8x8
    # a job pointing at a missing molecule is rejected
    jobs[5].mol = 3
    assert L.ppm_batch_plan(3, mols, 6, jobs, None, totals) == _lib.PPM_EINVAL
    jobs[5].mol = 2
    # springs may differ per job, the probe's LJ parameters and charges may not
    import dataclasses
    jobs[4].probe = _lib.probe_struct(dataclasses.replace(ws[2].probe, k_lat=(0.01, 0.02)))
    assert L.ppm_batch_plan(3, mols, 6, jobs, None, totals) == _lib.PPM_OK
    for change in (dict(q_pp=-0.1), dict(q_zz=-0.05), dict(R_pp=1.7), dict(eps_pp=0.01)):
        jobs[4].probe = _lib.probe_struct(dataclasses.replace(ws[2].probe, **change))
        assert L.ppm_batch_plan(3, mols, 6, jobs, None, totals) == _lib.PPM_EINVAL, change


def test_hartree_sizes_and_bad_arguments():
    L = _lib.lib()
    E, U = _lib.PPM_EINVAL, _lib.PPM_EUNSUPPORTED
    g = _lib.grid_struct(W.Grid((0, 0, 0), (0.1, 0.1, 0.1), (240, 30, 27)))
    nbytes = L.ppm_hartree_workspace_bytes(g)
    n = 240 * 30 * 27
    assert nbytes >= 3 * ((n * 16 + 255) // 256 * 256) and nbytes % 256 == 0
    for bad in ((7, 8, 8), (8, 8, 1030), (8, 11, 8)):        # prime factor 7/11, too long
        gb = _lib.grid_struct(W.Grid((0, 0, 0), (0.1, 0.1, 0.1), bad))
        assert L.ppm_hartree_workspace_bytes(gb) == 0
        assert L.ppm_hartree_ff(gb, FAKE, FAKE, 0, FAKE, FAKE, 1 << 40, None) == U
    assert L.ppm_hartree_ff(g, None, FAKE, 0, FAKE, FAKE, nbytes, None) == E
    assert L.ppm_hartree_ff(g, FAKE, FAKE, 2, FAKE, FAKE, nbytes, None) == E
    assert L.ppm_hartree_ff(g, FAKE, FAKE, 0, FAKE, FAKE, nbytes - 1, None) == E
    assert L.ppm_hartree_ff(g, FAKE, FAKE, 0, FAKE, None, nbytes, None) == E
    assert L.ppm_tip_density(g, 0.0, -0.05, 0.0, FAKE, None) == E
    assert L.ppm_tip_density(g, float("nan"), -0.05, 0.7, FAKE, None) == E
    assert L.ppm_tip_density(g, 0.0, -0.05, 0.7, None, None) == E


def test_python_wrappers_reject_bad_buffers_before_launch():
    """The bindings pass bare pointers, so every wrapper checks shape, dtype,
    contiguity and device of each buffer against the grid and scan it is called
    with and raises before the library is called.  CPU tensors of the right
    shape reach the device check, which is the last one."""
    import torch
    import paper_2401_14564_amd as ppm
    grid = W.Grid((0.0, 0.0, 0.0), (0.1, 0.1, 0.1), (8, 6, 10))
    scan = W.Scan(0.1, 0.1, 0.1, 0.1, 3, 2, 4.0, 0.1, 12)
    probe, fire, dfp = W.Probe(), W.Fire(), W.DfParams()
    good_ff = torch.zeros((10, 6, 8, 4))
    short_ff = torch.zeros((9, 6, 8, 4))
    with pytest.raises(ValueError, match="shape"):
        ppm.relaxed_scan(grid, short_ff, probe, fire, scan)
    with pytest.raises(ValueError, match="dtype"):
        ppm.relaxed_scan(grid, good_ff.double(), probe, fire, scan)
    with pytest.raises(ValueError, match="contiguous"):
        ppm.relaxed_scan(grid, torch.zeros((8, 6, 10, 4)).permute(2, 1, 0, 3), probe, fire, scan)
    with pytest.raises(ValueError, match="device"):
        ppm.relaxed_scan(grid, good_ff, probe, fire, scan)
    with pytest.raises(ValueError, match="shape"):
        ppm.relaxed_scan_tricubic(grid, torch.zeros((10, 6, 9)), probe, fire, scan)
    with pytest.raises(ValueError, match="shape"):
        ppm.lateral_stiffness(grid, short_ff, probe, scan, torch.zeros((12, 2, 3, 4)))
    with pytest.raises(ValueError, match="pp"):
        ppm.lateral_stiffness(grid, good_ff, probe, scan, torch.zeros((12, 2, 4, 4)))
    with pytest.raises(ValueError, match="dtype"):
        ppm.df(torch.zeros((12, 2, 3), dtype=torch.float64), 0.1, dfp)
    with pytest.raises(ValueError, match="device"):
        ppm.df(torch.zeros((12, 2, 3)), 0.1, dfp)
    atoms = (torch.zeros((2, 3), dtype=torch.float64), torch.zeros(3, dtype=torch.float64),
             torch.zeros(3, dtype=torch.float64), torch.zeros(3, dtype=torch.float64))
    with pytest.raises(ValueError, match="atoms"):
        ppm.atoms_to_device(atoms, device="cpu")
    with pytest.raises(ValueError, match="grad_df"):
        ppm.relaxed_scan_backward(grid, good_ff, probe, scan, dfp, atoms, torch.zeros((12, 2, 3, 4)),
                                  torch.zeros((12, 2, 3)))
    with pytest.raises(ValueError, match="out\\['df'\\]"):
        ppm.relaxed_scan(grid, good_ff, probe, fire, scan, dfp=dfp,
                         out={"df": torch.zeros((12, 2, 3))})


def test_microbench_library_exports_its_header():
    """The benchmark's measurement kernels (libppm_microbench.so) export what
    include/ppm_microbench.h declares and reject bad arguments on the host."""
    src = open(os.path.join(ROOT, "include", "ppm_microbench.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = sorted(set(re.findall(r"\b(ppm_mb_[a-z_0-9]+)\s*\(", src)))
    assert names == ["ppm_mb_gather", "ppm_mb_gather_band_bytes", "ppm_mb_issue", "ppm_mb_pair"]
    L = ct.CDLL(os.path.join(ROOT, "paper_2401_14564_amd", "libppm_microbench.so"))
    for n in names:
        assert hasattr(L, n), n
    L.ppm_mb_gather_band_bytes.restype = ct.c_size_t
    assert L.ppm_mb_gather_band_bytes() == 64 * 64 * 32 * 16
    L.ppm_mb_gather.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_uint32,
                                ct.c_void_p, ct.c_void_p]
    L.ppm_mb_pair.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p]
    assert L.ppm_mb_gather(None, 1, 1, 1, 0, FAKE, None) == -1
    assert L.ppm_mb_gather(FAKE, 1, 0, 1, 0, FAKE, None) == -1
    assert L.ppm_mb_pair(0, 1, 1, None, None) == -1
    L.ppm_mb_issue.argtypes = [ct.c_int, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p]
    assert L.ppm_mb_issue(4, 1, 1, FAKE, None) == -1       # unknown kind
    assert L.ppm_mb_issue(0, 1, 0, FAKE, None) == -1
    assert L.ppm_mb_issue(0, 1, 1, None, None) == -1


def test_tuning_arguments_rejected_on_host():
    """Launch shapes outside the tuner's candidates are rejected before any
    launch; the tuners need somewhere to write their choice; a batch plan
    counts bricks with each molecule's depth."""
    L = _lib.lib()
    E = _lib.PPM_EINVAL
    g = _lib.grid_struct(W.Grid((0, 0, 0), (0.1, 0.1, 0.1), (20, 20, 20)))
    pr = _lib.probe_struct(W.Probe())
    for bad in (4, 7, 12, -1):
        assert L.ppm_build_ff_tuned(g, pr, _lib.Tuning(bad, 0), 1, FAKE, FAKE, FAKE, FAKE, FAKE,
                                    None) == E
    sc = _lib.scan_struct(W.Scan(0.5, 0.5, 0.1, 0.1, 4, 4, 3.0, 0.1, 12))
    fi = _lib.fire_struct(W.Fire())
    for bad in (4, 32, -8):
        assert L.ppm_relaxed_scan_tuned(g, FAKE, pr, fi, sc, _lib.Tuning(0, bad), FAKE, None,
                                        None, None, None) == E
    for bad in (2, -1):     # scan_fz_direct is 0 or 1
        assert L.ppm_relaxed_scan_tuned(g, FAKE, pr, fi, sc, _lib.Tuning(0, 8, bad), FAKE, None,
                                        None, None, None) == E
    assert L.ppm_tune_build_ff(g, pr, 1, FAKE, FAKE, FAKE, FAKE, FAKE, None, None, None) == E
    assert L.ppm_tune_relaxed_scan(g, FAKE, pr, fi, sc, FAKE, None, None, None, None, None,
                                   None) == E
    # plan: depth 6 bricks, a bad depth rejected
    w = W.config3_molecule(0)
    mols = (_lib.BatchMol * 1)()
    mols[0].grid = _lib.grid_struct(w.grid)
    mols[0].n_atoms = w.atoms.n
    mols[0].ff_nzb = 6
    totals = (ct.c_int64 * 5)()
    assert L.ppm_batch_plan(1, mols, 0, None, None, totals) == _lib.PPM_OK
    nx, ny, nz = w.grid.n
    assert totals[1] == ((nx + 15) // 16) * ((ny + 15) // 16) * ((nz + 5) // 6)
    mols[0].ff_nzb = 5
    assert L.ppm_batch_plan(1, mols, 0, None, None, totals) == E


def test_noalloc_backward_limit_checked_on_host():
    """The no-alloc backward rejects a workload beyond its static array (and a
    bad scan) on the host, before it looks up the array or launches anything."""
    L = _lib.lib()
    w = W.config1()
    args = (_lib.grid_struct(w.grid), FAKE, _lib.probe_struct(w.probe), _lib.scan_struct(w.scan),
            _lib.df_struct(w.df), w.atoms.n) + (FAKE,) * 10 + (None,)
    assert L.ppm_relaxed_scan_backward_noalloc(*args) == _lib.PPM_ERANGE
    bad = _lib.scan_struct(W.Scan(0.0, 0.0, 0.1, 0.1, 0, 4, 3.0, 0.1, 12))
    args = args[:3] + (bad,) + args[4:]
    assert L.ppm_relaxed_scan_backward_noalloc(*args) == _lib.PPM_EINVAL
