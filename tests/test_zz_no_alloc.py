"""ppm_relaxed_scan_backward_noalloc (static device workspace, no allocation)
against ppm_relaxed_scan_backward with a caller-provided workspace, through
the C ABI: two calls in a row, the second on a smaller input, each bit for bit
equal to the workspace call (same kernels, deterministic reduction); and the
size limit rejected before any launch."""
import ctypes as ct

import numpy as np
import pytest
import torch

import paper_2401_14564_amd as ppm
from paper_2401_14564_amd import _lib, workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(grid, ff, probe, scan, dfp, atoms, pp, gdf):
    L = _lib.lib()
    pos, q, R, eps = ppm.atoms_to_device(atoms)
    n = int(q.numel())
    g = {k: torch.full(s, np.nan, dtype=torch.float64, device=ff.device)
         for k, s in (("pos", (n, 3)), ("q", (n,)), ("R", (n,)), ("eps", (n,)))}
    st = L.ppm_relaxed_scan_backward_noalloc(
        _lib.grid_struct(grid), _lib.ptr(ff), _lib.probe_struct(probe), _lib.scan_struct(scan),
        _lib.df_struct(dfp), n, _lib.ptr(pos), _lib.ptr(q), _lib.ptr(R), _lib.ptr(eps),
        _lib.ptr(pp), _lib.ptr(gdf), _lib.ptr(g["pos"]), _lib.ptr(g["q"]), _lib.ptr(g["R"]),
        _lib.ptr(g["eps"]), ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, g


def test_noalloc_backward_equals_workspace_call_on_two_calls():
    w, _ = W.config4()
    scans = [W.Scan(w.scan.x0, w.scan.y0, 0.1, 0.1, 96, 80, w.scan.z_top, 0.1, 28),
             W.Scan(w.scan.x0 + 2.0, w.scan.y0 + 1.5, 0.1, 0.1, 24, 20, w.scan.z_top, 0.1, 16)]
    ff = ppm.build_ff(w.grid, w.probe, w.atoms)
    gen = torch.Generator("cuda").manual_seed(11)
    for i, scan in enumerate(scans):
        print(f"no-alloc call {i}: scan {scan.nx}x{scan.ny}x{scan.nz}", flush=True)
        res = ppm.relaxed_scan(w.grid, ff, w.probe, w.fire, scan, dfp=w.df)
        gdf = torch.randn(res["df"].shape, device="cuda", generator=gen)
        ref = ppm.relaxed_scan_backward(w.grid, ff, w.probe, scan, w.df, w.atoms, res["pp"], gdf)
        st, got = _noalloc(w.grid, ff, w.probe, scan, w.df, w.atoms, res["pp"], gdf)
        torch.cuda.synchronize()
        assert st == _lib.PPM_OK, _lib.string(st)
        for k in ref:
            assert torch.equal(got[k], ref[k]), (i, k)


def test_noalloc_backward_rejects_inputs_beyond_its_array():
    L = _lib.lib()
    w = W.config1()
    # the full paper-scale lattice needs ~276 MiB of workspace
    need = L.ppm_backward_workspace_bytes(_lib.scan_struct(w.scan), w.atoms.n)
    assert need > 64 * 1024 * 1024
    fake = torch.empty(1, device="cuda")
    st, _ = _noalloc(w.grid, fake, w.probe, w.scan, w.df, w.atoms, fake, fake)
    assert st == _lib.PPM_ERANGE
