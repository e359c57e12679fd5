"""ctypes binding of libppm (include/ppm.h): structs, signatures, loading.

Argument marshalling only.  Every step of the probe-particle path runs in the
HIP kernels of libppm.so; if the library is missing this module raises instead
of falling back to anything else.
"""
from __future__ import annotations

import ctypes as ct
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libppm.so")

PPM_OK = 0
PPM_EINVAL = -1
PPM_ERANGE = -2
PPM_EHIP = -3
PPM_EUNSUPPORTED = -4

EXPORTED = (
    "ppm_status_string", "ppm_last_hip_error", "ppm_df_half_width", "ppm_build_ff",
    "ppm_relaxed_scan", "ppm_df", "ppm_backward_workspace_bytes",
    "ppm_relaxed_scan_backward", "ppm_batch_plan", "ppm_batch_build_ff",
    "ppm_batch_relaxed_scan", "ppm_lateral_stiffness", "ppm_build_energy",
    "ppm_relaxed_scan_tricubic", "ppm_tip_density", "ppm_hartree_workspace_bytes",
    "ppm_hartree_ff", "ppm_build_ff_tuned", "ppm_relaxed_scan_tuned", "ppm_tune_build_ff",
    "ppm_tune_relaxed_scan", "ppm_relaxed_scan_backward_noalloc",
)


class PPMError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = string(status) if _LIB is not None else str(status)
        extra = ""
        if status == PPM_EHIP and _LIB is not None:
            extra = f" (hipError {int(_LIB.ppm_last_hip_error())})"
        super().__init__(f"{where}: {msg}{extra}")
        self.status = status


class Grid(ct.Structure):
    _fields_ = [("origin", ct.c_double * 3), ("step", ct.c_double * 3), ("n", ct.c_int32 * 3),
                ("periodic_xy", ct.c_int32), ("cutoff", ct.c_double)]


class Probe(ct.Structure):
    _fields_ = [("R_pp", ct.c_double), ("eps_pp", ct.c_double), ("q_pp", ct.c_double),
                ("k_lat", ct.c_double * 2), ("k_rad", ct.c_double), ("d0", ct.c_double * 3),
                ("q_zz", ct.c_double)]


class Fire(ct.Structure):
    _fields_ = [("dt0", ct.c_double), ("dt_max", ct.c_double), ("f_inc", ct.c_double),
                ("f_dec", ct.c_double), ("alpha0", ct.c_double), ("f_alpha", ct.c_double),
                ("mass", ct.c_double), ("f_conv", ct.c_double), ("n_min", ct.c_int32),
                ("max_iter", ct.c_int32)]


class Scan(ct.Structure):
    _fields_ = [("x0", ct.c_double), ("y0", ct.c_double), ("dx", ct.c_double),
                ("dy", ct.c_double), ("nx", ct.c_int32), ("ny", ct.c_int32),
                ("z_top", ct.c_double), ("dz", ct.c_double), ("nz", ct.c_int32)]


class DfParams(ct.Structure):
    _fields_ = [("A", ct.c_double), ("f0", ct.c_double), ("k_cant", ct.c_double)]


class Tuning(ct.Structure):
    _fields_ = [("ff_nzb", ct.c_int32), ("scan_tile", ct.c_int32),
                ("scan_fz_direct", ct.c_int32)]


class BatchMol(ct.Structure):
    _fields_ = [("grid", Grid), ("atom_begin", ct.c_int32), ("n_atoms", ct.c_int32),
                ("ff_nzb", ct.c_int32), ("reserved", ct.c_int32),
                ("ff_offset", ct.c_int64), ("brick_begin", ct.c_int64)]


class BatchScan(ct.Structure):
    _fields_ = [("probe", Probe), ("scan", Scan), ("mol", ct.c_int32), ("reserved", ct.c_int32),
                ("fz_offset", ct.c_int64), ("df_offset", ct.c_int64), ("tile_begin", ct.c_int64)]


_LIB = None
_LOCK = threading.Lock()


def lib():
    """Load libppm.so (built in-tree by paper_2401_14564_amd.build)."""
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with "
                    "`python -m paper_2401_14564_amd.build` (hipcc, gfx950)")
            L = ct.CDLL(LIB_PATH)
            vp, i32, d, st = ct.c_void_p, ct.c_int32, ct.c_double, ct.c_int32
            P = ct.POINTER
            L.ppm_status_string.argtypes = [st]
            L.ppm_status_string.restype = ct.c_char_p
            L.ppm_last_hip_error.restype = i32
            L.ppm_df_half_width.argtypes = [d, d]
            L.ppm_df_half_width.restype = i32
            L.ppm_build_ff.argtypes = [P(Grid), P(Probe), i32, vp, vp, vp, vp, vp, vp]
            L.ppm_build_ff.restype = st
            L.ppm_relaxed_scan.argtypes = [P(Grid), vp, P(Probe), P(Fire), P(Scan), vp, vp,
                                           P(DfParams), vp, vp]
            L.ppm_relaxed_scan.restype = st
            L.ppm_df.argtypes = [vp, i32, i32, i32, d, P(DfParams), vp, vp]
            L.ppm_df.restype = st
            L.ppm_backward_workspace_bytes.argtypes = [P(Scan), i32]
            L.ppm_backward_workspace_bytes.restype = ct.c_size_t
            L.ppm_relaxed_scan_backward.argtypes = [P(Grid), vp, P(Probe), P(Scan), P(DfParams),
                                                    i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp,
                                                    vp, ct.c_size_t, vp]
            L.ppm_relaxed_scan_backward.restype = st
            L.ppm_relaxed_scan_backward_noalloc.argtypes = [P(Grid), vp, P(Probe), P(Scan),
                                                            P(DfParams), i32, vp, vp, vp, vp,
                                                            vp, vp, vp, vp, vp, vp, vp]
            L.ppm_relaxed_scan_backward_noalloc.restype = st
            L.ppm_batch_plan.argtypes = [i32, P(BatchMol), i32, P(BatchScan), P(DfParams),
                                         P(ct.c_int64)]
            L.ppm_batch_plan.restype = st
            L.ppm_batch_build_ff.argtypes = [i32, P(BatchMol), vp, P(Probe), vp, vp, vp, vp, vp,
                                             vp]
            L.ppm_batch_build_ff.restype = st
            L.ppm_batch_relaxed_scan.argtypes = [i32, P(BatchMol), vp, i32, P(BatchScan), vp,
                                                 P(Fire), P(DfParams), vp, vp, vp, vp]
            L.ppm_batch_relaxed_scan.restype = st
            L.ppm_lateral_stiffness.argtypes = [P(Grid), vp, P(Probe), P(Scan), vp, vp, vp]
            L.ppm_lateral_stiffness.restype = st
            L.ppm_build_energy.argtypes = [P(Grid), P(Probe), i32, vp, vp, vp, vp, vp, vp]
            L.ppm_build_energy.restype = st
            L.ppm_relaxed_scan_tricubic.argtypes = [P(Grid), vp, P(Probe), P(Fire), P(Scan), vp,
                                                    vp, P(DfParams), vp, vp]
            L.ppm_relaxed_scan_tricubic.restype = st
            L.ppm_tip_density.argtypes = [P(Grid), d, d, d, vp, vp]
            L.ppm_tip_density.restype = st
            L.ppm_hartree_workspace_bytes.argtypes = [P(Grid)]
            L.ppm_hartree_workspace_bytes.restype = ct.c_size_t
            L.ppm_hartree_ff.argtypes = [P(Grid), vp, vp, i32, vp, vp, ct.c_size_t, vp]
            L.ppm_hartree_ff.restype = st
            L.ppm_build_ff_tuned.argtypes = [P(Grid), P(Probe), P(Tuning), i32, vp, vp, vp, vp,
                                             vp, vp]
            L.ppm_build_ff_tuned.restype = st
            L.ppm_relaxed_scan_tuned.argtypes = [P(Grid), vp, P(Probe), P(Fire), P(Scan),
                                                 P(Tuning), vp, vp, P(DfParams), vp, vp]
            L.ppm_relaxed_scan_tuned.restype = st
            L.ppm_tune_build_ff.argtypes = [P(Grid), P(Probe), i32, vp, vp, vp, vp, vp, vp,
                                            P(Tuning), vp]
            L.ppm_tune_build_ff.restype = st
            L.ppm_tune_relaxed_scan.argtypes = [P(Grid), vp, P(Probe), P(Fire), P(Scan), vp, vp,
                                                P(DfParams), vp, vp, P(Tuning), vp]
            L.ppm_tune_relaxed_scan.restype = st
            _LIB = L
    return _LIB


def string(status: int) -> str:
    return lib().ppm_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != PPM_OK:
        raise PPMError(int(status), where)


# ------------------------------------------------------------------ structs
def grid_struct(g) -> Grid:
    return Grid((ct.c_double * 3)(*g.origin), (ct.c_double * 3)(*g.step),
                (ct.c_int32 * 3)(*[int(v) for v in g.n]), int(g.periodic_xy), float(g.cutoff))


def probe_struct(p) -> Probe:
    return Probe(p.R_pp, p.eps_pp, p.q_pp, (ct.c_double * 2)(*p.k_lat), p.k_rad,
                 (ct.c_double * 3)(*p.d0), float(getattr(p, "q_zz", 0.0)))


def fire_struct(f) -> Fire:
    return Fire(f.dt0, f.dt_max, f.f_inc, f.f_dec, f.alpha0, f.f_alpha, f.mass, f.f_conv,
                int(f.n_min), int(f.max_iter))


def scan_struct(s) -> Scan:
    return Scan(s.x0, s.y0, s.dx, s.dy, int(s.nx), int(s.ny), s.z_top, s.dz, int(s.nz))


def df_struct(d) -> DfParams:
    return DfParams(d.A, d.f0, d.k_cant)


def tuning_struct(t) -> Tuning | None:
    """ctypes Tuning from anything with ff_nzb / scan_tile attributes (None -> NULL)."""
    if t is None:
        return None
    return Tuning(int(getattr(t, "ff_nzb", 0)), int(getattr(t, "scan_tile", 0)),
                  int(getattr(t, "scan_fz_direct", 0)))


def ptr(t):
    """Device pointer of a tensor (None -> NULL); raises for a host tensor, whose
    address a kernel cannot use."""
    if t is None:
        return None
    if t.device.type != "cuda":
        raise ValueError(f"expected a device tensor, got one on {t.device}")
    return ct.c_void_p(t.data_ptr())
