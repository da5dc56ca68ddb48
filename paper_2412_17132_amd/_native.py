"""ctypes declarations of the libgwc C ABI (include/gwc.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  The library must have been built (``__graft_entry__.build()``);
loading fails loudly otherwise -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_double, c_int, c_int32, c_void_p

LIB_NAME = "libgwc.so"
LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), LIB_NAME)

GWC_OK = 0
STATUS_NAMES = {
    0: "GWC_OK",
    -1: "GWC_ERR_INVALID_ARG",
    -2: "GWC_ERR_SHAPE",
    -3: "GWC_ERR_NONPOSITIVE_GAP",
    -4: "GWC_ERR_NONFINITE",
    -5: "GWC_ERR_FACTORIZATION",
    -6: "GWC_ERR_OUT_OF_MEMORY",
    -7: "GWC_ERR_DEVICE",
    -8: "GWC_ERR_UNSUPPORTED",
}
MODES = {"full": 0, "decoupled": 1}
PRECISIONS = {"fp64": 0, "bf16x3": 1, "fp16x3": 2, "fp8": 3}

EXPORTED_SYMBOLS = (
    "gwc_sigma_core",
    "gwc_spectral_cumulant",
    "gwc_spectral_cumulant_noalloc",
    "gwc_last_error",
    "gwc_version",
    "gwc_timing_enable",
    "gwc_timing_get",
    "gwc_system_create",
    "gwc_system_destroy",
    "gwc_sigma_core_resident",
    "gwc_server_create",
    "gwc_server_submit",
    "gwc_server_wait",
    "gwc_server_stats",
    "gwc_server_destroy",
    "gwc_probe_peak",
    "gwc_sigma_analytic",
    "gwc_evgw0",
)


class GwcSystem(Structure):
    _fields_ = [
        ("n_aux", c_int32), ("n_occ", c_int32), ("n_virt", c_int32),
        ("eps", c_void_p), ("occ", c_void_p), ("M_oo", c_void_p), ("M_ov", c_void_p),
    ]


class GwcWacParams(Structure):
    _fields_ = [
        ("n_core_pts", c_int32), ("core_min", c_double), ("core_max", c_double),
        ("n_val_pts", c_int32), ("delta_lower", c_double), ("delta_upper", c_double),
    ]


class GwcQpParams(Structure):
    _fields_ = [("max_iter", c_int32), ("tol", c_double), ("step", c_double)]


class GwcSigmaArgs(Structure):
    _fields_ = [
        ("n_core", c_int32), ("core_idx", c_void_p),
        ("n_imag", c_int32), ("omega_imag", c_void_p), ("w_imag", c_void_p),
        ("n_real", c_int32), ("omega_real", c_void_p),
        ("eta", c_double), ("vxc", c_void_p),
        ("mode", c_int32), ("precision", c_int32),
        ("sym_group", c_void_p), ("wac", c_void_p), ("qp", c_void_p),
    ]


class GwcSigmaOut(Structure):
    _fields_ = [
        ("sigma_c", c_void_p), ("im_sigma_dec", c_void_p), ("sigma_c_eps", c_void_p),
        ("sigma_x", c_void_p), ("e_qp", c_void_p), ("e_qp_newton", c_void_p),
        ("qp_iterations", c_void_p),
    ]


class GwcAnalyticArgs(Structure):
    _fields_ = [
        ("n_core", c_int32), ("core_idx", c_void_p), ("n_real", c_int32),
        ("omega_real", c_void_p), ("eta", c_double), ("vxc", c_void_p),
    ]


class GwcAnalyticOut(Structure):
    _fields_ = [
        ("sigma_c", c_void_p), ("sigma_c_eps", c_void_p), ("sigma_x", c_void_p),
        ("e_qp", c_void_p), ("a_gw", c_void_p), ("a_dh", c_void_p), ("omega_exc", c_void_p),
        ("sweeps", c_void_p),
    ]


class GwcEvgwParams(Structure):
    _fields_ = [("max_outer", c_int32), ("tol_outer", c_double), ("max_newton", c_int32),
                ("tol_newton", c_double)]


class GwcEvgwArgs(Structure):
    _fields_ = [
        ("M_vv", c_void_p), ("n_core", c_int32), ("core_idx", c_void_p), ("n_real", c_int32),
        ("omega_real", c_void_p), ("eta", c_double), ("vxc", c_void_p), ("params", c_void_p),
    ]


class GwcEvgwOut(Structure):
    _fields_ = [
        ("e_qp", c_void_p), ("e_first", c_void_p), ("sigma_x", c_void_p), ("sigma_c", c_void_p),
        ("a_ev", c_void_p), ("newton", c_void_p), ("outer", c_void_p),
    ]


class GwcCumulantArgs(Structure):
    _fields_ = [
        ("n_real", c_int32), ("omega_real", c_void_p), ("im_sigma", c_void_p),
        ("eps_n", c_double), ("e_qp", c_double), ("eta", c_double),
        ("n_t", c_int32), ("d_omega", c_double),
        ("n_out", c_int32), ("omega_out_min", c_double),
    ]


class GwcServerConfig(Structure):
    _fields_ = [("n_slots", c_int32), ("hbm_budget_bytes", c_double), ("batch_bytes", c_double)]


class GwcRequest(Structure):
    _fields_ = [
        ("system", c_void_p), ("core_idx", c_int32),
        ("n_imag", c_int32), ("omega_imag", c_void_p), ("w_imag", c_void_p),
        ("n_real", c_int32), ("omega_real", c_void_p),
        ("eta", c_double), ("vxc", c_double), ("mode", c_int32), ("precision", c_int32),
        ("n_t", c_int32), ("d_omega", c_double), ("n_out", c_int32),
        ("omega_out_min_rel", c_double),
    ]


class GwcRequestResult(Structure):
    _fields_ = [
        ("status", c_int32), ("e_qp", c_double), ("sigma_x", c_double),
        ("sigma_c_eps", c_double * 2), ("z", c_double * 2),
        ("im_sigma_dec", c_void_p), ("A", c_void_p), ("sigma_c", c_void_p),
        ("t_submit", c_double), ("t_start", c_double), ("t_end", c_double),
        ("footprint_bytes", c_double),
    ]


class GwcServerStats(Structure):
    _fields_ = [
        ("queued", c_int32), ("active", c_int32), ("peak_active", c_int32),
        ("completed", ctypes.c_longlong), ("in_use_bytes", c_double),
        ("peak_in_use_bytes", c_double), ("budget_bytes", c_double),
        ("kept_bytes", c_double), ("refused", ctypes.c_longlong),
    ]


class GwcError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.status_name}: {message}")


_lib = None


def load(path: str = LIB_PATH):
    """Load libgwc (once).  torch is imported first so that the library binds
    to the same HIP runtime instance as torch's allocator and streams."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(the GPU path has no fallback)")
    import torch  # noqa: F401  (one HIP runtime per process)
    lib = ctypes.CDLL(path)
    lib.gwc_sigma_core.argtypes = [POINTER(GwcSystem), POINTER(GwcSigmaArgs),
                                   POINTER(GwcSigmaOut), c_void_p]
    lib.gwc_sigma_core.restype = c_int
    lib.gwc_spectral_cumulant.argtypes = [POINTER(GwcCumulantArgs), c_void_p, c_void_p, c_void_p]
    lib.gwc_spectral_cumulant.restype = c_int
    lib.gwc_spectral_cumulant_noalloc.argtypes = [POINTER(GwcCumulantArgs), c_void_p, c_void_p,
                                                  c_void_p]
    lib.gwc_spectral_cumulant_noalloc.restype = c_int
    lib.gwc_last_error.argtypes = []
    lib.gwc_last_error.restype = ctypes.c_char_p
    lib.gwc_version.argtypes = []
    lib.gwc_version.restype = c_int
    lib.gwc_timing_enable.argtypes = [c_int]
    lib.gwc_timing_enable.restype = c_int
    lib.gwc_timing_get.argtypes = [ctypes.c_char_p, POINTER(c_double), POINTER(ctypes.c_longlong),
                                   POINTER(c_double)]
    lib.gwc_timing_get.restype = c_int
    lib.gwc_system_create.argtypes = [POINTER(GwcSystem), POINTER(c_void_p)]
    lib.gwc_system_create.restype = c_int
    lib.gwc_system_destroy.argtypes = [c_void_p]
    lib.gwc_system_destroy.restype = c_int
    lib.gwc_sigma_core_resident.argtypes = [c_void_p, POINTER(GwcSigmaArgs), POINTER(GwcSigmaOut),
                                            c_void_p]
    lib.gwc_sigma_core_resident.restype = c_int
    lib.gwc_server_create.argtypes = [POINTER(GwcServerConfig), POINTER(c_void_p)]
    lib.gwc_server_create.restype = c_int
    lib.gwc_server_submit.argtypes = [c_void_p, POINTER(GwcRequest), POINTER(ctypes.c_int64)]
    lib.gwc_server_submit.restype = c_int
    lib.gwc_server_wait.argtypes = [c_void_p, ctypes.c_int64, POINTER(GwcRequestResult)]
    lib.gwc_server_wait.restype = c_int
    lib.gwc_server_stats.argtypes = [c_void_p, POINTER(GwcServerStats)]
    lib.gwc_server_stats.restype = c_int
    lib.gwc_server_destroy.argtypes = [c_void_p]
    lib.gwc_server_destroy.restype = c_int
    lib.gwc_sigma_analytic.argtypes = [POINTER(GwcSystem), POINTER(GwcAnalyticArgs),
                                       POINTER(GwcAnalyticOut), c_void_p]
    lib.gwc_sigma_analytic.restype = c_int
    lib.gwc_evgw0.argtypes = [POINTER(GwcSystem), POINTER(GwcEvgwArgs), POINTER(GwcEvgwOut),
                              c_void_p]
    lib.gwc_evgw0.restype = c_int
    lib.gwc_probe_peak.argtypes = [c_int, POINTER(c_double), c_void_p]
    lib.gwc_probe_peak.restype = c_int
    _lib = lib
    return lib


def check(status: int):
    if status != GWC_OK:
        msg = _lib.gwc_last_error().decode() if _lib is not None else ""
        raise GwcError(status, msg)
