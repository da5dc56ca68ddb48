"""Python binding of libgwc: the same entry points as the C ABI, argument
marshalling only.

Arrays may be torch tensors (CUDA/HIP device or CPU) or NumPy arrays; device
tensors are passed by pointer, host arrays are staged by the library itself.
Outputs are allocated on the device of `M_ov` unless given.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import _native as N


def _torch():
    import torch
    return torch


def _is_tensor(x) -> bool:
    try:
        return isinstance(x, _torch().Tensor)
    except ImportError:  # pragma: no cover
        return False


def _as_arg(x, dtype: str, keep: list):
    """Pointer of a contiguous array of the given dtype ('f8' or 'i4')."""
    if x is None:
        return None
    if _is_tensor(x):
        torch = _torch()
        want = torch.float64 if dtype == "f8" else torch.int32
        if x.dtype != want or not x.is_contiguous():
            x = x.to(want).contiguous()
        keep.append(x)
        return x.data_ptr()
    arr = np.ascontiguousarray(x, dtype=np.float64 if dtype == "f8" else np.int32)
    keep.append(arr)
    return arr.ctypes.data


def _stream_handle(stream):
    if stream is not None:
        return stream
    torch = _torch()
    if torch.cuda.is_available():
        return torch.cuda.current_stream().cuda_stream
    return None


def _alloc(shape, like, integer=False):
    if _is_tensor(like) and like.is_cuda:
        torch = _torch()
        return torch.empty(shape, dtype=torch.int32 if integer else torch.float64, device=like.device)
    return np.empty(shape, dtype=np.int32 if integer else np.float64)


def gwc_sigma_core(eps, occ, M_oo, M_ov, core_idx, omega_imag, w_imag, omega_real, eta,
                   vxc=None, mode: str = "full", precision: str = "fp64",
                   out: Optional[dict] = None, stream=None, sym_group=None, wac=None,
                   qp=None) -> dict:
    """Sigma^c_n(w) of the core states by contour deformation (gwc_sigma_core).

    sym_group: optional [n_basis] int32 labels of symmetry-equivalent core levels.
    wac: optional dict of CD-WAC settings (n_core_pts, core_min, core_max,
    n_val_pts, delta_lower, delta_upper; Hartree) -- CD-WAC instead of CD.
    qp: optional dict (max_iter, tol, step; Hartree) -- also solve the G0W0
    quasiparticle equation by Newton's method (e_qp_newton, qp_iterations).
    Returns a dict with sigma_c [n_core][n_real][2] (None in decoupled mode),
    im_sigma_dec [n_core][n_real], sigma_c_eps [n_core][2], sigma_x, e_qp."""
    lib = N.load()
    n_aux, n_occ, n_virt = (int(s) for s in M_ov.shape)
    n_core = int(core_idx.shape[0])
    n_imag = int(omega_imag.shape[0])
    n_real = int(omega_real.shape[-1])
    keep: list = []
    sys = N.GwcSystem(n_aux, n_occ, n_virt, _as_arg(eps, "f8", keep), _as_arg(occ, "f8", keep),
                      _as_arg(M_oo, "f8", keep), _as_arg(M_ov, "f8", keep))
    args = N.GwcSigmaArgs(n_core, _as_arg(core_idx, "i4", keep), n_imag,
                          _as_arg(omega_imag, "f8", keep), _as_arg(w_imag, "f8", keep), n_real,
                          _as_arg(omega_real, "f8", keep), float(eta), _as_arg(vxc, "f8", keep),
                          N.MODES[mode], N.PRECISIONS[precision], _as_arg(sym_group, "i4", keep),
                          wac_arg(wac, keep), qp_arg(qp, keep))
    if out is None:
        out = {
            "sigma_c": _alloc((n_core, n_real, 2), M_ov) if mode == "full" else None,
            "im_sigma_dec": _alloc((n_core, n_real), M_ov),
            "sigma_c_eps": _alloc((n_core, 2), M_ov),
            "sigma_x": _alloc((n_core,), M_ov),
            "e_qp": _alloc((n_core,), M_ov),
        }
        if qp is not None:
            out["e_qp_newton"] = _alloc((n_core,), M_ov)
            out["qp_iterations"] = _alloc((n_core,), M_ov, integer=True)
    o = N.GwcSigmaOut(*(_as_out(out.get(k)) for k in
                        ("sigma_c", "im_sigma_dec", "sigma_c_eps", "sigma_x", "e_qp",
                         "e_qp_newton", "qp_iterations")))
    N.check(lib.gwc_sigma_core(sys, args, o, _stream_handle(stream)))
    return out


def gwc_sigma_analytic(eps, occ, M_oo, M_ov, core_idx, omega_real, eta, vxc=None,
                       out: Optional[dict] = None, stream=None) -> dict:
    """Fully analytic G0W0 Sigma^c_n(w) of the core states (gwc_sigma_analytic):
    Casida excitations, transition moments and the pole sum of Eq. sigma_spectral.
    Returns a dict with sigma_c [n_core][n_real][2], sigma_c_eps [n_core][2],
    sigma_x, e_qp, a_gw and a_dh [n_core][n_real], omega_exc [n_occ n_virt]
    (ascending) and sweeps [1] (int32)."""
    lib = N.load()
    n_aux, n_occ, n_virt = (int(s) for s in M_ov.shape)
    n_core = int(core_idx.shape[0])
    n_real = int(omega_real.shape[-1])
    keep: list = []
    sys = N.GwcSystem(n_aux, n_occ, n_virt, _as_arg(eps, "f8", keep), _as_arg(occ, "f8", keep),
                      _as_arg(M_oo, "f8", keep), _as_arg(M_ov, "f8", keep))
    args = N.GwcAnalyticArgs(n_core, _as_arg(core_idx, "i4", keep), n_real,
                             _as_arg(omega_real, "f8", keep), float(eta), _as_arg(vxc, "f8", keep))
    if out is None:
        out = {
            "sigma_c": _alloc((n_core, n_real, 2), M_ov),
            "sigma_c_eps": _alloc((n_core, 2), M_ov),
            "sigma_x": _alloc((n_core,), M_ov),
            "e_qp": _alloc((n_core,), M_ov),
            "a_gw": _alloc((n_core, n_real), M_ov),
            "a_dh": _alloc((n_core, n_real), M_ov),
            "omega_exc": _alloc((n_occ * n_virt,), M_ov),
            "sweeps": np.zeros(1, dtype=np.int32),
        }
    o = N.GwcAnalyticOut(*(_as_out(out.get(k)) for k in
                           ("sigma_c", "sigma_c_eps", "sigma_x", "e_qp", "a_gw", "a_dh",
                            "omega_exc", "sweeps")))
    N.check(lib.gwc_sigma_analytic(sys, args, o, _stream_handle(stream)))
    return out


def gwc_evgw0(eps, occ, M_oo, M_ov, M_vv, core_idx, omega_real, eta, vxc=None, params=None,
              out: Optional[dict] = None, stream=None) -> dict:
    """evGW0 quasiparticle energies of every state (gwc_evgw0, Eq. ev_sigma_spectral).

    vxc: optional [n_basis]; params: optional dict (max_outer, tol_outer,
    max_newton, tol_newton).  Returns a dict with e_qp, e_first, sigma_x
    [n_basis], sigma_c [n_core][n_real][2], a_ev [n_core][n_real], newton
    [n_basis] and outer [1] (int32)."""
    import ctypes
    lib = N.load()
    n_aux, n_occ, n_virt = (int(s) for s in M_ov.shape)
    nb = n_occ + n_virt
    n_core = int(core_idx.shape[0])
    n_real = int(omega_real.shape[-1])
    keep: list = []
    sys = N.GwcSystem(n_aux, n_occ, n_virt, _as_arg(eps, "f8", keep), _as_arg(occ, "f8", keep),
                      _as_arg(M_oo, "f8", keep), _as_arg(M_ov, "f8", keep))
    pp = None
    if params is not None:
        p = N.GwcEvgwParams(int(params["max_outer"]), float(params["tol_outer"]),
                            int(params["max_newton"]), float(params["tol_newton"]))
        keep.append(p)
        pp = ctypes.addressof(p)
    args = N.GwcEvgwArgs(_as_arg(M_vv, "f8", keep), n_core, _as_arg(core_idx, "i4", keep), n_real,
                         _as_arg(omega_real, "f8", keep), float(eta), _as_arg(vxc, "f8", keep), pp)
    if out is None:
        out = {
            "e_qp": _alloc((nb,), M_ov), "e_first": _alloc((nb,), M_ov),
            "sigma_x": _alloc((nb,), M_ov), "sigma_c": _alloc((n_core, n_real, 2), M_ov),
            "a_ev": _alloc((n_core, n_real), M_ov), "newton": _alloc((nb,), M_ov, integer=True),
            "outer": np.zeros(1, dtype=np.int32),
        }
    o = N.GwcEvgwOut(*(_as_out(out.get(k)) for k in
                       ("e_qp", "e_first", "sigma_x", "sigma_c", "a_ev", "newton", "outer")))
    N.check(lib.gwc_evgw0(sys, args, o, _stream_handle(stream)))
    return out


def wac_paper_settings(n_core_pts: int = 100, n_val_pts: int = 100) -> dict:
    """The paper's CD-WAC settings (section "Computational Details"): 100 core-window
    and 100 valence-window points, core window 0..40 eV, valence margins 8 % below
    and 1 % above; energies in Hartree."""
    return dict(n_core_pts=n_core_pts, core_min=0.0, core_max=40.0 / 27.211386245988,
                n_val_pts=n_val_pts, delta_lower=0.08, delta_upper=0.01)


def qp_arg(qp, keep: list):
    """Pointer to a gwc_qp_params built from a dict (None: no Newton solve)."""
    if qp is None:
        return None
    import ctypes
    p = N.GwcQpParams(int(qp["max_iter"]), float(qp["tol"]), float(qp["step"]))
    keep.append(p)
    return ctypes.addressof(p)


def wac_arg(wac, keep: list):
    """Pointer to a gwc_wac_params built from a dict (None: contour deformation)."""
    if wac is None:
        return None
    import ctypes
    p = N.GwcWacParams(int(wac["n_core_pts"]), float(wac["core_min"]), float(wac["core_max"]),
                       int(wac["n_val_pts"]), float(wac["delta_lower"]), float(wac["delta_upper"]))
    keep.append(p)
    return ctypes.addressof(p)


def _as_out(x):
    if x is None:
        return None
    if _is_tensor(x):
        assert x.dtype in (_torch().float64, _torch().int32) and x.is_contiguous()
        return x.data_ptr()
    assert x.dtype in (np.float64, np.int32) and x.flags["C_CONTIGUOUS"]
    return x.ctypes.data


def gwc_spectral_cumulant(omega_real, im_sigma, eps_n, e_qp, eta, n_t, d_omega, n_out,
                          omega_out_min, A_out=None, z_out=None, stream=None):
    """GW+C spectral function of one state (gwc_spectral_cumulant).
    Returns (A [n_out], z [2] = (Z, 1 - Z))."""
    lib = N.load()
    keep: list = []
    n_real = int(omega_real.shape[0])
    args = N.GwcCumulantArgs(n_real, _as_arg(omega_real, "f8", keep), _as_arg(im_sigma, "f8", keep),
                             float(eps_n), float(e_qp), float(eta), int(n_t), float(d_omega),
                             int(n_out), float(omega_out_min))
    if A_out is None:
        A_out = _alloc((int(n_out),), im_sigma)
    if z_out is None:
        z_out = _alloc((2,), im_sigma)
    N.check(lib.gwc_spectral_cumulant(args, _as_out(A_out), _as_out(z_out), _stream_handle(stream)))
    return A_out, z_out


def gwc_spectral_cumulant_noalloc(omega_real, im_sigma, eps_n, e_qp, eta, n_t, d_omega, n_out,
                                  omega_out_min, A_out, z_out=None, stream=None):
    """gwc_spectral_cumulant_noalloc: the same spectral function with no device
    allocation in the library (n_t <= 2^19, n_real <= 2^15).  The caller passes
    the outputs (A_out [n_out], z_out [2] or None); returns (A_out, z_out)."""
    lib = N.load()
    keep: list = []
    n_real = int(omega_real.shape[0])
    args = N.GwcCumulantArgs(n_real, _as_arg(omega_real, "f8", keep), _as_arg(im_sigma, "f8", keep),
                             float(eps_n), float(e_qp), float(eta), int(n_t), float(d_omega),
                             int(n_out), float(omega_out_min))
    N.check(lib.gwc_spectral_cumulant_noalloc(args, _as_out(A_out), _as_out(z_out),
                                              _stream_handle(stream)))
    return A_out, z_out


def to_device(system, device="cuda"):
    """Device-resident copies (torch tensors) of a system's arrays."""
    torch = _torch()

    def t(x, dt=torch.float64):
        return None if x is None else torch.as_tensor(np.ascontiguousarray(x)).to(device=device, dtype=dt)

    return dict(
        eps=t(system.eps), occ=t(system.occ), M_oo=t(system.M_oo), M_ov=t(system.M_ov),
        core_idx=t(system.core_idx, torch.int32), omega_imag=t(system.omega_imag),
        w_imag=t(system.w_imag), omega_real=t(system.omega_real), eta=float(system.eta),
        vxc=t(getattr(system, "vxc", None)),
    )


def timing_enable(on: bool = True) -> None:
    """Clear and (de)activate the per-kernel event timing of libgwc."""
    N.check(N.load().gwc_timing_enable(1 if on else 0))


def timing_get(kernel: str) -> dict:
    """Summed event time (ms), launch count and algorithmic flops of one kernel."""
    import ctypes
    ms, n, fl = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
    N.check(N.load().gwc_timing_get(kernel.encode(), ctypes.byref(ms), ctypes.byref(n),
                                    ctypes.byref(fl)))
    return {"total_ms": ms.value, "launches": n.value, "flops": fl.value}


PROBE_KINDS = {"fp64_mfma": 0, "bf16_mfma": 1, "fp16_mfma": 2, "hbm_copy": 3, "fp8_mfma_k32": 4,
               "fp8_mfma_k128": 5}


def probe_peak(kind: str) -> float:
    """Measured device peak: MFMA TFLOP/s for the *_mfma kinds, GB/s for hbm_copy."""
    import ctypes
    v = ctypes.c_double()
    N.check(N.load().gwc_probe_peak(PROBE_KINDS[kind], ctypes.byref(v), None))
    return v.value


def version() -> int:
    return int(N.load().gwc_version())
