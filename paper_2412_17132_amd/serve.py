"""Binding of the device-resident systems and the request server of libgwc
(gwc_system_create / gwc_sigma_core_resident / gwc_server_*): argument
marshalling only; admission, slots and execution are in the library."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native as N
from .api import _as_arg, _as_out, _stream_handle, qp_arg, wac_arg


class ResidentSystem:
    """A system kept on the device by the library (gwc_system_create)."""

    def __init__(self, eps, occ, M_oo, M_ov):
        lib = N.load()
        n_aux, n_occ, n_virt = (int(s) for s in M_ov.shape)
        keep: list = []
        sys = N.GwcSystem(n_aux, n_occ, n_virt, _as_arg(eps, "f8", keep), _as_arg(occ, "f8", keep),
                          _as_arg(M_oo, "f8", keep), _as_arg(M_ov, "f8", keep))
        h = ctypes.c_void_p()
        N.check(lib.gwc_system_create(sys, ctypes.byref(h)))
        self.handle = h
        self.n_aux, self.n_occ, self.n_virt = n_aux, n_occ, n_virt
        self.eps = np.asarray(eps.cpu() if hasattr(eps, "cpu") else eps, dtype=np.float64).copy()

    @classmethod
    def from_system(cls, s):
        return cls(s.eps, s.occ, s.M_oo, s.M_ov)

    def sigma_core(self, core_idx, omega_imag, w_imag, omega_real, eta, vxc=None, mode="full",
                   precision="fp64", stream=None, sym_group=None, wac=None, qp=None):
        """gwc_sigma_core_resident; outputs as NumPy arrays."""
        lib = N.load()
        keep: list = []
        core_idx = np.ascontiguousarray(core_idx, dtype=np.int32)
        omega_real = np.ascontiguousarray(omega_real, dtype=np.float64).reshape(len(core_idx), -1)
        n_core, n_real = omega_real.shape
        n_imag = len(omega_imag)
        args = N.GwcSigmaArgs(n_core, _as_arg(core_idx, "i4", keep), n_imag,
                              _as_arg(omega_imag, "f8", keep), _as_arg(w_imag, "f8", keep), n_real,
                              _as_arg(omega_real, "f8", keep), float(eta), _as_arg(vxc, "f8", keep),
                              N.MODES[mode], N.PRECISIONS[precision], _as_arg(sym_group, "i4", keep),
                              wac_arg(wac, keep), qp_arg(qp, keep))
        out = {
            "sigma_c": np.empty((n_core, n_real, 2)) if mode == "full" else None,
            "im_sigma_dec": np.empty((n_core, n_real)),
            "sigma_c_eps": np.empty((n_core, 2)),
            "sigma_x": np.empty(n_core),
            "e_qp": np.empty(n_core),
        }
        if qp is not None:
            out["e_qp_newton"] = np.empty(n_core)
            out["qp_iterations"] = np.empty(n_core, dtype=np.int32)
        o = N.GwcSigmaOut(*(_as_out(out.get(k)) for k in
                            ("sigma_c", "im_sigma_dec", "sigma_c_eps", "sigma_x", "e_qp",
                             "e_qp_newton", "qp_iterations")))
        N.check(lib.gwc_sigma_core_resident(self.handle, args, o, _stream_handle(stream)))
        return out

    def close(self):
        if self.handle:
            N.check(N.load().gwc_system_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """gwc_server_*: continuous batching of single-core-state requests."""

    def __init__(self, n_slots=4, hbm_budget_bytes=64 << 30, batch_bytes=0):
        lib = N.load()
        h = ctypes.c_void_p()
        N.check(lib.gwc_server_create(N.GwcServerConfig(int(n_slots), float(hbm_budget_bytes),
                                                        float(batch_bytes)), ctypes.byref(h)))
        self.handle = h
        self._pending = {}

    def submit(self, system: ResidentSystem, core_idx, omega_imag, w_imag, omega_real, eta,
               mode="decoupled", precision="fp64", vxc=0.0, n_t=0, d_omega=0.0, n_out=0,
               omega_out_min_rel=0.0) -> int:
        wi = np.ascontiguousarray(omega_imag, dtype=np.float64)
        ww = np.ascontiguousarray(w_imag, dtype=np.float64)
        wr = np.ascontiguousarray(omega_real, dtype=np.float64)
        rq = N.GwcRequest(system.handle, int(core_idx), len(wi), wi.ctypes.data, ww.ctypes.data,
                          len(wr), wr.ctypes.data, float(eta), float(vxc), N.MODES[mode],
                          N.PRECISIONS[precision], int(n_t), float(d_omega), int(n_out),
                          float(omega_out_min_rel))
        t = ctypes.c_int64()
        N.check(N.load().gwc_server_submit(self.handle, rq, ctypes.byref(t)))
        self._pending[t.value] = (len(wr), int(n_out), mode)
        return t.value

    def wait(self, ticket: int) -> dict:
        n_real, n_out, mode = self._pending.pop(ticket)
        im = np.empty(n_real)
        A = np.empty(max(n_out, 1))
        sc = np.empty((n_real, 2)) if mode == "full" else None
        res = N.GwcRequestResult()
        res.im_sigma_dec = im.ctypes.data
        res.A = A.ctypes.data if n_out > 0 else None
        res.sigma_c = sc.ctypes.data if sc is not None else None
        N.check(N.load().gwc_server_wait(self.handle, int(ticket), ctypes.byref(res)))
        return {
            "e_qp": res.e_qp, "sigma_x": res.sigma_x,
            "sigma_c_eps": complex(res.sigma_c_eps[0], res.sigma_c_eps[1]),
            "z": (res.z[0], res.z[1]), "im_sigma_dec": im, "A": A[:n_out] if n_out > 0 else None,
            "sigma_c": None if sc is None else sc[:, 0] + 1j * sc[:, 1],
            "t_submit": res.t_submit, "t_start": res.t_start, "t_end": res.t_end,
            "footprint_bytes": res.footprint_bytes,
        }

    def stats(self) -> dict:
        st = N.GwcServerStats()
        N.check(N.load().gwc_server_stats(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in N.GwcServerStats._fields_}

    def close(self):
        if self.handle:
            N.check(N.load().gwc_server_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
