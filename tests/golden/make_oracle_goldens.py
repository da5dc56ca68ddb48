"""Writes oracle values of the benzene-, naphthalene- and pentacene-sized
workloads (c2, c3, c4) for the GPU parity tests, where the oracle is too slow
to run inside a test.

For one core state per workload (core 0) it stores, from `oracle/` alone:

* Sigma^c_n(w_j) = -I_n(w_j) + R_n(w_j) at a few grid points (section
  "Self-energy evaluation", Eqs. cd_terms, cd_imaginary, cd_residue,
  cd_prefactors), with the decoupled Im Sigma there;
* Sigma^c_n(eps_n), Sigma^x_n and E_QP (Eqs. sigma_x, QPGWC);
* optionally Im Sigma^dec_n on the whole real grid (Eq.
  cd_sigma_imaginary_decoupled), the input of the cumulant spectral function.

Inputs come from `workloads` (seeded); a digest of the energies and of a slice
of M_ov is stored so that a test can tell when the generator has changed.

    python tests/golden/make_oracle_goldens.py c2 c3 c4

Run on the CPU; c4 takes about two hours on 8 cores.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import sigma as OS  # noqa: E402
from workloads import CONFIGS, system_from_config  # noqa: E402

# per workload: grid points with Sigma^c, and whether Im Sigma^dec is stored on
# the whole grid
PLAN = {
    "c2": {"points": [0, 200], "dec_grid": True},
    "c3": {"points": [0, 200], "dec_grid": True},
    "c4": {"points": [300], "dec_grid": False},
}


def digest(s):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(s.eps).tobytes())
    h.update(np.ascontiguousarray(s.M_ov[:, 0, :8]).tobytes())
    h.update(np.ascontiguousarray(s.M_oo[:, 0, :]).tobytes())
    return h.hexdigest()


def path_for(name):
    return os.path.join(HERE, f"oracle_{name}_core0.json")


def make(name):
    plan = PLAN[name]
    t_start = time.perf_counter()
    s = system_from_config(CONFIGS[name])
    c = 0
    n = int(s.core_idx[c])
    L = OS.ov_matrix(s.M_ov)
    d = OS.transition_energies(s.eps, s.n_occ)
    W = OS.w_imag_axis(L, d, s.M_oo, s.M_ov, [n], s.omega_imag)[0]
    print(f"{name}: imaginary axis done ({time.perf_counter() - t_start:.0f} s)", flush=True)
    points = []
    for j in plan["points"]:
        w = float(s.omega_real[c, j])
        sc, imd, _ = OS.sigma_c_at(L, d, s.eps, s.occ, s.M_oo, s.M_ov, n, w, s.eta, W,
                                   s.omega_imag, s.w_imag)
        points.append({"j": j, "omega": w, "sigma_c": [sc.real, sc.imag], "im_sigma_dec": imd})
        print(f"{name}: point {j} done ({time.perf_counter() - t_start:.0f} s)", flush=True)
    s_eps, _, _ = OS.sigma_c_at(L, d, s.eps, s.occ, s.M_oo, s.M_ov, n, float(s.eps[n]), s.eta, W,
                                s.omega_imag, s.w_imag)
    sx = OS.exchange(s.M_oo, n)
    e_qp = float(s.eps[n]) + sx + float(s_eps.real)
    print(f"{name}: E_QP done ({time.perf_counter() - t_start:.0f} s)", flush=True)
    rec = {
        "workload": name,
        "core": c,
        "orbital": n,
        "inputs_sha256": digest(s),
        "points": points,
        "sigma_c_eps": [s_eps.real, s_eps.imag],
        "sigma_x": sx,
        "e_qp": e_qp,
    }
    if plan["dec_grid"]:
        im = np.zeros(s.omega_real.shape[1])
        for j in range(im.size):
            _, terms = OS.residue(L, d, s.eps, s.occ, s.M_oo, s.M_ov, n, float(s.omega_real[c, j]),
                                  s.eta, m_subset=[n])
            im[j] = OS.im_decoupled(terms, [n])
        rec["im_sigma_dec_grid"] = [float(x) for x in im]
        print(f"{name}: Im Sigma^dec grid done ({time.perf_counter() - t_start:.0f} s)", flush=True)
    rec["oracle_seconds"] = round(time.perf_counter() - t_start, 1)
    with open(path_for(name), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(f"wrote {path_for(name)}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or ["c2", "c3", "c4"]:
        make(name)
