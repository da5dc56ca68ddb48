"""Oracle: the CD-WAC self-energy (contour deformation with W analytically
continued by a Pade approximant).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy/SciPy in
complex128; the steps follow the paper's description of CD-WAC (section
"Numerical GW+C scheme", Eq. pade_approximation):

1. W^c_nm is computed at reference frequencies: the imaginary-axis nodes of
   the I_n quadrature (reused) and real frequencies in a core window and a
   valence window;
2. for every pair (n, m) with residue terms, a continued fraction
   W(z) ~ a_1 / (1 + a_2 (z - z_1) / (1 + a_3 (z - z_2) / (1 + ...)))
   is fitted through its reference points by Thiele's reciprocal-difference
   recursion (the Pade form of Eq. pade_approximation);
3. every residue term f_m W^c_nm(|eps_m - w| + i eta) of R_n takes W from the
   fit; I_n, Sigma^x and E_QP are as in contour deformation.

Readings (the windows are defined in a reference the paper cites):
* a real reference point is z = x + i eta, x the argument |eps_m - w| of the
  residues, so the fit is evaluated on the same line it was fitted on;
* core window: N_C points spaced evenly on [x_C^min, x_C^max]; a pair (n, m)
  belongs to it when every residue argument x of that pair is <= x_C^max;
* valence window (all other pairs of core n): N_V points spaced evenly on
  [(1 - d_lower) x_min, (1 + d_upper) x_max], x_min / x_max the smallest and
  largest residue argument over the valence pairs of n;
* a pair's nodes are the imaginary nodes i w_k (ascending) followed by its
  window's real points (ascending).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import sigma as S


def thiele_fit(z: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Coefficients a_1..a_P of the continued fraction through (z_p, u_p):
    g_1(z_j) = u_j, g_p(z_j) = (g_{p-1}(z_{p-1}) - g_{p-1}(z_j)) /
    ((z_j - z_{p-1}) g_{p-1}(z_j)), a_p = g_p(z_p)."""
    z = np.asarray(z, dtype=complex)
    g = np.array(u, dtype=complex)
    P = len(z)
    a = np.zeros(P, dtype=complex)
    a[0] = g[0]
    for p in range(1, P):
        prev = g[p - 1]
        for j in range(p, P):
            g[j] = (prev - g[j]) / ((z[j] - z[p - 1]) * g[j])
        a[p] = g[p]
    return a


def thiele_eval(a: np.ndarray, z_nodes: np.ndarray, z: complex) -> complex:
    """a_1 / (1 + a_2 (z - z_1) / (1 + ... a_P (z - z_{P-1}))), evaluated from
    the innermost level outwards."""
    P = len(a)
    t = 1.0 + 0.0j
    for p in range(P - 1, 0, -1):
        t = 1.0 + a[p] * (z - z_nodes[p - 1]) / t
    return complex(a[0] / t)


def screened_all(L, delta, M_oo, M_ov, n: int, z: complex, ms) -> np.ndarray:
    """W^c_nm(z) for every m in ms from one LU of 1 - Pi(z)."""
    Pi = S.polarizability(L, delta, z)
    lu = sla.lu_factor(np.eye(Pi.shape[0]) - Pi)
    B = np.stack([S.pair_vector(M_oo, M_ov, n, m) for m in ms], axis=1).astype(complex)
    X = sla.lu_solve(lu, B)
    return np.sum(B * X, axis=0) - np.sum(B * B, axis=0)


def windows(eps, occ, n: int, omegas, eta, params, m_subset_grid=None):
    """Reference windows of core n.  Returns (pairs, x_core, x_val): pairs maps m
    to "core" or "val" for every m with a residue term; x_core / x_val are the
    real reference abscissae (empty when no pair uses the window)."""
    xs = {}
    pts = list(omegas)
    for j, w in enumerate(pts + [float(eps[n])]):
        subset = m_subset_grid if (m_subset_grid is not None and j < len(pts)) else None
        for m, f, z in S.residue_terms(eps, occ, float(w), eta, subset):
            xs.setdefault(m, []).append(z.real)
    pairs = {}
    for m, x in xs.items():
        pairs[m] = "core" if max(x) <= params["core_max"] else "val"
    x_core = np.array([])
    x_val = np.array([])
    if any(v == "core" for v in pairs.values()):
        x_core = np.linspace(params["core_min"], params["core_max"], params["n_core_pts"])
    vals = [x for m, v in pairs.items() if v == "val" for x in xs[m]]
    if vals:
        lo = (1.0 - params["delta_lower"]) * min(vals)
        hi = (1.0 + params["delta_upper"]) * max(vals)
        x_val = np.linspace(lo, hi, params["n_val_pts"])
    return pairs, x_core, x_val


def sigma_core_wac(eps, occ, M_oo, M_ov, core_idx, omega_imag, w_imag, omega_real, eta,
                   params, vxc=None, mode: str = "full", sym_group=None):
    """CD-WAC counterpart of oracle.sigma.sigma_core (same outputs)."""
    eps = np.asarray(eps, dtype=float)
    occ = np.asarray(occ, dtype=float)
    n_occ = M_oo.shape[1]
    L = S.ov_matrix(M_ov)
    delta = S.transition_energies(eps, n_occ)
    cores = [int(n) for n in core_idx]
    omega_real = np.asarray(omega_real, dtype=float).reshape(len(cores), -1)
    n_real = omega_real.shape[1]
    vxc = np.zeros(len(cores)) if vxc is None else np.asarray(vxc, dtype=float)
    omega_imag = np.asarray(omega_imag, dtype=float)

    W = S.w_imag_axis(L, delta, M_oo, M_ov, cores, omega_imag)
    sigma_c = np.zeros((len(cores), n_real), dtype=complex) if mode == "full" else None
    im_dec = np.zeros((len(cores), n_real))
    sigma_c_eps = np.zeros(len(cores), dtype=complex)
    sigma_x = np.zeros(len(cores))
    e_qp = np.zeros(len(cores))
    for c, n in enumerate(cores):
        sym = S.equivalent_set(n, sym_group, n_occ)
        grid = [float(w) for w in omega_real[c]]
        pairs, x_core, x_val = windows(eps, occ, n, grid, eta, params,
                                       None if mode == "full" else sym)
        ms = sorted(pairs)
        ref = {}
        for name, xs in (("core", x_core), ("val", x_val)):
            rows = []
            for x in xs:
                rows.append(screened_all(L, delta, M_oo, M_ov, n, complex(x, eta), ms))
            ref[name] = (np.array([complex(x, eta) for x in xs]), np.array(rows))
        fits = {}
        for i, m in enumerate(ms):
            zr, vals = ref[pairs[m]]
            nodes = np.concatenate([1j * omega_imag, zr])
            u = np.concatenate([W[c, m].astype(complex), vals[:, i]])
            fits[m] = (thiele_fit(nodes, u), nodes)

        def res(w, subset=None):
            total = 0.0 + 0.0j
            terms = {}
            for m, f, z in S.residue_terms(eps, occ, w, eta, subset):
                a, nodes = fits[m]
                terms[m] = f * thiele_eval(a, nodes, z)
                total += terms[m]
            return total, terms

        for j, w in enumerate(grid):
            if mode == "full":
                R, terms = res(w)
                sigma_c[c, j] = -S.imag_integral(W[c], eps, omega_imag, w_imag, w) + R
            else:
                _, terms = res(w, sym)
            im_dec[c, j] = S.im_decoupled(terms, sym)
        R, _ = res(float(eps[n]))
        s_eps = -S.imag_integral(W[c], eps, omega_imag, w_imag, float(eps[n])) + R
        sigma_c_eps[c] = s_eps
        sigma_x[c] = S.exchange(M_oo, n)
        e_qp[c] = float(eps[n]) + sigma_x[c] + float(np.real(s_eps)) - vxc[c]
    return dict(sigma_c=sigma_c, im_sigma_dec=im_dec, sigma_c_eps=sigma_c_eps,
                sigma_x=sigma_x, e_qp=e_qp, w_imag=W)


def paper_params(n_core_pts: int = 100, n_val_pts: int = 100) -> dict:
    """The paper's CD-WAC settings (section "Computational Details"): 100 core and
    100 valence points, core window 0..40 eV, valence margins 8 % below and 1 %
    above (Hartree units)."""
    ev = 27.211386245988
    return dict(n_core_pts=n_core_pts, core_min=0.0, core_max=40.0 / ev, n_val_pts=n_val_pts,
                delta_lower=0.08, delta_upper=0.01)
