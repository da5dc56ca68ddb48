"""Oracle: fully analytic G0W0 self-energy of core states and the G0W0 and
G_DH W0 spectral functions.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy in float64.

Steps, in the paper's order (section "GW for core levels", fully analytic
route):
1. RPA excitations (Eqs. rpa_casida, rpa_matrices).  For real orbitals and a
   closed shell (singlet block A = Delta + 2K, B = 2K, K_ia,jb = (ia|jb) =
   sum_P M^P_ia M^P_jb) the problem is solved in its symmetric form
       C Z = Omega^2 Z,  C = (A - B)^1/2 (A + B) (A - B)^1/2 = Delta^2 + 4 Delta^1/2 K Delta^1/2,
   with X + Y = Delta^1/2 Z Omega^-1/2 (a library eigensolver is the step).
2. Transition moments (Eq. density_shifts), singlet spin factor sqrt(2):
       rho^nu_nm = sqrt(2) sum_ia (nm|ia) (X + Y)^nu_ia.
3. Sigma^c_n(w) = sum_{m, nu} (rho^nu_nm)^2 / (w - eps_m + (Omega^nu - i eta) sgn(eps_F - eps_m))
   (Eq. sigma_spectral; sgn = +1 for occupied m, -1 for virtual m).
4. Sigma^x_n = -sum_i (ni|in) over occupied i (Eq. sigma_x); the quasiparticle
   energy of Eq. QPGWC, E_QP = eps_n + Sigma^x_n + Re Sigma^c_n(eps_n) - v^xc_n,
   and the level-specific Hedin shift DH_n = E_QP - eps_n (Eq. hedin_shift).
5. Spectral functions (Eq. A_explicit_real_imaginary, Sigma = Sigma^x + Sigma^c):
       A^G0W0_n(w) = (1/pi) |Im Sigma^c_n(w)| /
                     ((w - eps_n + v^xc_n - Sigma^x_n - Re Sigma^c_n(w))^2 + (Im Sigma^c_n(w))^2)
   and, with Sigma^{c,DH}_n(w) = Sigma^c_n(w - DH_n) (Eq. hedin_sigma_spectral),
   A^{G_DH W0}_n at w + DH_n, that is the same expression with w - eps_n
   replaced by w + DH_n - eps_n and Sigma^c still taken at w.

Pins (tests/test_oracle_analytic.py): the excitations equal those of the
non-Hermitian Casida problem; the moment sum rule
sum_nu Omega^nu (rho^nu_nm)^2 = 2 sum_ia (nm|ia)^2 Delta_ia; the static limit
-2 sum_nu rho^2 / Omega = W^c_nm(0) from the RI linear solve of the contour-
deformation oracle; Sigma^c equals the contour-deformation oracle as
eta -> 0 away from poles; the three-level model's closed form; A^{G_DH W0} at
E_QP equals 1 / (pi |Im Sigma^c_n(eps_n)|); A from Eq. A_definition.
"""
from __future__ import annotations

import numpy as np


def transition_energies(eps: np.ndarray, n_occ: int) -> np.ndarray:
    """Delta_ia = eps_a - eps_i in the row-major (i, a) order."""
    eps = np.asarray(eps, dtype=float)
    return (eps[None, n_occ:] - eps[:n_occ, None]).reshape(-1)


def casida_matrix(eps, n_occ, M_ov):
    """C = Delta^2 + 4 Delta^1/2 K Delta^1/2 (step 1) and Delta."""
    delta = transition_energies(eps, n_occ)
    L = np.asarray(M_ov, dtype=float).reshape(M_ov.shape[0], -1)   # [P][ia]
    sd = np.sqrt(delta)
    V = 2.0 * sd[:, None] * L.T                                    # [ia][P]
    C = V @ V.T
    C[np.diag_indices_from(C)] += delta * delta
    return C, delta


def rpa_excitations(eps, n_occ, M_ov):
    """(Omega[nu] ascending, XpY[ia][nu]) from the symmetric Casida form."""
    C, delta = casida_matrix(eps, n_occ, M_ov)
    lam, Z = np.linalg.eigh(C)
    Om = np.sqrt(lam)
    XpY = np.sqrt(delta)[:, None] * Z / np.sqrt(Om)[None, :]
    return Om, XpY


def transition_moments(M_oo, M_ov, n, XpY):
    """rho^nu_nm for one occupied n and all m (occupied first): rho[m][nu]."""
    Bn = np.concatenate([M_oo[:, n, :], M_ov[:, n, :]], axis=1)   # [P][m] = M^P_nm
    L = M_ov.reshape(M_ov.shape[0], -1)                           # [P][ia]
    return np.sqrt(2.0) * ((Bn.T @ L) @ XpY)


def sigma_c(eps, n_occ, rho, Om, omega, eta):
    """Eq. sigma_spectral at every w in `omega` (array), one state n (rho[m][nu])."""
    eps = np.asarray(eps, dtype=float)
    sgn = np.where(np.arange(eps.size) < n_occ, 1.0, -1.0)
    r2 = rho * rho
    out = np.empty(np.size(omega), dtype=complex)
    for j, w in enumerate(np.atleast_1d(omega)):
        den = (w - eps)[:, None] + (Om[None, :] - 1j * eta) * sgn[:, None]
        out[j] = np.sum(r2 / den)
    return out


def exchange(M_oo, n):
    """Eq. sigma_x over occupied i: -sum_i (ni|in) = -sum_i sum_P (M^P_ni)^2."""
    return -float(np.sum(M_oo[:, n, :] ** 2))


def spectral_function(omega, eps_n, sigma_x, sig_c, vxc=0.0, shift=0.0):
    """Eq. A_explicit_real_imaginary with w replaced by w + shift (shift = DH_n
    gives A^{G_DH W0} at w + DH_n from Sigma^c at w)."""
    omega = np.asarray(omega, dtype=float)
    re = omega + shift - eps_n + vxc - sigma_x - sig_c.real
    im = sig_c.imag
    return np.abs(im) / (np.pi * (re * re + im * im))


def sigma_analytic(eps, occ, M_oo, M_ov, core_idx, omega_real, eta, vxc=None):
    """Oracle for the `gwc_sigma_analytic` entry point.

    omega_real: [n_core][n_real].  Returns a dict with omega_exc [N_ov]
    (ascending), sigma_c [n_core][n_real], sigma_c_eps [n_core], sigma_x,
    e_qp, a_gw and a_dh ([n_core][n_real])."""
    eps = np.asarray(eps, dtype=float)
    n_occ = int(np.sum(np.asarray(occ) > 0))
    omega_real = np.atleast_2d(np.asarray(omega_real, dtype=float))
    n_core = len(core_idx)
    vxc = np.zeros(n_core) if vxc is None else np.asarray(vxc, dtype=float)
    Om, XpY = rpa_excitations(eps, n_occ, M_ov)
    out = {k: [] for k in ("sigma_c", "sigma_c_eps", "sigma_x", "e_qp", "a_gw", "a_dh")}
    for c, n in enumerate(core_idx):
        n = int(n)
        rho = transition_moments(M_oo, M_ov, n, XpY)
        sc = sigma_c(eps, n_occ, rho, Om, omega_real[c], eta)
        sce = sigma_c(eps, n_occ, rho, Om, [eps[n]], eta)[0]
        sx = exchange(M_oo, n)
        eqp = eps[n] + sx + sce.real - vxc[c]
        out["sigma_c"].append(sc)
        out["sigma_c_eps"].append(sce)
        out["sigma_x"].append(sx)
        out["e_qp"].append(eqp)
        out["a_gw"].append(spectral_function(omega_real[c], eps[n], sx, sc, vxc[c]))
        out["a_dh"].append(spectral_function(omega_real[c], eps[n], sx, sc, vxc[c],
                                             shift=eqp - eps[n]))
    res = {k: np.array(v) for k, v in out.items()}
    res["omega_exc"] = Om
    return res


def sigma_analytic_system(sys, vxc=None):
    return sigma_analytic(sys.eps, sys.occ, sys.M_oo, sys.M_ov, sys.core_idx, sys.omega_real,
                          sys.eta, vxc)
