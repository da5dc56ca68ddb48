"""Independent references that pin the oracle (tests only).

Nothing here reuses the oracle's route.  The oracle evaluates W through the RI
polarisability and a linear solve, and Sigma^c by contour deformation; these
helpers take the paper's other route: the Casida eigenproblem (Eqs.
rpa_casida, rpa_matrices), transition moments (Eq. density_shifts), the
spectral form of W^c (Eq. W_spectral) and the fully analytic pole sum of
Sigma^c (Eq. sigma_spectral), all built from explicit four-index integrals.

Closed-shell spin adaptation (the paper's equations are in spin orbitals):
the singlet block is A = Delta + 2 (ia|jb), B = 2 (ia|bj); the singlet
transition density carries a factor sqrt(2), rho^nu_mn = sqrt(2) sum_ia
(mn|ia) (X + Y)^nu_ia; triplets have no density and do not screen.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def four_index(M_left: np.ndarray, M_right: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum_P M^P_pq M^P_rs for two stacks M[P][p][q], M[P][r][s]."""
    return np.einsum("Ppq,Prs->pqrs", M_left, M_right)


def casida(eps, n_occ, M_ov):
    """Positive RPA excitation energies Omega^nu and (X+Y)^nu from the full
    non-Hermitian Casida problem [[A, B], [-B, -A]] (Eq. rpa_casida), normalised
    by X^T X - Y^T Y = 1.  Returns (Omega[nu], XpY[ia][nu])."""
    n_virt = M_ov.shape[2]
    delta = (eps[None, n_occ:] - eps[:n_occ, None]).reshape(-1)
    K = four_index(M_ov, M_ov).reshape(n_occ * n_virt, n_occ * n_virt)  # (ia|jb)
    A = np.diag(delta) + 2.0 * K
    B = 2.0 * K  # (ia|bj) = (ia|jb) for real orbitals
    H = np.block([[A, B], [-B, -A]])
    w, V = sla.eig(H)
    w = np.real(w)
    V = np.real(V)
    keep = w > 0
    w, V = w[keep], V[:, keep]
    order = np.argsort(w)
    w, V = w[order], V[:, order]
    nov = delta.size
    X, Y = V[:nov], V[nov:]
    norm = np.sum(X * X, axis=0) - np.sum(Y * Y, axis=0)
    X = X / np.sqrt(norm)[None, :]
    Y = Y / np.sqrt(norm)[None, :]
    return w, X + Y


def casida_symmetric(eps, n_occ, M_ov):
    """Same excitations via the symmetric form (A-B)^1/2 (A+B) (A-B)^1/2 Z = Omega^2 Z,
    X + Y = (A-B)^1/2 Z Omega^-1/2.  Usable for larger N_ov than `casida`."""
    n_virt = M_ov.shape[2]
    delta = (eps[None, n_occ:] - eps[:n_occ, None]).reshape(-1)
    L = M_ov.reshape(M_ov.shape[0], -1)
    K = L.T @ L
    sd = np.sqrt(delta)
    C = np.diag(delta * delta) + 4.0 * (sd[:, None] * K * sd[None, :])
    w2, Z = np.linalg.eigh(C)
    Om = np.sqrt(w2)
    XpY = sd[:, None] * Z / np.sqrt(Om)[None, :]
    return Om, XpY


def transition_moments(M_oo, M_ov, n, XpY):
    """rho^nu_nm for one n and all m: sqrt(2) sum_ia (nm|ia) (X+Y)^nu_ia (Eq.
    density_shifts, singlet).  Returns rho[m][nu]."""
    n_occ = M_oo.shape[1]
    Bn = np.concatenate([M_oo[:, n, :], M_ov[:, n, :]], axis=1)  # [P][m]
    L = M_ov.reshape(M_ov.shape[0], -1)                           # [P][ia]
    nm_ia = Bn.T @ L                                              # (nm|ia)
    return np.sqrt(2.0) * nm_ia @ XpY


def w_pole(rho_m, Om, z):
    """Eq. W_spectral with the broadening folded into complex z:
    W^c_nm(z) = sum_nu rho^2 [1/(z - Omega) - 1/(z + Omega)]."""
    z = np.asarray(z, dtype=complex)
    r2 = rho_m ** 2
    return np.sum(r2 * (1.0 / (z[..., None] - Om) - 1.0 / (z[..., None] + Om)), axis=-1)


def sigma_pole_sum(eps, n_occ, rho, Om, omega, eta):
    """Fully analytic Sigma^c_n(omega), Eq. sigma_spectral:
    sum_{m,nu} rho^2 / (omega - eps_m + (Omega - i eta) sgn(eps_F - eps_m))."""
    sgn = np.where(np.arange(len(eps)) < n_occ, 1.0, -1.0)
    den = omega - eps[:, None] + (Om[None, :] - 1j * eta) * sgn[:, None]
    return complex(np.sum(rho ** 2 / den))


def cd_closed_form(eps, n_occ, rho, Om, omega, eta):
    """Contour-deformation value with an exact imaginary-axis integral:
    -I + R, I = -sum_{m,nu} rho^2 sgn(a)/(|a| + Omega) (a = omega - eps_m,
    0 when a = 0), R = sum_m f_m W_pole(|eps_m - omega| + i eta), f_m with
    Theta(0) = 1/2.  Derived from Eqs. cd_terms..cd_prefactors with the spectral
    W of Eq. W_spectral using int_0^inf dx/((x^2+a^2)(x^2+W^2)) = pi/(2|a|W(|a|+W))."""
    a = omega - eps
    I = -np.sum(rho ** 2 * (np.sign(a)[:, None] / (np.abs(a)[:, None] + Om[None, :])))
    R = 0.0 + 0.0j
    for m in range(len(eps)):
        occ = m < n_occ
        if occ:
            f = -1.0 if eps[m] > omega else (-0.5 if eps[m] == omega else 0.0)
        else:
            f = 1.0 if eps[m] < omega else (0.5 if eps[m] == omega else 0.0)
        if f != 0.0:
            R += f * complex(w_pole(rho[m], Om, abs(eps[m] - omega) + 1j * eta))
    return complex(-I + R), complex(-I), complex(R)
