"""Oracle: G0W0 correlation self-energy of a core state by contour deformation.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy/SciPy in
float64; every step follows the paper's order.

Readings of the paper used here (it cites the RI working equations instead of
printing them):
* Closed-shell RI polarisability, Pi_PQ(z) = sum_ia M^P_ia M^Q_ia chi_ia(z) with
  chi_ia(z) = 2 (f_i - f_a) Delta_ia / (z^2 - Delta_ia^2), f_i = 2, f_a = 0,
  Delta_ia = eps_a - eps_i > 0.  On the imaginary axis z = i w this is
  -4 Delta / (w^2 + Delta^2), so Pi(i w) is negative semidefinite.
* Correlation part of the screened interaction between the pair (n, m),
  W^c_nm(z) = b_nm^T [(1 - Pi(z))^-1 - 1] b_nm with b_nm = M_nm (length N_aux).
* The imaginary-axis integral (Eq. cd_imaginary) is evaluated with eta -> 0 in
  the integrand; W(i w) is real and even in w, so only the even part
  a / (a^2 + w^2) of the propagator survives and the integral is folded onto
  (0, inf):  I_n(w) = (1/pi) sum_m int_0^inf dw' W^c_nm(i w') a/(a^2 + w'^2),
  a = w - eps_m.  The term is 0 when a == 0 exactly.
* Residue prefactors (Eq. cd_prefactors) use Theta(0) = 1/2: f_m = -1 for an
  occupied m with eps_m > w, -1/2 when eps_m == w, and +1 (+1/2) for a virtual m
  with eps_m < w (eps_m == w).  This keeps Sigma^c continuous at w = eps_m.
* Exchange (Eq. sigma_x) sums over occupied m only.
* E_QP is Eq. QPGWC: eps_n + Sigma^x_n + Re Sigma^c_n(eps_n) - v^xc_n.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------------------
# RI building blocks
# ----------------------------------------------------------------------------

def ov_matrix(M_ov: np.ndarray) -> np.ndarray:
    """L = M_ov viewed as an N_aux x (N_occ N_virt) matrix, pair index (i, a)."""
    n_aux = M_ov.shape[0]
    return M_ov.reshape(n_aux, -1)


def transition_energies(eps: np.ndarray, n_occ: int) -> np.ndarray:
    """Delta_ia = eps_a - eps_i, flattened with the same (i, a) order as L."""
    return (eps[None, n_occ:] - eps[:n_occ, None]).reshape(-1)


def chi_ov(z: complex, delta: np.ndarray) -> np.ndarray:
    """Closed-shell independent-particle response of every ia pair at complex z:
    2 (f_i - f_a) Delta / (z^2 - Delta^2) with f_i - f_a = 2."""
    z = complex(z)
    return 4.0 * delta / (z * z - delta * delta)


def polarizability(L: np.ndarray, delta: np.ndarray, z: complex) -> np.ndarray:
    """Pi(z) = L diag(chi(z)) L^T  (N_aux x N_aux, complex symmetric)."""
    return (L * chi_ov(z, delta)[None, :]) @ L.T


def polarizability_imag(L: np.ndarray, delta: np.ndarray, w: float) -> np.ndarray:
    """Pi(i w), real: chi = -4 Delta / (w^2 + Delta^2)."""
    chi = -4.0 * delta / (w * w + delta * delta)
    return (L * chi[None, :]) @ L.T


def pair_vector(M_oo: np.ndarray, M_ov: np.ndarray, n: int, m: int) -> np.ndarray:
    """b_nm = M^P_nm for an occupied n and any orbital m (occupied first)."""
    n_occ = M_oo.shape[1]
    if m < n_occ:
        return M_oo[:, n, m]
    return M_ov[:, n, m - n_occ]


def pair_block(M_oo: np.ndarray, M_ov: np.ndarray, n: int) -> np.ndarray:
    """B_n = [b_n0, ..., b_n(N_basis-1)] as an N_aux x N_basis matrix."""
    return np.concatenate([M_oo[:, n, :], M_ov[:, n, :]], axis=1)


def screened_element(L: np.ndarray, delta: np.ndarray, b: np.ndarray, z: complex) -> complex:
    """W^c_nm(z) = b^T (1 - Pi(z))^-1 b - b^T b, with a partial-pivoting LU of the
    complex symmetric matrix 1 - Pi(z)."""
    n_aux = L.shape[0]
    A = np.eye(n_aux, dtype=complex) - polarizability(L, delta, z)
    lu = sla.lu_factor(A, check_finite=False)
    x = sla.lu_solve(lu, b.astype(complex), check_finite=False)
    return complex(b @ x - b @ b)


# ----------------------------------------------------------------------------
# Imaginary axis (Eq. cd_imaginary)
# ----------------------------------------------------------------------------

def w_imag_axis(L, delta, M_oo, M_ov, cores, omega_imag) -> np.ndarray:
    """W^c_nm(i w_k) for every requested core n, every orbital m and every node.

    For each node: Cholesky factor of the SPD matrix 1 - Pi(i w_k), then for
    each core n the solve with B_n.  Returns W[c][m][k] (c indexes `cores`)."""
    n_aux = L.shape[0]
    n_basis = M_oo.shape[1] + M_ov.shape[2]
    W = np.zeros((len(cores), n_basis, len(omega_imag)))
    eye = np.eye(n_aux)
    blocks = [pair_block(M_oo, M_ov, int(n)) for n in cores]
    for k, w in enumerate(omega_imag):
        C = sla.cho_factor(eye - polarizability_imag(L, delta, float(w)), check_finite=False)
        for c, B in enumerate(blocks):
            X = sla.cho_solve(C, B, check_finite=False)
            W[c, :, k] = np.sum(B * X, axis=0) - np.sum(B * B, axis=0)
    return W


def imag_integral(Wn: np.ndarray, eps: np.ndarray, omega_imag: np.ndarray,
                  w_imag: np.ndarray, omega: float) -> float:
    """I_n(omega) = (1/pi) sum_k w_k sum_m W^c_nm(i w_k) a_m / (a_m^2 + w_k^2),
    a_m = omega - eps_m; a term with a_m == 0 is 0.  Wn is [m][k]."""
    a = (omega - eps)[:, None]                       # [m][1]
    g = a / (a * a + omega_imag[None, :] ** 2)       # [m][k]; exactly 0 when a == 0
    return float(np.sum(w_imag[None, :] * Wn * g) / np.pi)


# ----------------------------------------------------------------------------
# Residues (Eqs. cd_residue, cd_prefactors)
# ----------------------------------------------------------------------------

def prefactor(eps_m: float, occupied: bool, omega: float) -> float:
    """f_m of Eq. cd_prefactors with Theta(0) = 1/2."""
    if occupied:
        if eps_m > omega:
            return -1.0
        if eps_m == omega:
            return -0.5
        return 0.0
    if eps_m < omega:
        return 1.0
    if eps_m == omega:
        return 0.5
    return 0.0


def residue_terms(eps, occ, omega, eta, m_subset=None):
    """The residue tasks at one frequency: list of (m, f_m, z = |eps_m - w| + i eta)."""
    out = []
    ms = range(len(eps)) if m_subset is None else m_subset
    for m in ms:
        f = prefactor(float(eps[m]), bool(occ[m] > 0), float(omega))
        if f != 0.0:
            out.append((int(m), f, complex(abs(float(eps[m]) - float(omega)), float(eta))))
    return out


def residue(L, delta, eps, occ, M_oo, M_ov, n, omega, eta, m_subset=None):
    """R_n(omega) = sum_m f_m W^c_nm(|eps_m - omega| + i eta).  Also returns the
    per-m terms f_m W^c_nm as a dict."""
    total = 0.0 + 0.0j
    terms = {}
    for m, f, z in residue_terms(eps, occ, omega, eta, m_subset):
        val = f * screened_element(L, delta, pair_vector(M_oo, M_ov, n, m), z)
        terms[m] = val
        total += val
    return total, terms


# ----------------------------------------------------------------------------
# Exchange and the full self-energy
# ----------------------------------------------------------------------------

def exchange(M_oo: np.ndarray, n: int) -> float:
    """Sigma^x_n = -sum_{i occ} (n i | i n) = -sum_i sum_P (M^P_ni)^2."""
    return float(-np.sum(M_oo[:, n, :] ** 2))


def equivalent_set(n: int, sym_group, n_occ: int) -> list:
    """The symmetry-equivalent core levels of n (Eq.
    sigma_spectral_decoupled_symmetric): every orbital whose label in sym_group
    equals n's non-negative label, in ascending order; just [n] when sym_group is
    None or n's label is negative.  The set must be occupied."""
    if sym_group is None or int(sym_group[n]) < 0:
        return [int(n)]
    g = int(sym_group[n])
    out = [m for m in range(len(sym_group)) if int(sym_group[m]) == g]
    if any(m >= n_occ for m in out):
        raise ValueError("an equivalent set must contain occupied orbitals only")
    return out


def im_decoupled(terms: dict, sym: list) -> float:
    """Decoupled Im Sigma^c_n(omega) = sum_{i in Sym(n)} f_i Im W^c_ni(|eps_i - omega|
    + i eta) (Eqs. cd_sigma_imaginary_decoupled, sigma_spectral_decoupled_symmetric),
    summed in ascending i from the residue terms f_i W^c_ni."""
    total = 0.0
    for m in sym:
        if m in terms:
            total += float(np.imag(terms[m]))
    return total


def sigma_c_at(L, delta, eps, occ, M_oo, M_ov, n, omega, eta, Wn, omega_imag, w_imag, sym=None):
    """Sigma^c_n(omega) = -I_n(omega) + R_n(omega) (Eq. cd_terms) and the decoupled
    imaginary part over the equivalent set `sym` (default [n]; Eqs.
    cd_sigma_imaginary_decoupled, sigma_spectral_decoupled_symmetric).
    Returns (sigma_c, im_sigma_dec, terms)."""
    I = imag_integral(Wn, eps, omega_imag, w_imag, omega)
    R, terms = residue(L, delta, eps, occ, M_oo, M_ov, n, omega, eta)
    im_dec = im_decoupled(terms, [n] if sym is None else sym)
    return -I + R, im_dec, terms


def qp_newton(L, delta, eps, occ, M_oo, M_ov, n, eta, Wn, omega_imag, w_imag, vxc=0.0,
              max_iter=30, tol=1e-8, step=1e-4):
    """The G0W0 quasiparticle equation (Eq. quasiparticle_equation),
    E = eps_n + Sigma^x_n + Re Sigma^c_n(E) - v^xc_n, by Newton's method from
    E = eps_n with the derivative from a centred difference of step h:
    f(E) = E - eps_n - Sigma^x_n - Re Sigma^c_n(E) + v^xc_n,
    f'(E) ~ (f(E + h) - f(E - h)) / (2 h),  E <- E - f(E) / f'(E),
    stopping when |Delta E| < tol.  Returns (E, iterations), iterations = -1 when
    max_iter steps did not converge (E is then the last iterate)."""
    sx = exchange(M_oo, n)
    en = float(eps[n])

    def f(E):
        sc, _, _ = sigma_c_at(L, delta, eps, occ, M_oo, M_ov, n, E, eta, Wn, omega_imag, w_imag)
        return E - en - sx - sc.real + vxc

    E = en
    for it in range(1, max_iter + 1):
        fm, f0, fp = f(E - step), f(E), f(E + step)
        dE = -f0 / ((fp - fm) / (2.0 * step))
        E = E + dE
        if abs(dE) < tol:
            return E, it
    return E, -1


def sigma_core(eps, occ, M_oo, M_ov, core_idx, omega_imag, w_imag, omega_real, eta,
               vxc=None, mode: str = "full", sym_group=None, qp=None):
    """Full oracle for the `gwc_sigma_core` entry point.

    mode "full": Sigma^c_n on every real grid point (all residue terms);
    mode "decoupled": only the residues of n's equivalent set on the grid
    (gives ImSigma^dec; the set is [n] unless sym_group labels equivalent core
    levels), plus the full Sigma^c_n(eps_n) for E_QP.  Returns a dict with sigma_c
    [n_core][n_real] complex (None in decoupled mode), im_sigma_dec
    [n_core][n_real], sigma_c_eps [n_core] complex, sigma_x, e_qp [n_core]; with
    qp = dict(max_iter, tol, step) also e_qp_newton and qp_iterations [n_core]
    (the G0W0 quasiparticle equation by Newton's method, qp_newton)."""
    eps = np.asarray(eps, dtype=float)
    occ = np.asarray(occ, dtype=float)
    n_occ = M_oo.shape[1]
    L = ov_matrix(M_ov)
    delta = transition_energies(eps, n_occ)
    cores = [int(n) for n in core_idx]
    omega_real = np.asarray(omega_real, dtype=float).reshape(len(cores), -1)
    n_real = omega_real.shape[1]
    vxc = np.zeros(len(cores)) if vxc is None else np.asarray(vxc, dtype=float)

    W = w_imag_axis(L, delta, M_oo, M_ov, cores, omega_imag)
    sigma_c = np.zeros((len(cores), n_real), dtype=complex) if mode == "full" else None
    im_dec = np.zeros((len(cores), n_real))
    sigma_c_eps = np.zeros(len(cores), dtype=complex)
    sigma_x = np.zeros(len(cores))
    e_qp = np.zeros(len(cores))
    for c, n in enumerate(cores):
        sym = equivalent_set(n, sym_group, n_occ)
        for j in range(n_real):
            w = float(omega_real[c, j])
            if mode == "full":
                s, d, _ = sigma_c_at(L, delta, eps, occ, M_oo, M_ov, n, w, eta, W[c],
                                     omega_imag, w_imag, sym=sym)
                sigma_c[c, j] = s
                im_dec[c, j] = d
            else:
                _, terms = residue(L, delta, eps, occ, M_oo, M_ov, n, w, eta, m_subset=sym)
                im_dec[c, j] = im_decoupled(terms, sym)
        s_eps, _, _ = sigma_c_at(L, delta, eps, occ, M_oo, M_ov, n, float(eps[n]), eta, W[c],
                                 omega_imag, w_imag)
        sigma_c_eps[c] = s_eps
        sigma_x[c] = exchange(M_oo, n)
        e_qp[c] = float(eps[n]) + sigma_x[c] + float(np.real(s_eps)) - vxc[c]
    out = dict(sigma_c=sigma_c, im_sigma_dec=im_dec, sigma_c_eps=sigma_c_eps,
               sigma_x=sigma_x, e_qp=e_qp, w_imag=W)
    if qp is not None:
        res = [qp_newton(L, delta, eps, occ, M_oo, M_ov, n, eta, W[c], omega_imag, w_imag,
                         float(vxc[c]), qp["max_iter"], qp["tol"], qp["step"])
               for c, n in enumerate(cores)]
        out["e_qp_newton"] = np.array([r[0] for r in res])
        out["qp_iterations"] = np.array([r[1] for r in res])
    return out


def sigma_core_system(sys, mode: str = "full", sym_group=None, qp=None):
    """Convenience wrapper taking an object with the ABI's fields as attributes."""
    return sigma_core(sys.eps, sys.occ, sys.M_oo, sys.M_ov, sys.core_idx, sys.omega_imag,
                      sys.w_imag, sys.omega_real, sys.eta, vxc=getattr(sys, "vxc", None),
                      mode=mode, sym_group=sym_group, qp=qp)


def count_residue_tasks(eps, occ, core_idx, omega_real, mode: str = "full",
                        sym_group=None) -> int:
    """Number of (n, w, m) residue terms the path evaluates (grid plus w = eps_n)."""
    total = 0
    n_occ = int(np.sum(np.asarray(occ) > 0))
    omega_real = np.asarray(omega_real).reshape(len(core_idx), -1)
    for c, n in enumerate(core_idx):
        n = int(n)
        sym = equivalent_set(n, sym_group, n_occ)
        for w in omega_real[c]:
            if mode == "full":
                total += len(residue_terms(eps, occ, float(w), 0.0))
            else:
                total += len(residue_terms(eps, occ, float(w), 0.0, m_subset=sym))
        total += len(residue_terms(eps, occ, float(eps[n]), 0.0))
    return total
