"""Oracle: numerical GW+C spectral function of one core state.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy in float64.

Steps, in the paper's order (section "Numerical GW+C scheme"):
1. the truncated Landau cumulant (Eq. landau_cumulant_truncated)
       C~(t) = (1/pi) int dw |Im Sigma^c_n(w + eps_n)| / w^2 (e^{-i w t} - 1),
   evaluated as a trapezoid sum over the supplied real grid (Im Sigma is zero
   outside it), nu_j = w_j - eps_n, with the nu_j = 0 term set to 0;
2. the cumulant propagator in time (Eq. cumulant_propagator_numerical_time)
       G^C(t) = G^QP_0(t) e^{C~(t)},  G^QP_0(t) = -i Theta(t) e^{-i E_QP t - eta t}
   (retarded quasiparticle propagator with the broadening of Eq. eq:GQP);
3. the Fourier transform to frequency by FFT (Eqs. cumulant_propagator_fourier
   and cumulant_propagator_convolution: the time-domain product is the
   convolution of the two frequency-domain factors);
4. A(w) = -Im G^C(w) / pi (Eq. eq:AGWC), and Z = exp(-sum_j c_j), the weight of
   the quasiparticle peak, with 1 - Z the total satellite weight.

Discretisation (the paper gives n_t = n_FFT and the energy resolution only):
dt = 2 pi / (n_t d_omega), t_k = k dt for k < n_t, Theta(0) = 1/2 at t_0, and
G(w_l) = dt sum_k G_k e^{i w_l t_k} on w_l = omega_out_min + l d_omega.
"""
from __future__ import annotations

import numpy as np


def trapezoid_weights(x: np.ndarray) -> np.ndarray:
    """q_j with sum_j q_j f(x_j) the trapezoid rule on the (increasing) grid x."""
    x = np.asarray(x, dtype=float)
    q = np.zeros_like(x)
    if x.size < 2:
        return q
    h = np.diff(x)
    q[:-1] += 0.5 * h
    q[1:] += 0.5 * h
    return q


def cumulant_weights(omega_real, im_sigma, eps_n):
    """(nu_j, c_j) with c_j = q_j |Im Sigma_j| / (pi nu_j^2), c_j = 0 where nu_j = 0."""
    omega_real = np.asarray(omega_real, dtype=float)
    nu = omega_real - float(eps_n)
    g = np.abs(np.asarray(im_sigma, dtype=float)) / np.pi
    q = trapezoid_weights(omega_real)
    nz = nu != 0.0
    c = np.zeros_like(nu)
    c[nz] = q[nz] * g[nz] / (nu[nz] * nu[nz])
    return nu, c


def landau_cumulant(nu: np.ndarray, c: np.ndarray, t: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """C~(t_k) = sum_j c_j (exp(-i nu_j t_k) - 1), chunked over t."""
    out = np.empty(t.shape[0], dtype=complex)
    for s in range(0, t.shape[0], chunk):
        tt = t[s:s + chunk]
        out[s:s + chunk] = (np.exp(-1j * tt[:, None] * nu[None, :]) - 1.0) @ c
    return out


def time_grid(n_t: int, d_omega: float):
    dt = 2.0 * np.pi / (n_t * d_omega)
    return dt, np.arange(n_t) * dt


def propagator_time(ctilde: np.ndarray, t: np.ndarray, e_qp: float, eta: float) -> np.ndarray:
    """G_k = -i theta_k exp(-i E_QP t_k - eta t_k) exp(C~(t_k)), theta_0 = 1/2."""
    theta = np.ones_like(t)
    theta[0] = 0.5
    return -1j * theta * np.exp(-1j * e_qp * t - eta * t) * np.exp(ctilde)


def to_frequency(G: np.ndarray, t: np.ndarray, dt: float, omega_out_min: float) -> np.ndarray:
    """G(w_l) = dt sum_k G_k exp(i w_l t_k), w_l = omega_out_min + l d_omega, for all
    l < n_t (one full period), via exp(i w_l t_k) = exp(i w_0 t_k) exp(2 pi i l k / n_t)."""
    n = G.shape[0]
    return dt * np.fft.ifft(G * np.exp(1j * omega_out_min * t)) * n


def spectral_cumulant(omega_real, im_sigma, eps_n, e_qp, eta, n_t, d_omega, n_out,
                      omega_out_min):
    """Oracle for the `gwc_spectral_cumulant` entry point.

    Returns (A[n_out], Z, 1 - Z) with A on omega_out_min + l d_omega."""
    nu, c = cumulant_weights(omega_real, im_sigma, eps_n)
    dt, t = time_grid(int(n_t), float(d_omega))
    ct = landau_cumulant(nu, c, t)
    G = propagator_time(ct, t, float(e_qp), float(eta))
    Gw = to_frequency(G, t, dt, float(omega_out_min))
    A = -np.imag(Gw[:int(n_out)]) / np.pi
    Z = float(np.exp(-np.sum(c)))
    return A, Z, 1.0 - Z
