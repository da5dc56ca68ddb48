"""Pins of the cumulant oracle: sum rule, Poisson satellites, the paper's
three-level model, and the first-order expansion (Eq. im_sigma_satellites).

The reference for each check is a closed form that does not use the oracle's
FFT: the discrete-time Lorentzian of one exponential mode is summed as a
geometric series.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import cumulant as C
from workloads import EV_PER_HA

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def discrete_line(x, n_t, d_omega, eta):
    """(1/pi) Re[ dt (1/2 + sum_{m=1}^{n_t-1} r^m) ], r = exp((i x - eta) dt): the
    spectral line that the discretised propagator -i theta e^{(i x - eta) t}
    produces at frequency offset x (geometric sum, no FFT)."""
    dt = 2 * np.pi / (n_t * d_omega)
    r = np.exp((1j * np.asarray(x) - eta) * dt)
    s = 0.5 + r * (1 - r ** (n_t - 1)) / (1 - r)
    return np.real(dt * s) / np.pi


def _grid(eps_n, lo_ev=-25.0, n=501):
    return np.linspace(eps_n + lo_ev / EV_PER_HA, eps_n, n)


def test_sum_rule_full_period():
    """sum_l A_l d_omega = 1 over one full FFT period (theta_0 = 1/2, C~(0) = 0)."""
    eps_n, e_qp, eta = -10.6, -11.3, 0.1 / EV_PER_HA
    w = _grid(eps_n)
    im = -0.02 * np.exp(-((w - eps_n + 0.4) / 0.05) ** 2)
    n_t, dw = 2 ** 14, 0.01 / EV_PER_HA
    A, Z, S = C.spectral_cumulant(w, im, eps_n, e_qp, eta, n_t, dw, n_t, e_qp - 60 / EV_PER_HA)
    assert abs(np.sum(A) * dw - 1.0) < 1e-12
    assert 0 < Z < 1 and abs(Z + S - 1) < 1e-15


@pytest.mark.parametrize("c_target", [0.05, 0.4, 1.3])
def test_single_mode_poisson_weights(c_target):
    """Im Sigma nonzero at one grid point nu* = -Omega gives C~(t) = a(e^{i Omega t} - 1)
    and A = e^{-a} sum_k a^k/k! line(w - E_QP + k Omega); the amplitudes found by
    least squares on the exact discrete lines equal e^{-a} a^k / k!."""
    eps_n, e_qp, eta = -10.6, -11.25, 0.1 / EV_PER_HA
    w = _grid(eps_n)
    j = 200
    Om = eps_n - w[j]
    q = C.trapezoid_weights(w)[j]
    im = np.zeros_like(w)
    im[j] = -c_target * np.pi * Om * Om / q      # gives c_j = c_target exactly
    n_t, dw = 2 ** 14, 0.01 / EV_PER_HA
    w0 = e_qp - 120 / EV_PER_HA
    A, Z, _ = C.spectral_cumulant(w, im, eps_n, e_qp, eta, n_t, dw, n_t, w0)
    wl = w0 + np.arange(n_t) * dw
    K = 20
    basis = np.stack([discrete_line(wl - e_qp + k * Om, n_t, dw, eta) for k in range(K)], axis=1)
    amp, *_ = np.linalg.lstsq(basis, A, rcond=None)
    ref = np.array([math.exp(-c_target) * c_target ** k / math.factorial(k) for k in range(K)])
    assert np.max(np.abs(amp - ref)) < 1e-10
    assert abs(Z - math.exp(-c_target)) < 1e-14


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "three_level_model.json")))["cases"])
def test_three_level_model_satellites(case):
    """The paper's three-level model (Fig. model_system): with the decoupled
    Im Sigma of one RPA mode (Omega, rho), GW+C puts satellites at E_QP - k Omega
    with Poisson weights in gamma = rho^2/Omega^2 (golden file).  Tolerances
    cover the finite eta and the truncation of Im Sigma to the grid window."""
    Om = 10.0 / EV_PER_HA
    rho2 = case["gamma"] * Om * Om
    eta = 0.1 / EV_PER_HA
    eps_n, e_qp = -10.6, -11.2
    w = np.linspace(eps_n - 60 / EV_PER_HA, eps_n, 6001)
    x = np.abs(eps_n - w)
    z = x + 1j * eta
    Wcc = rho2 * 2 * Om / (z * z - Om * Om)
    f = np.where(w < eps_n, -1.0, -0.5)
    im = f * np.imag(Wcc)
    n_t, dw = 2 ** 15, 0.01 / EV_PER_HA
    w0 = e_qp - 100 / EV_PER_HA
    A, Z, _ = C.spectral_cumulant(w, im, eps_n, e_qp, eta, n_t, 0.01 / EV_PER_HA, n_t, w0)
    wl = w0 + np.arange(n_t) * dw
    for k, ref in enumerate(case["poisson_weights"][:4]):
        centre = e_qp - k * Om
        win = np.abs(wl - centre) < 0.5 * Om
        weight = np.sum(A[win]) * dw
        assert abs(weight - ref) < 0.03 * max(ref, 0.05), (k, weight, ref)
        if ref > 1e-2:
            peak = wl[win][np.argmax(A[win])]
            assert abs(peak - centre) < 0.03 / EV_PER_HA
    # -ln Z = gamma plus the anti-resonant tail of Im W(x + i eta) near x = 0,
    # (4/pi) gamma (eta/Omega) ln(Omega/grid step) ~ 0.09 gamma here
    assert abs(-math.log(Z) - case["gamma"]) < 0.1 * case["gamma"]


def test_first_order_expansion():
    """Eq. im_sigma_satellites: for weak coupling lambda, A - Z line(w - E_QP)
    approaches Z sum_j c_j line(w - E_QP - nu_j); the residual is O(lambda^2),
    so its ratio to the satellite signal halves with lambda."""
    eps_n, e_qp, eta = -10.6, -11.25, 0.1 / EV_PER_HA
    w = _grid(eps_n, n=301)
    shape = -np.exp(-((w - eps_n + 0.35) / 0.04) ** 2) - 0.5 * np.exp(-((w - eps_n + 0.6) / 0.03) ** 2)
    n_t, dw = 2 ** 13, 0.01 / EV_PER_HA
    w0 = e_qp - 40 / EV_PER_HA
    wl = w0 + np.arange(n_t) * dw
    ratios = []
    for lam in (1e-3, 5e-4):
        im = lam * shape
        A, Z, _ = C.spectral_cumulant(w, im, eps_n, e_qp, eta, n_t, dw, n_t, w0)
        nu, c = C.cumulant_weights(w, im, eps_n)
        sat = Z * sum(cj * discrete_line(wl - e_qp - nj, n_t, dw, eta) for nj, cj in zip(nu, c) if cj)
        resid = A - Z * discrete_line(wl - e_qp, n_t, dw, eta) - sat
        ratios.append(np.max(np.abs(resid)) / np.max(np.abs(sat)))
    assert ratios[0] < 0.05
    assert 1.8 < ratios[0] / ratios[1] < 2.2


def test_trapezoid_weights():
    x = np.array([0.0, 0.1, 0.3, 0.6, 1.0])
    q = C.trapezoid_weights(x)
    assert abs(np.sum(q * x) - 0.5) < 1e-15          # exact for linear functions
    assert abs(np.sum(q) - 1.0) < 1e-15


def literal_route_spectrum(w, im, eps_n, e_qp, eta, omega_out, n_e=2 ** 16, decay_lengths=30.0):
    """A(w) by the paper's frequency-domain route (Eqs. cumulant_propagator_fourier
    and cumulant_propagator_convolution), independent of the oracle's product in
    time: the spectrum of exp(C~(t)) alone, then a numerical convolution with the
    analytic quasiparticle propagator G^QP_0(w) = 1/(w - E_QP + i eta_QP).

    The broadening eta is split as eta/2 on G^QP_0 and a damping exp(-eta|t|/2) on
    exp(C~(t)); their product in time carries exp(-eta t), as the oracle's does.
    exp(C~(t)) is sampled on t in [-T, T), T = decay_lengths / (eta/2), with
    C~(-t) = conj C~(t), and transformed by one FFT:
        E(w'_l) = dt sum_k exp(C~(t_k) - eta |t_k| / 2) exp(i w'_l t_k);
    then G^C(w) = (1/2 pi) sum_l dw' G^QP_0(w - w'_l) E(w'_l)."""
    nu, c = C.cumulant_weights(w, im, eps_n)
    half = 0.5 * eta
    dt = 2 * decay_lengths / half / n_e
    k = np.arange(-n_e // 2, n_e // 2)
    t = k * dt
    f = np.exp(C.landau_cumulant(nu, c, t) - half * np.abs(t))
    dwp = 2 * np.pi / (n_e * dt)
    wp = k * dwp
    E = dt * np.fft.fftshift(np.fft.ifft(np.fft.ifftshift(f))) * n_e
    G = np.empty(len(omega_out), dtype=complex)
    for s in range(0, len(omega_out), 256):
        ww = np.asarray(omega_out[s:s + 256])
        G[s:s + 256] = (1.0 / (ww[:, None] - wp[None, :] - e_qp + 1j * half)) @ E * dwp / (2 * np.pi)
    return -G.imag / np.pi


@pytest.mark.parametrize("amp", [0.02, 0.3])
def test_literal_frequency_route(amp):
    """The oracle's product in time followed by one FFT equals the paper's
    frequency-domain route (FFT of exp(C~), convolution with G^QP_0).

    With Theta(0) = 1/2 the oracle's discrete time sum is exactly the continuous
    transform periodised with period Omega = n_t d_omega (Poisson summation), so
    the two differ by the Lorentzian tails of the periodic images: at most
    (eta/pi) sum_{p != 0} 1/(p Omega - D)^2 < 4 (eta/pi) / (Omega - D)^2 with D
    the largest distance between an output point and the spectral weight.  The
    literal route's own errors (window exp(-30), the FFT's periodic images,
    trapezoid convolution of functions analytic in a strip of width eta/2 on a
    step of eta/60) are orders below that.  A Theta(0) = 1 slip would shift A by
    1/(n_t d_omega) and a sign slip in exp(-i nu t) would mirror the satellites."""
    eps_n, e_qp, eta = -10.6, -11.25, 0.1 / EV_PER_HA
    w = _grid(eps_n, n=401)
    im = -amp * (np.exp(-((w - eps_n + 0.4) / 0.05) ** 2)
                 + 0.5 * np.exp(-((w - eps_n + 0.7) / 0.08) ** 2))
    n_t, dw = 2 ** 15, 0.01 / EV_PER_HA
    w0 = e_qp - 100 / EV_PER_HA
    A, Z, _ = C.spectral_cumulant(w, im, eps_n, e_qp, eta, n_t, dw, n_t, w0)
    wl = w0 + np.arange(n_t) * dw
    idx = np.nonzero((wl > e_qp - 40 / EV_PER_HA) & (wl < e_qp + 10 / EV_PER_HA))[0][::4]
    A_lit = literal_route_spectrum(w, im, eps_n, e_qp, eta, wl[idx])
    D = 40 / EV_PER_HA + (eps_n - w[0])
    bound = 4 * (eta / np.pi) / (n_t * dw - D) ** 2
    err = np.max(np.abs(A_lit - A[idx]))
    assert err < bound, (err, bound)
    # the satellite region carries weight (the comparison is not only the QP peak)
    sat = (wl[idx] < e_qp - 0.2 / EV_PER_HA)
    assert np.sum(A_lit[sat]) * 4 * dw > 0.5 * (1 - Z)
