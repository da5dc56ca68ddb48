"""Pins of the fully analytic G0W0 oracle (Eqs. rpa_casida .. sigma_spectral,
A_explicit_real_imaginary, hedin_sigma_spectral) by routes other than its own:
the non-Hermitian Casida problem, an eigenvector-free sum rule, the RI linear
solve and the contour-deformation integral of the CD oracle, the three-level
model's closed form, and the Hedin-shift fixed point."""
import numpy as np
import pytest

import reference_forms as RF
from oracle import analytic as AN
from oracle import sigma as S
from workloads import CONFIGS, mgl_grid, system_from_config
from workloads.configs import small_config


def _tiny(seed=11, n_occ=3, n_virt=5, n_aux=12, n_core=1, **kw):
    return system_from_config(small_config(n_occ=n_occ, n_virt=n_virt, n_aux=n_aux,
                                           n_core=n_core, seed=seed, **kw))


def test_excitations_match_non_hermitian_casida():
    """The symmetric form's Omega and X + Y equal those of the full
    [[A, B], [-B, -A]] problem (a factor slip in C = Delta^2 + 4 Delta^1/2 K
    Delta^1/2 would move every Omega)."""
    s = _tiny(seed=21, n_occ=3, n_virt=6, n_aux=14)
    Om, XpY = AN.rpa_excitations(s.eps, s.n_occ, s.M_ov)
    Om2, XpY2 = RF.casida(s.eps, s.n_occ, s.M_ov)
    assert np.allclose(Om, Om2, rtol=1e-12, atol=0)
    # eigenvectors up to sign (the spectrum is non-degenerate here)
    sgn = np.sign(np.sum(XpY * XpY2, axis=0))
    assert np.allclose(XpY * sgn, XpY2, rtol=0, atol=1e-10)


@pytest.mark.parametrize("n", [0, 1])
def test_moment_sum_rule(n):
    """(X+Y) Omega (X+Y)^T = Delta, so sum_nu Omega^nu (rho^nu_nm)^2 =
    2 sum_ia (nm|ia)^2 Delta_ia for every m, without eigenvectors."""
    s = _tiny(seed=23, n_occ=4, n_virt=7, n_aux=16, n_core=2)
    Om, XpY = AN.rpa_excitations(s.eps, s.n_occ, s.M_ov)
    rho = AN.transition_moments(s.M_oo, s.M_ov, n, XpY)
    eri = np.concatenate([RF.four_index(s.M_oo, s.M_ov)[n], RF.four_index(s.M_ov, s.M_ov)[n]])
    delta = AN.transition_energies(s.eps, s.n_occ).reshape(s.n_occ, -1)
    ref = 2 * np.einsum("mia,ia->m", eri ** 2, delta)
    assert np.allclose(np.sum(Om[None, :] * rho ** 2, axis=1), ref, rtol=1e-11, atol=0)


def test_static_limit_equals_ri_solve():
    """W^c_nm(0) = -2 sum_nu rho^2 / Omega (Eq. W_spectral at w = 0) equals
    b^T[(1 - Pi(0))^-1 - 1] b from the contour-deformation oracle's RI solve."""
    s = _tiny(seed=25, n_occ=3, n_virt=5, n_aux=12)
    Om, XpY = AN.rpa_excitations(s.eps, s.n_occ, s.M_ov)
    rho = AN.transition_moments(s.M_oo, s.M_ov, 0, XpY)
    L, d = S.ov_matrix(s.M_ov), S.transition_energies(s.eps, s.n_occ)
    for m in range(s.n_basis):
        w0 = S.screened_element(L, d, S.pair_vector(s.M_oo, s.M_ov, 0, m), 0.0)
        assert abs(-2 * np.sum(rho[m] ** 2 / Om) - w0.real) <= 1e-12 * abs(w0)


def test_sigma_equals_contour_deformation_as_eta_vanishes():
    """Sigma^c from the pole sum equals -I + R of the CD oracle (imaginary-axis
    quadrature plus residues) away from poles, below, between and above the
    occupied levels."""
    s = _tiny(seed=31, n_occ=3, n_virt=6, n_aux=14)
    Om, XpY = AN.rpa_excitations(s.eps, s.n_occ, s.M_ov)
    rho = AN.transition_moments(s.M_oo, s.M_ov, 0, XpY)
    L, d = S.ov_matrix(s.M_ov), S.transition_energies(s.eps, s.n_occ)
    x, w = mgl_grid(400, 0.5)
    W = S.w_imag_axis(L, d, s.M_oo, s.M_ov, [0], x)
    eta = 1e-9
    oms = [float(s.eps[0]) - 0.7, float(s.eps[0]) + 1.1, 0.5 * (s.eps[2] + s.eps[3]),
           float(s.eps[4]) + 0.05]
    ps = AN.sigma_c(s.eps, s.n_occ, rho, Om, oms, eta)
    for om, p in zip(oms, ps):
        sc, _, _ = S.sigma_c_at(L, d, s.eps, s.occ, s.M_oo, s.M_ov, 0, om, eta, W[0], x, w)
        assert abs(sc - p) <= 1e-8 * abs(p), om


def test_three_level_model_closed_form():
    """One auxiliary function, core c, valence o, virtual v, (c v) = (c o) = 0:
    Omega^2 = D^2 + 4 m^2 D, rho_cc^2 = 2 b^2 m^2 D / Omega, and Sigma^c_c(w) =
    rho^2 / (w - eps_c + Omega - i eta) (hand-derived)."""
    eps = np.array([-10.6, -0.9, 0.3])
    occ = np.array([2.0, 2.0, 0.0])
    mval, bcc = 0.45, 0.8
    M_ov = np.zeros((1, 2, 1))
    M_ov[0, 1, 0] = mval
    M_oo = np.zeros((1, 2, 2))
    M_oo[0, 0, 0] = bcc
    M_oo[0, 1, 1] = 0.3
    D = eps[2] - eps[1]
    Om = np.sqrt(D * D + 4 * mval * mval * D)
    rho2 = 2 * bcc * bcc * mval * mval * D / Om
    eta = 0.004
    om = np.array([-11.0, -10.6, -10.0])
    r = AN.sigma_analytic(eps, occ, M_oo, M_ov, [0], om[None, :], eta)
    # the core transition c -> v is uncoupled and keeps Omega = eps_v - eps_c
    assert np.allclose(r["omega_exc"], [Om, eps[2] - eps[0]], rtol=1e-14, atol=0)
    ref = rho2 / (om - eps[0] + Om - 1j * eta)
    assert np.allclose(r["sigma_c"][0], ref, rtol=1e-13, atol=0)
    assert abs(r["sigma_x"][0] + bcc * bcc) < 1e-15


def test_hedin_fixed_point_and_definition():
    """A^{G_DH W0} at w = E_QP (that is w + DH_n with w = eps_n) equals
    1 / (pi |Im Sigma^c_n(eps_n)|): the real part of the Dyson denominator
    vanishes there.  Both spectral functions equal |Im G| / pi with G from
    Eq. gw_full_propagator (Eq. A_definition)."""
    s = system_from_config(CONFIGS["c1"])
    om = np.array(s.omega_real)
    om[0, 7] = s.eps[s.core_idx[0]]
    r = AN.sigma_analytic(s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, om, s.eta)
    sce = r["sigma_c_eps"][0]
    assert abs(r["sigma_c"][0, 7] - sce) <= 1e-14 * abs(sce)
    assert abs(r["a_dh"][0, 7] - 1 / (np.pi * abs(sce.imag))) <= 1e-12 * r["a_dh"][0, 7]
    en, sx = s.eps[s.core_idx[0]], r["sigma_x"][0]
    G = 1.0 / (om[0] - en - sx - r["sigma_c"][0])
    assert np.allclose(r["a_gw"][0], np.abs(G.imag) / np.pi, rtol=1e-12, atol=0)
    dh = r["e_qp"][0] - en
    Gdh = 1.0 / (om[0] + dh - en - sx - r["sigma_c"][0])
    assert np.allclose(r["a_dh"][0], np.abs(Gdh.imag) / np.pi, rtol=1e-12, atol=0)


def test_quasiparticle_energy_matches_cd_oracle_on_c1():
    """E_QP (Eq. QPGWC) from the analytic Sigma^c(eps_n) with eta -> 0 equals the
    CD oracle's with a converged imaginary grid (c1 shapes)."""
    s = system_from_config(CONFIGS["c1"])
    x, w = mgl_grid(300, 0.5)
    eta = 1e-8
    cd = S.sigma_core(s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, x, w, s.omega_real[:, :3], eta)
    an = AN.sigma_analytic(s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, s.omega_real[:, :3], eta)
    assert np.allclose(an["e_qp"], cd["e_qp"], rtol=1e-10, atol=0)
    assert np.allclose(an["sigma_x"], cd["sigma_x"], rtol=1e-14, atol=0)
