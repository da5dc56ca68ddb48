"""Pins of the CD-WAC oracle (Eq. pade_approximation) against what the
mathematics fixes: interpolation at the nodes, exact recovery of a rational
function of low order, and equality with contour deformation when the
reference points determine W (for a system with few RPA poles W^c_nm(z) is a
rational function, Eq. W_spectral)."""
import numpy as np

import reference_forms as RF
from oracle import sigma as S
from oracle import wac as WA
from workloads import system_from_config
from workloads.configs import small_config


def test_thiele_interpolates_its_nodes():
    rng = np.random.default_rng(0)
    z = rng.normal(size=14) + 1j * rng.normal(size=14)
    u = rng.normal(size=14) + 1j * rng.normal(size=14)
    a = WA.thiele_fit(z, u)
    for zz, uu in zip(z, u):
        assert abs(WA.thiele_eval(a, z, zz) - uu) <= 1e-12 * abs(uu)


def test_thiele_recovers_a_pole_sum():
    """sum_k r_k [1/(z - O_k) - 1/(z + O_k)] with 3 poles pairs is a (5, 6)
    rational function: 13 or more nodes on the imaginary axis and on the line
    Im z = 0.02 fix it everywhere."""
    Om = np.array([0.5, 1.3, 2.2])
    r = np.array([0.3, 0.1, 0.2])

    def f(z):
        return np.sum(r * (1 / (z - Om) - 1 / (z + Om)))

    for P in (13, 20):
        zn = np.concatenate([1j * np.linspace(0.2, 5, P // 2),
                             np.linspace(0.1, 3, P - P // 2) + 0.02j])
        a = WA.thiele_fit(zn, [f(x) for x in zn])
        for t in (0.7 + 0.02j, 1.9 + 0.02j, 3j, 0.05 + 0.02j, 2.6 + 0.02j):
            assert abs(WA.thiele_eval(a, zn, t) - f(t)) <= 1e-11 * abs(f(t))


def test_fit_of_w_matches_spectral_w():
    """The fitted W^c_nn of a small system equals the Casida spectral W
    (Eq. W_spectral) between the reference points."""
    s = system_from_config(small_config(n_occ=3, n_virt=5, n_aux=12, seed=11))
    L, d = S.ov_matrix(s.M_ov), S.transition_energies(s.eps, s.n_occ)
    Om, XpY = RF.casida_symmetric(s.eps, s.n_occ, s.M_ov)
    rho = RF.transition_moments(s.M_oo, s.M_ov, 0, XpY)
    W = S.w_imag_axis(L, d, s.M_oo, s.M_ov, [0], s.omega_imag)
    xs = np.linspace(0.0, 2.0, 60)
    zr = xs + 1j * s.eta
    vals = np.array([WA.screened_all(L, d, s.M_oo, s.M_ov, 0, z, [0])[0] for z in zr])
    nodes = np.concatenate([1j * s.omega_imag, zr])
    a = WA.thiele_fit(nodes, np.concatenate([W[0, 0].astype(complex), vals]))
    for x in (0.013, 0.41, 0.877, 1.333, 1.99):
        z = x + 1j * s.eta
        exact = RF.w_pole(rho[0], Om, z)
        assert abs(WA.thiele_eval(a, nodes, z) - exact) <= 1e-9 * abs(exact)


def test_wac_equals_cd_when_references_determine_w():
    """15 transitions give W^c_nm rational of order ~30 in z; 80 reference
    points per window fix it, so CD-WAC reproduces the CD self-energy."""
    s = system_from_config(small_config(n_occ=3, n_virt=5, n_aux=12, n_real=9, seed=11))
    cd = S.sigma_core_system(s)
    w = WA.sigma_core_wac(s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, s.omega_imag, s.w_imag,
                          s.omega_real, s.eta, WA.paper_params(80, 80))
    scale = np.max(np.abs(cd["sigma_c"]))
    assert np.max(np.abs(w["sigma_c"] - cd["sigma_c"])) <= 1e-11 * scale
    assert np.max(np.abs(w["im_sigma_dec"] - cd["im_sigma_dec"])) <= 1e-11 * scale
    assert np.allclose(w["e_qp"], cd["e_qp"], rtol=1e-12, atol=0)
    # too few points: the fit is visibly off (the test above is not vacuous)
    w20 = WA.sigma_core_wac(s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, s.omega_imag, s.w_imag,
                            s.omega_real, s.eta, WA.paper_params(20, 20))
    assert np.max(np.abs(w20["sigma_c"] - cd["sigma_c"])) > 1e-4 * scale


def test_wac_decoupled_matches_full_and_windows():
    s = system_from_config(small_config(n_occ=4, n_virt=6, n_aux=14, n_core=2, n_real=6,
                                        seed=17))
    p = WA.paper_params(24, 24)
    args = (s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, s.omega_imag, s.w_imag, s.omega_real,
            s.eta, p)
    full = WA.sigma_core_wac(*args, mode="full")
    dec = WA.sigma_core_wac(*args, mode="decoupled")
    # the valence windows differ between the modes (decoupled places them from the
    # residues at eps_n only); W is smooth there, so E_QP agrees to rounding
    assert np.allclose(full["e_qp"], dec["e_qp"], rtol=1e-10, atol=0)
    # the m = n fit uses the same core-window nodes in both modes
    assert np.allclose(full["im_sigma_dec"], dec["im_sigma_dec"], rtol=0, atol=0)
    pairs, xc, xv = WA.windows(s.eps, s.occ, int(s.core_idx[0]), list(s.omega_real[0]), s.eta, p)
    assert pairs[int(s.core_idx[0])] == "core"
    assert all(pairs[m] == "val" for m in range(s.n_core, s.n_occ))
    assert xc[0] == p["core_min"] and xc[-1] == p["core_max"] and len(xc) == 24
    assert len(xv) == 24 and xv[0] < xv[-1]
