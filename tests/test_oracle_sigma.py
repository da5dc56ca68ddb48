"""Pins of the self-energy oracle against what the paper and the mathematics fix.

Each test uses a route other than the oracle's own: the Casida eigenproblem
and the spectral forms of W and Sigma (`reference_forms`), explicit
four-index integrals, textbook integrals, exact invariants, or a one-mode
model with a hand-derived closed form.
"""
import numpy as np
import pytest

import reference_forms as RF
from oracle import sigma as S
from workloads import CONFIGS, mgl_grid, system_from_config
from workloads.configs import small_config


def _tiny(seed=11, n_occ=3, n_virt=5, n_aux=12, n_core=1, **kw):
    return system_from_config(small_config(n_occ=n_occ, n_virt=n_virt, n_aux=n_aux,
                                           n_core=n_core, seed=seed, **kw))


def _ri(s):
    return S.ov_matrix(s.M_ov), S.transition_energies(s.eps, s.n_occ)


# --- the imaginary-axis grid ---------------------------------------------------

@pytest.mark.parametrize("a", [0.05, 0.5, 3.0, 20.0])
def test_mgl_grid_integrates_lorentzian(a):
    """int_0^inf dx / (x^2 + a^2) = pi / (2a); the mapped Gauss-Legendre rule
    converges to it as the node count grows."""
    errs = []
    for n in (24, 50, 100, 200):
        x, w = mgl_grid(n, 0.5)
        errs.append(abs(np.sum(w / (x * x + a * a)) - np.pi / (2 * a)) / (np.pi / (2 * a)))
    assert errs[-1] < 1e-8
    assert errs[-1] <= max(errs[0], 1e-13)
    x, w = mgl_grid(24, 0.5)
    assert np.all(x > 0) and np.all(w > 0) and np.all(np.diff(x) > 0)


# --- Pi --------------------------------------------------------------------------

def test_pi_imag_axis_negative_semidefinite():
    """Pi(i w) <= 0 for every node (c1 shapes)."""
    s = system_from_config(CONFIGS["c1"])
    L, d = _ri(s)
    for w in s.omega_imag:
        P = S.polarizability_imag(L, d, float(w))
        ev = np.linalg.eigvalsh(P)
        assert ev.max() <= 1e-14 * np.abs(ev).max()
        # the complex-z form agrees with the real form on the imaginary axis
        Pz = S.polarizability(L, d, 1j * float(w))
        assert np.max(np.abs(Pz.imag)) == 0.0
        assert np.allclose(Pz.real, P, rtol=1e-14, atol=1e-16)


def test_pi_explicit_loop():
    """Pi_PQ(z) = sum_ia M^P_ia M^Q_ia 4 Delta_ia / (z^2 - Delta_ia^2) by loops."""
    s = _tiny(n_occ=2, n_virt=3, n_aux=4)
    L, d = _ri(s)
    z = 0.37 + 0.01j
    P = S.polarizability(L, d, z)
    ref = np.zeros((4, 4), dtype=complex)
    for Pi in range(4):
        for Q in range(4):
            for i in range(2):
                for a in range(3):
                    D = s.eps[2 + a] - s.eps[i]
                    ref[Pi, Q] += s.M_ov[Pi, i, a] * s.M_ov[Q, i, a] * 4 * D / (z * z - D * D)
    assert np.allclose(P, ref, rtol=1e-14, atol=1e-17)


# --- W against the Casida spectral form -------------------------------------------

@pytest.mark.parametrize("seed", [11, 12])
def test_screened_element_matches_casida(seed):
    """W^c_nm(z) by the RI solve equals Eq. W_spectral with Omega, rho from the
    Casida problem, for occupied and virtual m and z on and off both axes."""
    s = _tiny(seed=seed, n_occ=3, n_virt=5, n_aux=12, n_core=2)
    L, d = _ri(s)
    Om, XpY = RF.casida(s.eps, s.n_occ, s.M_ov)
    for n in (0, 1):
        rho = RF.transition_moments(s.M_oo, s.M_ov, n, XpY)
        for m in range(s.n_basis):
            b = S.pair_vector(s.M_oo, s.M_ov, n, m)
            for z in (0.3 + 0.01j, 0.7j, 5.0 + 0.003j, 0.05 + 0.0037j, 1.3 + 0.5j):
                w1 = S.screened_element(L, d, b, z)
                w2 = complex(RF.w_pole(rho[m], Om, z))
                assert abs(w1 - w2) <= 1e-11 * abs(w2), (n, m, z)


def test_w_imag_axis_matches_casida_c1():
    """On c1 (N_ov = 175): W^c_nm(i w_k) from the Cholesky route equals the
    spectral form; it is real and <= 0."""
    s = system_from_config(CONFIGS["c1"])
    L, d = _ri(s)
    W = S.w_imag_axis(L, d, s.M_oo, s.M_ov, [0], s.omega_imag)
    Om, XpY = RF.casida_symmetric(s.eps, s.n_occ, s.M_ov)
    rho = RF.transition_moments(s.M_oo, s.M_ov, 0, XpY)
    for m in range(0, s.n_basis, 3):
        ref = RF.w_pole(rho[m], Om, 1j * s.omega_imag)
        assert np.max(np.abs(ref.imag)) < 1e-12 * np.max(np.abs(ref))
        # norm-wise: the pole form loses digits to cancellation at large w
        assert np.max(np.abs(W[0, m] - ref.real)) <= 1e-11 * np.max(np.abs(ref))
    assert np.all(W <= 0)


# --- Sigma^c ---------------------------------------------------------------------

def test_residue_matches_closed_form_c1():
    """R_n(w) = sum_m f_m W_pole(|eps_m - w| + i eta) at c1 size, to 1e-11."""
    s = system_from_config(CONFIGS["c1"])
    L, d = _ri(s)
    Om, XpY = RF.casida_symmetric(s.eps, s.n_occ, s.M_ov)
    rho = RF.transition_moments(s.M_oo, s.M_ov, 0, XpY)
    for w in (s.omega_real[0, 3], s.omega_real[0, 77], float(s.eps[0])):
        R, _ = S.residue(L, d, s.eps, s.occ, s.M_oo, s.M_ov, 0, float(w), s.eta)
        _, _, Rref = RF.cd_closed_form(s.eps, s.n_occ, rho, Om, float(w), s.eta)
        assert abs(R - Rref) <= 1e-11 * abs(Rref)


def test_imag_integral_converges_to_closed_form():
    """The quadrature of Eq. cd_imaginary approaches its exact value as the
    grid grows (not a 1e-9 check: it measures quadrature error)."""
    s = _tiny(seed=21, n_occ=3, n_virt=6, n_aux=14)
    L, d = _ri(s)
    Om, XpY = RF.casida(s.eps, s.n_occ, s.M_ov)
    rho = RF.transition_moments(s.M_oo, s.M_ov, 0, XpY)
    omegas = [float(s.eps[0]) - 0.4, float(s.eps[0]) - 2.0, float(s.eps[0]) + 0.3]
    errs = []
    for n in (24, 40, 100, 200, 400):
        x, w = mgl_grid(n, 0.5)
        W = S.w_imag_axis(L, d, s.M_oo, s.M_ov, [0], x)
        e = 0.0
        for om in omegas:
            I = S.imag_integral(W[0], s.eps, x, w, om)
            a = om - s.eps
            Iref = -np.sum(rho ** 2 * (np.sign(a)[:, None] / (np.abs(a)[:, None] + Om[None, :])))
            e = max(e, abs(I - Iref) / abs(Iref))
        errs.append(e)
    assert errs[-1] < 1e-9
    assert errs[-1] < errs[0]
    assert errs[2] < errs[0]


def test_sigma_matches_pole_sum_as_eta_vanishes():
    """With eta -> 0 and an accurate grid, -I + R equals the fully analytic
    pole sum of Eq. sigma_spectral away from its poles, in all four
    occupied/virtual and above/below cases."""
    s = _tiny(seed=31, n_occ=3, n_virt=6, n_aux=14)
    L, d = _ri(s)
    Om, XpY = RF.casida(s.eps, s.n_occ, s.M_ov)
    rho = RF.transition_moments(s.M_oo, s.M_ov, 0, XpY)
    x, w = mgl_grid(400, 0.5)
    W = S.w_imag_axis(L, d, s.M_oo, s.M_ov, [0], x)
    eta = 1e-9
    # below the core, between core and valence, in the gap, above the LUMO
    for om in (float(s.eps[0]) - 0.7, float(s.eps[0]) + 1.1, 0.5 * (s.eps[2] + s.eps[3]),
               float(s.eps[4]) + 0.05):
        sc, _, _ = S.sigma_c_at(L, d, s.eps, s.occ, s.M_oo, s.M_ov, 0, om, eta, W[0], x, w)
        ps = RF.sigma_pole_sum(s.eps, s.n_occ, rho, Om, om, eta)
        assert abs(sc - ps) <= 1e-8 * abs(ps), om


def test_sigma_at_eps_n_uses_half_theta():
    """At w = eps_n the m = n term takes Theta(0) = 1/2 and a zero imaginary-axis
    term; the result equals the pole sum (both one-sided limits of the exact
    CD expression).  Theta(0) = 1 or 0 would be off by rho^2/Omega per mode."""
    s = _tiny(seed=41, n_occ=3, n_virt=6, n_aux=14)
    L, d = _ri(s)
    Om, XpY = RF.casida(s.eps, s.n_occ, s.M_ov)
    rho = RF.transition_moments(s.M_oo, s.M_ov, 0, XpY)
    x, w = mgl_grid(400, 0.5)
    W = S.w_imag_axis(L, d, s.M_oo, s.M_ov, [0], x)
    om = float(s.eps[0])
    sc, _, terms = S.sigma_c_at(L, d, s.eps, s.occ, s.M_oo, s.M_ov, 0, om, 1e-9, W[0], x, w)
    ps = RF.sigma_pole_sum(s.eps, s.n_occ, rho, Om, om, 1e-9)
    assert abs(sc.real - ps.real) <= 1e-8 * abs(ps)
    cf, _, _ = RF.cd_closed_form(s.eps, s.n_occ, rho, Om, om, s.eta)
    sc2, _, _ = S.sigma_c_at(L, d, s.eps, s.occ, s.M_oo, s.M_ov, 0, om, s.eta, W[0], x, w)
    assert abs(sc2 - cf) <= 1e-9 * abs(cf)
    assert 0 in terms  # the m = n residue is present with weight 1/2


def test_one_mode_model_closed_form():
    """One auxiliary function, one core c, one valence o, one virtual v, with the
    core-valence couplings set to zero (the three-level model of the paper's
    section on the validity of GW+C).  By hand: Pi(z) = 4 m^2 D/(z^2 - D^2),
    Omega^2 = D^2 + 4 m^2 D, W^c_cc(z) = b^2 4 m^2 D / (z^2 - Omega^2), so
    rho^2 = 2 b^2 m^2 D / Omega and Sigma^c_c(w) -> rho^2/(w - eps_c + Omega)."""
    eps = np.array([-10.6, -0.9, 0.3])   # core, valence, virtual (Ha)
    occ = np.array([2.0, 2.0, 0.0])
    mval, bcc = 0.45, 0.8
    M_ov = np.zeros((1, 2, 1))
    M_ov[0, 1, 0] = mval                 # (o v); the core-virtual coupling is 0
    M_oo = np.zeros((1, 2, 2))
    M_oo[0, 0, 0] = bcc                  # (c c); (c o) = 0
    M_oo[0, 1, 1] = 0.3
    L, d = S.ov_matrix(M_ov), S.transition_energies(eps, 2)
    D = eps[2] - eps[1]
    Om = np.sqrt(D * D + 4 * mval * mval * D)
    rho2 = 2 * bcc * bcc * mval * mval * D / Om
    for z in (0.2 + 0.01j, 2.0j, Om + 0.05 + 0.001j):
        Wcc = S.screened_element(L, d, M_oo[:, 0, 0], z)
        assert abs(Wcc - rho2 * 2 * Om / (z * z - Om * Om)) < 1e-13
    x, w = mgl_grid(400, 0.5)
    W = S.w_imag_axis(L, d, M_oo, M_ov, [0], x)
    for om in (eps[0] - 0.3, eps[0] - Om - 0.2, eps[0] + 0.4):
        sc, _, _ = S.sigma_c_at(L, d, eps, occ, M_oo, M_ov, 0, om, 1e-10, W[0], x, w)
        ref = rho2 / (om - eps[0] + Om)
        assert abs(sc - ref) < 1e-9 * abs(ref)
    sc, _, _ = S.sigma_c_at(L, d, eps, occ, M_oo, M_ov, 0, float(eps[0]), 1e-10, W[0], x, w)
    assert abs(sc.real - rho2 / Om) < 1e-9 * rho2 / Om


# --- exchange, invariants, modes -------------------------------------------------

def test_exchange_textbook():
    """Sigma^x_n = -sum_{i occ} (n i | i n) with explicit four-index integrals."""
    s = _tiny(seed=51, n_occ=4, n_virt=3, n_aux=9, n_core=2)
    eri = RF.four_index(s.M_oo, s.M_oo)
    for n in (0, 1):
        ref = -sum(eri[n, i, i, n] for i in range(s.n_occ))
        assert abs(S.exchange(s.M_oo, n) - ref) < 1e-15


def test_aux_rotation_invariance():
    """M -> O M for a random orthogonal O on the auxiliary index: Pi -> O Pi O^T
    and every output of the oracle is unchanged."""
    s = _tiny(seed=61, n_occ=3, n_virt=5, n_aux=10, n_real=5)
    rng = np.random.default_rng(5)
    O, _ = np.linalg.qr(rng.standard_normal((10, 10)))
    r1 = S.sigma_core_system(s)
    s.M_ov = np.einsum("PQ,Qia->Pia", O, s.M_ov)
    s.M_oo = np.einsum("PQ,Qij->Pij", O, s.M_oo)
    r2 = S.sigma_core_system(s)
    for k in ("sigma_c", "sigma_c_eps", "sigma_x", "e_qp", "im_sigma_dec"):
        a, b = np.asarray(r1[k]), np.asarray(r2[k])
        assert np.allclose(a, b, rtol=1e-11, atol=1e-14), k


def test_full_and_decoupled_agree_on_im_dec_and_eqp():
    s = _tiny(seed=71, n_occ=4, n_virt=5, n_aux=12, n_core=2, n_real=7)
    full = S.sigma_core_system(s, mode="full")
    dec = S.sigma_core_system(s, mode="decoupled")
    assert dec["sigma_c"] is None
    assert np.array_equal(full["im_sigma_dec"], dec["im_sigma_dec"])
    assert np.array_equal(full["e_qp"], dec["e_qp"])
    # Im Sigma^c comes from the residues only (Eq. cd_sigma_imaginary)
    L, d = _ri(s)
    for c, n in enumerate(s.core_idx):
        for j in (0, 3, 6):
            om = float(s.omega_real[c, j])
            R, _ = S.residue(L, d, s.eps, s.occ, s.M_oo, s.M_ov, int(n), om, s.eta)
            assert full["sigma_c"][c, j].imag == R.imag


def test_eqp_is_hedin_shift_fixed_point():
    """E = eps_n + Delta H_n solves E = eps_n + Sigma^x + Re Sigma^c(E - Delta H) - v^xc."""
    s = _tiny(seed=81, n_real=3)
    s.vxc = np.array([-0.37])
    r = S.sigma_core_system(s)
    dH = r["sigma_x"][0] + r["sigma_c_eps"][0].real - s.vxc[0]
    assert r["e_qp"][0] == pytest.approx(s.eps[0] + dH, abs=1e-15)


# --- symmetry-equivalent core levels ------------------------------------------

def _equivalent_pair(seed=91):
    s = _tiny(seed=seed, n_occ=4, n_virt=6, n_aux=14, n_core=2, n_real=6,
              real_abs_ev=(-300.0, -280.0))
    s.eps = s.eps.copy()
    s.eps[1] = s.eps[0]  # two degenerate (symmetry-equivalent) core levels
    sym = -np.ones(s.n_basis, dtype=np.int32)
    sym[0] = sym[1] = 3
    return s, sym


def test_symmetric_decoupling_matches_pole_form():
    """Eq. sigma_spectral_decoupled_symmetric in its CD form: the decoupled Im
    Sigma of core n sums f_i Im W^c_ni(|eps_i - w| + i eta) over the equivalent
    cores i; checked against the Casida spectral W of each pair (n, i)."""
    s, sym = _equivalent_pair()
    out = S.sigma_core_system(s, mode="decoupled", sym_group=sym)
    Om, XpY = RF.casida_symmetric(s.eps, s.n_occ, s.M_ov)
    for c, n in enumerate(s.core_idx):
        rho = RF.transition_moments(s.M_oo, s.M_ov, int(n), XpY)
        ref = np.zeros(s.omega_real.shape[1])
        for j, w in enumerate(s.omega_real[c]):
            for i in (0, 1):
                f = S.prefactor(float(s.eps[i]), True, float(w))
                if f != 0.0:
                    ref[j] += f * RF.w_pole(rho[i], Om, abs(float(s.eps[i]) - w) + 1j * s.eta).imag
        assert np.max(np.abs(out["im_sigma_dec"][c] - ref)) <= 1e-10 * np.max(np.abs(ref))
        # the partner term is not negligible here: the set changes the result
        plain = S.sigma_core_system(s, mode="decoupled")["im_sigma_dec"][c]
        assert np.max(np.abs(plain - ref)) > 1e-3 * np.max(np.abs(ref))


def test_symmetric_decoupling_defaults_and_full_mode():
    s, sym = _equivalent_pair(seed=92)
    none = S.sigma_core_system(s, mode="decoupled")
    unlabeled = S.sigma_core_system(s, mode="decoupled", sym_group=-np.ones(s.n_basis, int))
    assert np.array_equal(none["im_sigma_dec"], unlabeled["im_sigma_dec"])
    full = S.sigma_core_system(s, mode="full", sym_group=sym)
    dec = S.sigma_core_system(s, mode="decoupled", sym_group=sym)
    assert np.array_equal(full["im_sigma_dec"], dec["im_sigma_dec"])
    assert np.array_equal(full["e_qp"], dec["e_qp"])
    bad = sym.copy()
    bad[s.n_occ] = 3  # a virtual orbital in the set
    with pytest.raises(ValueError):
        S.sigma_core_system(s, mode="decoupled", sym_group=bad)


# --- the quasiparticle equation ---------------------------------------------------

def test_qp_newton_matches_one_pole_roots():
    """With the one-mode model, Sigma^c(w) = rho^2/(w - eps_c + Omega), the
    quasiparticle equation (Eq. quasiparticle_equation) is the quadratic
    x^2 + (Omega - s) x - (s Omega + rho^2) = 0 in x = E - eps_c, s = Sigma^x - v^xc.
    Its upper root is the QP solution and the lower one the satellite solution
    (the paper's two graphical solutions); Newton from eps_c finds the upper."""
    eps = np.array([-10.6, -0.9, 0.3])
    occ = np.array([2.0, 2.0, 0.0])
    mval, bcc = 0.45, 0.8
    M_ov = np.zeros((1, 2, 1))
    M_ov[0, 1, 0] = mval
    M_oo = np.zeros((1, 2, 2))
    M_oo[0, 0, 0] = bcc
    M_oo[0, 1, 1] = 0.3
    L, d = S.ov_matrix(M_ov), S.transition_energies(eps, 2)
    D = eps[2] - eps[1]
    Om = np.sqrt(D * D + 4 * mval * mval * D)
    rho2 = 2 * bcc * bcc * mval * mval * D / Om
    x, w = mgl_grid(400, 0.5)
    W = S.w_imag_axis(L, d, M_oo, M_ov, [0], x)
    for vxc in (0.0, -0.35):
        s = -bcc * bcc - vxc
        bq, cq = Om - s, -(s * Om + rho2)
        roots = np.sort(np.roots([1.0, bq, cq]).real)
        E, it = S.qp_newton(L, d, eps, occ, M_oo, M_ov, 0, 1e-10, W[0], x, w, vxc=vxc,
                            max_iter=40, tol=1e-12, step=1e-5)
        assert it > 0
        assert abs(E - (eps[0] + roots[1])) < 1e-8
        # the satellite root also solves the equation
        sc, _, _ = S.sigma_c_at(L, d, eps, occ, M_oo, M_ov, 0, eps[0] + roots[0], 1e-10, W[0], x, w)
        assert abs(roots[0] - (s + sc.real)) < 1e-8


def test_qp_newton_reports_non_convergence():
    s = _tiny(seed=83, n_real=3)
    out = S.sigma_core_system(s, qp=dict(max_iter=1, tol=1e-300, step=1e-4))
    assert out["qp_iterations"][0] == -1
    conv = S.sigma_core_system(s, qp=dict(max_iter=50, tol=1e-10, step=1e-4))
    assert conv["qp_iterations"][0] > 1
