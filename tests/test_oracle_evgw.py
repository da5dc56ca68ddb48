"""Pins of the evGW0 oracle (Eq. ev_sigma_spectral): its first iteration against
the contour-deformation oracle's G0W0 quasiparticle solution, the three-level
model's self-consistent closed form, the root bracketing on equations with
known roots, and the fixed point at convergence."""
import numpy as np
import pytest

from oracle import evgw as EV
from oracle import sigma as S
from workloads import mgl_grid, system_from_config, vv_block
from workloads.configs import small_config


def _scan_roots(fun, lo, hi, n=20001):
    E = np.linspace(lo, hi, n)
    f = np.array([fun(x)[0] for x in E])
    return E[:-1][np.sign(f[:-1]) != np.sign(f[1:])]


def test_qp_root_finds_the_roots_of_known_equations():
    """A one-pole quasiparticle equation f(E) = E - c - r (E - p) / ((E - p)^2 + h^2)
    has up to three roots; the bracketed solve returns one of them to 1e-12 from
    either side, including starts next to the pole where plain Newton cycles,
    within 8 steps (false position where Newton leaves the bracket: 5-6 steps;
    the bracket midpoint there took up to 11)."""
    c, r, p, h = 0.3, 0.02, 0.25, 0.004

    def fun(E):
        a = E - p
        den = a * a + h * h
        return E - c - r * a / den, 1.0 - r * (h * h - a * a) / (den * den)

    roots = _scan_roots(fun, -2, 2)
    assert len(roots) == 3
    for E0 in (-1.0, 0.0, 0.249, 0.251, 0.26, 0.5, 1.5):
        E, it = EV.qp_root(fun, E0, h, 1e-13, 200)
        assert 0 <= it <= 8
        assert abs(fun(E)[0]) < 1e-12
        assert np.min(np.abs(roots - E)) < 1e-3   # one of the scanned roots


def test_qp_root_accepts_a_root_found_at_a_bracket_end():
    """f(E) = E - r + 1e-17: the representable root r evaluates to f = 1e-17 > 0,
    so r becomes the bracket's upper end and the next Newton step rounds to
    exactly r.  That is convergence (two steps), not a step out of the bracket
    (which would bisect towards r for ~30 steps)."""
    r = 0.3
    E, it = EV.qp_root(lambda x: (x - r + 1e-17, 1.0), 0.31, 0.004, 1e-10, 200)
    assert 0 < it <= 3
    assert abs(E - r) < 1e-15


def test_first_iteration_is_the_g0w0_quasiparticle_solution():
    """With e^(0) = eps the first iteration solves the G0W0 quasiparticle
    equation; for weak coupling the root is unique, so it equals the Newton
    solution of the contour-deformation oracle (eta -> 0, converged grid)."""
    s = system_from_config(small_config(n_occ=4, n_virt=9, n_aux=24, n_core=2, seed=17, m_scale=0.12))
    vv = vv_block(s)
    eta = 1e-6
    r = EV.evgw0(s.eps, s.occ, s.M_oo, s.M_ov, vv, s.core_idx, s.omega_real, eta)
    L, d = S.ov_matrix(s.M_ov), S.transition_energies(s.eps, s.n_occ)
    x, w = mgl_grid(300, 0.5)
    for n in range(s.n_occ):
        W = S.w_imag_axis(L, d, s.M_oo, s.M_ov, [n], x)
        E, it = S.qp_newton(L, d, s.eps, s.occ, s.M_oo, s.M_ov, n, eta, W[0], x, w, tol=1e-12)
        assert it > 0
        assert abs(r["e_first"][n] - E) <= 1e-9 * abs(E), n
    assert r["outer"] > 1


def test_three_level_model_self_consistent_closed_form():
    """Core c, valence o, virtual v, one auxiliary function, (c o) = (c v) = 0.
    The only term of Sigma^c_c is m = c with the o -> v mode, and its pole moves
    with the core's own energy: at self-consistency
    E_c = eps_c + Sigma^x_c + rho^2 Omega / (Omega^2 + eta^2) - v^xc_c."""
    eps = np.array([-10.6, -0.9, 0.3])
    occ = np.array([2.0, 2.0, 0.0])
    mval, bcc = 0.45, 0.8
    M_ov = np.zeros((1, 2, 1))
    M_ov[0, 1, 0] = mval
    M_oo = np.zeros((1, 2, 2))
    M_oo[0, 0, 0] = bcc
    M_oo[0, 1, 1] = 0.3
    M_vv = np.full((1, 1, 1), 0.2)
    D = eps[2] - eps[1]
    Om = np.sqrt(D * D + 4 * mval * mval * D)
    rho2 = 2 * bcc * bcc * mval * mval * D / Om
    eta = 0.004
    vxc = np.array([-0.2, 0.1, 0.05])
    r = EV.evgw0(eps, occ, M_oo, M_ov, M_vv, [0], eps[None, :1] - 0.5, eta, vxc=vxc,
                 tol_outer=1e-13, tol_newton=1e-14)
    assert r["outer"] > 0
    ref = eps[0] - bcc * bcc + rho2 * Om / (Om * Om + eta * eta) - vxc[0]
    assert abs(r["e_qp"][0] - ref) < 1e-12
    # G0W0 (first iteration) sits elsewhere: the pole was at eps_c - Omega
    assert abs(r["e_first"][0] - ref) > 1e-3


def test_fixed_point_at_convergence():
    """At convergence every state's energy solves its quasiparticle equation
    with the final energies in G, to the stated tolerances."""
    s = system_from_config(small_config(n_occ=5, n_virt=14, n_aux=40, n_core=2, seed=23))
    vv = vv_block(s)
    r = EV.evgw0(s.eps, s.occ, s.M_oo, s.M_ov, vv, s.core_idx, s.omega_real, s.eta)
    assert r["outer"] > 0 and np.all(r["newton"] >= 0)
    Om, XpY = EV.AN.rpa_excitations(s.eps, s.n_occ, s.M_ov)
    r2 = EV.moments_all(s.M_oo, s.M_ov, vv, XpY)
    sgn = np.where(np.arange(s.n_basis) < s.n_occ, 1.0, -1.0)
    for n in range(s.n_basis):
        re, dre, _ = EV.pole_sum(r2[n], r["e_qp"], sgn, Om, r["e_qp"][n], s.eta)
        f = r["e_qp"][n] - s.eps[n] - r["sigma_x"][n] - re
        # |f| <= |f'| (tol_newton + tol_outer): the last Newton step and the last energy change
        assert abs(f) <= abs(1 - dre) * 2e-8, n


@pytest.mark.parametrize("n", [0, 3, 9])
def test_moments_all_match_single_state_moments(n):
    """rho for every pair equals the analytic oracle's rho for an occupied n;
    for virtual n the pair block uses M_vo = M_ov^T and M_vv."""
    from oracle import analytic as AN
    s = system_from_config(small_config(n_occ=4, n_virt=8, n_aux=20, seed=29))
    vv = vv_block(s)
    Om, XpY = AN.rpa_excitations(s.eps, s.n_occ, s.M_ov)
    r2 = EV.moments_all(s.M_oo, s.M_ov, vv, XpY)
    if n < s.n_occ:
        ref = AN.transition_moments(s.M_oo, s.M_ov, n, XpY) ** 2
    else:
        Bn = np.concatenate([s.M_ov[:, :, n - s.n_occ], vv[:, n - s.n_occ, :]], axis=1)
        ref = (np.sqrt(2.0) * (Bn.T @ s.M_ov.reshape(s.n_aux, -1)) @ XpY) ** 2
    assert np.allclose(r2[n], ref, rtol=1e-12, atol=1e-18)
    assert np.allclose(r2[:, n, :], r2[n], rtol=1e-12, atol=1e-18)   # symmetric in (n, m)


def test_first_iteration_by_state_equals_full_run():
    """`first_iteration` (one state at a time, for large systems) reproduces the
    first iteration of the full run."""
    s = system_from_config(small_config(n_occ=5, n_virt=14, n_aux=40, n_core=2, seed=23))
    vv = vv_block(s)
    full = EV.evgw0(s.eps, s.occ, s.M_oo, s.M_ov, vv, s.core_idx, s.omega_real, s.eta)
    states = [0, 1, 4, 7, 18]
    E, steps = EV.first_iteration(s.eps, s.occ, s.M_oo, s.M_ov, vv, states, s.eta)
    assert np.all(steps >= 0)
    assert np.allclose(E, full["e_first"][states], rtol=1e-13, atol=0)
