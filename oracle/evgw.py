"""Oracle: eigenvalue-self-consistent evGW0 quasiparticle energies.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain NumPy in float64.

Steps (section "GW for core levels: beyond G0W0", Eq. ev_sigma_spectral):
1. RPA excitations Omega^nu and X + Y once, as in the fully analytic route
   (`oracle.analytic`): W stays at the RPA level of the mean-field energies.
2. Transition moments rho^nu_nm (Eq. density_shifts) for every pair of states,
   from the RI coefficients of the oo, ov (= vo) and vv blocks.
3. Iteration k = 0, 1, ... from e^(0) = eps: every state's quasiparticle
   equation (Eq. quasiparticle_equation)
       E = eps_n + Sigma^x_n + Re Sigma^c,ev_n(E; e^(k)) - v^xc_n,
       Sigma^c,ev_n(w; e) = sum_{m,nu} (rho^nu_nm)^2 / (w - e_m + (Omega^nu - i eta) s_m)
   (s_m = sgn(eps_F - e_m): +1 for occupied, -1 for virtual m; the occupations
   stay those of the mean field) is solved for f(E) = E - eps_n - Sigma^x_n
   - Re Sigma + v^xc_n = 0 by a bracketed Newton iteration from E0 = e^(k)_n:
     a. since f(E) ~ E for large |E|, a root lies on the side d = -sign f(E0):
        points E0 + d eta 2^j (j = 0, 1, ...) are tried until f changes sign,
        which brackets a root between the last two points;
     b. Newton steps with the analytic derivative
          f' = 1 - d Re Sigma / dw,  d Re Sigma / dw = sum rho^2 (eta^2 - a^2) / (a^2 + eta^2)^2,
          a = w - e_m + s_m Omega,
        from the bracket end with the smaller |f|, each replaced by the
        Illinois false-position point of the (shrinking) bracket when it leaves
        it (the midpoint if that point rounds onto an end), until
        |Delta E| < tol_newton (more than max_newton steps flag the state);
   e^(k+1) = the roots; the iteration stops when max_n |e^(k+1)_n - e^(k)_n| < tol_outer.
   Plain Newton from E0 cycles for states whose root lies next to a pole of
   Sigma (virtual levels with corrections of ~10 eV on the synthetic inputs); the
   bracket makes every state's solve converge to a root of its equation.
4. With the final energies: Sigma^c,ev of the core states on their grids and
   A (Eq. A_explicit_real_imaginary with Sigma = Sigma^x + Sigma^c,ev).
Sigma^x_n = -sum_i (ni|in) over occupied i for every state (Eq. sigma_x).

Pins (tests/test_oracle_evgw.py): the first iteration equals the G0W0
quasiparticle solution of the contour-deformation oracle (eta -> 0); the
three-level model's closed form, in which the only pole of Sigma^c_c follows
the core's own energy, E_c = eps_c + Sigma^x_c + rho^2 Omega / (Omega^2 + eta^2);
the fixed-point residual of every state at convergence.
"""
from __future__ import annotations

import numpy as np

from . import analytic as AN


def pair_block_all(M_oo, M_ov, M_vv):
    """M[P][n][m] for all states n, m (occupied first)."""
    n_aux, n_occ, n_virt = M_ov.shape
    nb = n_occ + n_virt
    M = np.empty((n_aux, nb, nb))
    M[:, :n_occ, :n_occ] = M_oo
    M[:, :n_occ, n_occ:] = M_ov
    M[:, n_occ:, :n_occ] = M_ov.transpose(0, 2, 1)
    M[:, n_occ:, n_occ:] = M_vv
    return M


def moments_all(M_oo, M_ov, M_vv, XpY):
    """(rho^nu_nm)^2 as r2[n][m][nu] for every pair of states."""
    M = pair_block_all(M_oo, M_ov, M_vv)
    n_aux, nb, _ = M.shape
    L = M_ov.reshape(n_aux, -1)                                   # [P][ia]
    Rm = L @ XpY                                                  # [P][nu]
    rho = np.sqrt(2.0) * (M.reshape(n_aux, nb * nb).T @ Rm)       # [(n, m)][nu]
    return (rho * rho).reshape(nb, nb, -1)


def moments_of_states(M_oo, M_ov, M_vv, XpY, states):
    """(rho^nu_nm)^2 as r2[k][m][nu] for the listed states n = states[k] only
    (the rows `moments_all` would hold for them), for large systems."""
    n_aux, n_occ, n_virt = M_ov.shape
    L = M_ov.reshape(n_aux, -1)
    Rm = L @ XpY                                                  # [P][nu]
    out = []
    for n in states:
        if n < n_occ:
            Mn = np.concatenate([M_oo[:, n, :], M_ov[:, n, :]], axis=1)
        else:
            Mn = np.concatenate([M_ov[:, :, n - n_occ], M_vv[:, n - n_occ, :]], axis=1)
        rho = np.sqrt(2.0) * (Mn.T @ Rm)
        out.append(rho * rho)
    return np.array(out)


def first_iteration(eps, occ, M_oo, M_ov, M_vv, states, eta, vxc=None, max_newton=200,
                    tol_newton=1e-10):
    """Energies after the first iteration (e^(0) = eps in G, i.e. the G0W0
    quasiparticle solutions found from eps by step 3) for the listed states,
    each computed on its own: (E [len(states)], Newton steps)."""
    eps = np.asarray(eps, dtype=float)
    nb = eps.size
    n_occ = int(np.sum(np.asarray(occ) > 0))
    vxc = np.zeros(nb) if vxc is None else np.asarray(vxc, dtype=float)
    sgn = np.where(np.arange(nb) < n_occ, 1.0, -1.0)
    Om, XpY = AN.rpa_excitations(eps, n_occ, M_ov)
    r2 = moments_of_states(M_oo, M_ov, M_vv, XpY, states)
    sx = exchange_all(M_oo, M_ov)
    E_out, steps = [], []
    for k, n in enumerate(states):
        def fun(E, k=k, n=n):
            re, dre, _ = pole_sum(r2[k], eps, sgn, Om, E, eta)
            return E - eps[n] - sx[n] - re + vxc[n], 1.0 - dre
        E, it = qp_root(fun, eps[n], eta, tol_newton, max_newton)
        E_out.append(E)
        steps.append(it)
    return np.array(E_out), np.array(steps)


def exchange_all(M_oo, M_ov):
    """Sigma^x_n = -sum_i sum_P (M^P_ni)^2 for every state n."""
    sx_occ = -np.sum(M_oo ** 2, axis=(0, 2))
    sx_virt = -np.sum(M_ov ** 2, axis=(0, 1))
    return np.concatenate([sx_occ, sx_virt])


def pole_sum(r2n, e, sgn, Om, w, eta):
    """(Re Sigma, d Re Sigma / dw, Im Sigma) of one state at w; r2n[m][nu]."""
    a = (w - e)[:, None] + sgn[:, None] * Om[None, :]
    den = a * a + eta * eta
    re = np.sum(r2n * a / den)
    dre = np.sum(r2n * (eta * eta - a * a) / (den * den))
    im = np.sum(r2n * sgn[:, None] * eta / den)
    return re, dre, im


def qp_root(fun, E0, eta, tol, max_steps):
    """Step 3 for one state: bracket from E0, then safeguarded Newton (a step
    that leaves the bracket is replaced by the Illinois false-position point).
    fun(E) -> (f, f').  Returns (root, Newton steps) with steps = -1 when
    max_steps did not reach |Delta E| < tol."""
    f0, d0 = fun(E0)
    if f0 == 0.0:
        return E0, 0
    d = -1.0 if f0 > 0 else 1.0
    a, fa, da = E0, f0, d0
    h = eta
    for _ in range(1100):            # f ~ E: a sign change is reached within the double range
        b = E0 + d * h
        fb, db = fun(b)
        if fb == 0.0:
            return b, 0
        if (fb > 0) != (fa > 0):
            break
        a, fa, da = b, fb, db
        h *= 2.0
    lo, hi, flo, fhi = (a, b, fa, fb) if a < b else (b, a, fb, fa)
    E, f, df = (a, fa, da) if abs(fa) <= abs(fb) else (b, fb, db)
    kept = 0                         # -1: the last update moved lo, +1: it moved hi
    for it in range(1, max_steps + 1):
        En = E - f / df if df != 0.0 else lo - 1.0
        # a step onto an end is kept: at a root found at an end the step
        # rounds to zero, and that is convergence, not a step out
        if not (lo <= En <= hi):
            # false position on the bracket, the Illinois way: the f of an end
            # kept through two updates in a row is halved
            En = (lo * fhi - hi * flo) / (fhi - flo)
            if not (lo < En < hi):
                En = 0.5 * (lo + hi)
        if abs(En - E) < tol:
            return En, it
        E = En
        f, df = fun(E)
        if f == 0.0:
            return E, it
        if (f > 0) == (flo > 0):
            lo, flo = E, f
            if kept == -1:
                fhi *= 0.5
            kept = -1
        else:
            hi, fhi = E, f
            if kept == 1:
                flo *= 0.5
            kept = 1
    return E, -1


def evgw0(eps, occ, M_oo, M_ov, M_vv, core_idx, omega_real, eta, vxc=None, max_outer=100,
          tol_outer=1e-8, max_newton=200, tol_newton=1e-10):
    """Oracle for the `gwc_evgw0` entry point.

    vxc: [n_basis] or None.  Returns a dict with e_qp [n_basis], outer
    (iterations, -1 if not converged), newton [n_basis] (steps of the last
    iteration's bracketed Newton solves, -1 where they did not converge), sigma_x [n_basis],
    sigma_c [n_core][n_real], a_ev [n_core][n_real], omega_exc, and
    e_first [n_basis] (the energies after the first iteration: G0W0)."""
    eps = np.asarray(eps, dtype=float)
    nb = eps.size
    n_occ = int(np.sum(np.asarray(occ) > 0))
    vxc = np.zeros(nb) if vxc is None else np.asarray(vxc, dtype=float)
    sgn = np.where(np.arange(nb) < n_occ, 1.0, -1.0)
    Om, XpY = AN.rpa_excitations(eps, n_occ, M_ov)
    r2 = moments_all(M_oo, M_ov, M_vv, XpY)
    sx = exchange_all(M_oo, M_ov)
    e = eps.copy()
    e_first = None
    outer = -1
    newton = np.zeros(nb, dtype=int)
    for k in range(max_outer):
        e_new = np.empty(nb)
        for n in range(nb):
            def fun(E, n=n):
                re, dre, _ = pole_sum(r2[n], e, sgn, Om, E, eta)
                return E - eps[n] - sx[n] - re + vxc[n], 1.0 - dre
            e_new[n], newton[n] = qp_root(fun, e[n], eta, tol_newton, max_newton)
        delta = np.max(np.abs(e_new - e))
        e = e_new
        if e_first is None:
            e_first = e.copy()
        if delta < tol_outer:
            outer = k + 1
            break
    omega_real = np.atleast_2d(np.asarray(omega_real, dtype=float))
    sig = np.empty(omega_real.shape, dtype=complex)
    a_ev = np.empty(omega_real.shape)
    for c, n in enumerate(core_idx):
        n = int(n)
        for j, w in enumerate(omega_real[c]):
            re, _, im = pole_sum(r2[n], e, sgn, Om, w, eta)
            sig[c, j] = re + 1j * im
        den_re = omega_real[c] - eps[n] + vxc[n] - sx[n] - sig[c].real
        a_ev[c] = np.abs(sig[c].imag) / (np.pi * (den_re ** 2 + sig[c].imag ** 2))
    return dict(e_qp=e, outer=outer, newton=newton, sigma_x=sx, sigma_c=sig, a_ev=a_ev,
                omega_exc=Om, e_first=e_first)
