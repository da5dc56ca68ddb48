"""GPU parity of CD-WAC (Eq. pade_approximation) against the CD-WAC oracle.

A continued-fraction fit is well-conditioned only where its reference points
resolve W: when they do not, rounding in the reference values decides where
spurious poles land and no two implementations agree.  The parity cases are
therefore systems whose reference points resolve W, and each test first
checks that on the oracle: a 1e-14 relative perturbation of every reference
value moves Sigma^c by less than 1e-11 (relative to its maximum).  The bar is
then 1e-9, as for contour deformation: the GPU's reference values differ from
the oracle's by rounding (~1e-13) and the fit amplifies that by < 1e3.
"""
import numpy as np
import pytest

import paper_2412_17132_amd as gwc
from oracle import sigma as OS
from oracle import wac as OW
from spectra import satellite_peaks
from workloads import CONFIGS, EV_PER_HA, system_from_config
from workloads.configs import small_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-9

CASES = [
    # n_occ, n_virt, n_aux, n_core, n_imag, points per window, seed
    (4, 10, 40, 2, 24, 150, 7),
    (5, 14, 70, 2, 24, 300, 7),
]


def _oracle(s, p, mode="full", sym_group=None, perturb=0.0):
    if not perturb:
        return OW.sigma_core_wac(s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, s.omega_imag, s.w_imag,
                                 s.omega_real, s.eta, p, mode=mode, sym_group=sym_group)
    rng = np.random.default_rng(5)
    sa, wi = OW.screened_all, OW.S.w_imag_axis
    try:
        OW.screened_all = lambda *a: (lambda v: v * (1 + perturb * rng.standard_normal(v.shape)))(sa(*a))
        OW.S.w_imag_axis = lambda *a: (lambda v: v * (1 + perturb * rng.standard_normal(v.shape)))(wi(*a))
        return _oracle(s, p, mode, sym_group)
    finally:
        OW.screened_all, OW.S.w_imag_axis = sa, wi


def _gpu(s, p, mode="full", sym_group=None):
    d = gwc.to_device(s, torch.device("cuda:0"))
    out = gwc.gwc_sigma_core(d["eps"], d["occ"], d["M_oo"], d["M_ov"], d["core_idx"],
                             d["omega_imag"], d["w_imag"], d["omega_real"], d["eta"], mode=mode,
                             sym_group=sym_group, wac=p)
    torch.cuda.synchronize()
    return {k: (None if v is None else v.cpu().numpy()) for k, v in out.items()}


def _cplx(a):
    return a[..., 0] + 1j * a[..., 1]


@pytest.mark.parametrize("case", CASES, ids=[f"ov{c[0] * c[1]}_pts{c[5]}" for c in CASES])
@pytest.mark.parametrize("mode", ["full", "decoupled"])
def test_wac_parity_resolved(case, mode):
    n_occ, n_virt, n_aux, n_core, n_imag, npts, seed = case
    s = system_from_config(small_config(n_occ=n_occ, n_virt=n_virt, n_aux=n_aux, n_core=n_core,
                                        n_real=7, seed=seed, n_imag=n_imag))
    p = OW.paper_params(npts, npts)
    print(f"case wac {case} mode={mode}", flush=True)
    ref = _oracle(s, p, mode)
    if mode == "full":
        pert = _oracle(s, p, mode, perturb=1e-14)
        scale = np.max(np.abs(ref["sigma_c"]))
        assert np.max(np.abs(pert["sigma_c"] - ref["sigma_c"])) < 1e-11 * scale, "ill-conditioned case"
    out = _gpu(s, p, mode)
    if mode == "full":
        sc = _cplx(out["sigma_c"])
        assert np.max(np.abs(sc - ref["sigma_c"])) <= TOL * np.max(np.abs(ref["sigma_c"]))
        # resolved: CD-WAC equals contour deformation here
        cd = OS.sigma_core_system(s)
        assert np.max(np.abs(sc - cd["sigma_c"])) <= TOL * np.max(np.abs(cd["sigma_c"]))
    imd = out["im_sigma_dec"]
    assert np.max(np.abs(imd - ref["im_sigma_dec"])) <= TOL * np.max(np.abs(ref["im_sigma_dec"]))
    assert np.allclose(out["e_qp"], ref["e_qp"], rtol=TOL, atol=0)
    assert np.allclose(_cplx(out["sigma_c_eps"]), ref["sigma_c_eps"], rtol=TOL, atol=0)


def test_wac_with_equivalent_cores():
    s = system_from_config(small_config(n_occ=4, n_virt=10, n_aux=40, n_core=2, n_real=7, seed=7,
                                        n_imag=24))
    s.eps = s.eps.copy()
    s.eps[1] = s.eps[0]
    sym = -np.ones(s.n_basis, dtype=np.int32)
    sym[0] = sym[1] = 2
    p = OW.paper_params(150, 150)
    print("case wac equivalent cores", flush=True)
    ref = _oracle(s, p, "decoupled", sym)
    out = _gpu(s, p, "decoupled", sym)
    assert np.max(np.abs(out["im_sigma_dec"] - ref["im_sigma_dec"])) <= TOL * np.max(np.abs(ref["im_sigma_dec"]))


def test_wac_c1_quasiparticle_energy():
    """c1 with the paper's settings: the grid is not resolved by the reference
    points (parity is not defined there), but Sigma^c(eps_n) uses the core-window
    node x = 0 for m = n and smooth valence W, so E_QP stays within 1 meV of CD."""
    s = system_from_config(CONFIGS["c1"])
    print("case wac c1", flush=True)
    out = _gpu(s, OW.paper_params())
    assert np.all(np.isfinite(out["sigma_c"])) and np.all(np.isfinite(out["im_sigma_dec"]))
    cd = OS.sigma_core_system(s)
    assert np.max(np.abs(out["e_qp"] - cd["e_qp"])) * EV_PER_HA < 1e-3



def test_wac_breakdown_returns_factorization_error():
    """A core state whose RI coefficients vanish (M_nm = 0 for every m) has
    W^c_nm = 0 at every reference point, so Thiele's reciprocal differences
    divide by zero: CD-WAC returns GWC_ERR_FACTORIZATION (-5) as a status, with
    a message, and the library stays usable (contour deformation on the same
    system then gives Sigma^c = 0 exactly, and CD-WAC on an intact system
    succeeds)."""
    s = system_from_config(small_config(n_occ=4, n_virt=7, n_aux=30, n_core=1, n_real=5, seed=61))
    s.M_oo = s.M_oo.copy()
    s.M_ov = s.M_ov.copy()
    s.M_oo[:, 0, :] = 0.0
    s.M_oo[:, :, 0] = 0.0
    s.M_ov[:, 0, :] = 0.0
    p = gwc.wac_paper_settings(n_core_pts=20, n_val_pts=20)
    print("case zero core coefficients, CD-WAC", flush=True)
    with pytest.raises(gwc.GwcError) as ei:
        _gpu(s, p)
    assert ei.value.status == -5
    assert "continued-fraction" in str(ei.value)
    out = gwc.gwc_sigma_core(s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, s.omega_imag, s.w_imag,
                             s.omega_real, s.eta, mode="full")
    assert np.all(out["sigma_c"] == 0.0) and np.all(out["sigma_c_eps"] == 0.0)
    good = system_from_config(small_config(n_occ=4, n_virt=7, n_aux=30, n_core=1, n_real=5, seed=61))
    ok = _gpu(good, p)
    assert np.all(np.isfinite(ok["sigma_c"]))


def _spectrum(s, out, c):
    """A(w) on the GPU from 30 eV below E_QP (0.01 eV steps) and its satellites."""
    dev = torch.device("cuda:0")
    n = int(s.core_idx[c])
    e_qp = float(out["e_qp"][c])
    d_omega, n_out = 0.01 / EV_PER_HA, 3500
    w0 = e_qp - 30 / EV_PER_HA
    A, z = gwc.gwc_spectral_cumulant(torch.tensor(s.omega_real[c], device=dev),
                                     torch.tensor(out["im_sigma_dec"][c], device=dev),
                                     float(s.eps[n]), e_qp, s.eta, 2 ** 16, d_omega, n_out, w0)
    torch.cuda.synchronize()
    w = w0 + np.arange(n_out) * d_omega
    return np.asarray(satellite_peaks(w, A.cpu().numpy(), e_qp, float(z.cpu().numpy()[0]), s.eta))


@pytest.mark.parametrize("cfg,mode,structured", [("c1", "full", True), ("c1", "full", False),
                                                 ("c2", "decoupled", True),
                                                 ("c2", "decoupled", False)])
def test_wac_reproduces_cd_where_the_paper_claims(cfg, mode, structured):
    """CD-WAC against contour deformation with the paper's settings (section
    CD-WAC), every core state: E_QP within 4 meV, and the lowest-lying
    satellite of A(w) within 0.02 eV on core-localised inputs (the core's RI
    coefficients with other states scaled by 1e-3) and at c1.  c2 is taken in
    the DECOUPLED mode the paper uses CD-WAC with.  On c2 inputs without core
    localisation the lowest satellite of one core state moves by about half an
    eV, and higher satellites (more than about 12 eV below E_QP) move by up to
    an eV on either input: the synthetic W has more poles there than the
    reference points resolve, as the paper finds beyond its fitting window.
    Those are reported by the benchmark, not bounded here."""
    s = system_from_config(CONFIGS[cfg], structured=structured)
    print(f"case wac vs cd {cfg} {mode} structured={structured}", flush=True)
    cd = _gpu(s, None, mode)
    wac = _gpu(s, OW.paper_params(), mode)
    assert np.max(np.abs(wac["e_qp"] - cd["e_qp"])) * EV_PER_HA <= 4e-3
    if cfg == "c2" and not structured:
        return
    for c in range(s.n_core):
        p_cd, p_wac = _spectrum(s, cd, c), _spectrum(s, wac, c)
        assert len(p_cd) and len(p_wac)
        lowest = np.max(p_cd)
        assert np.min(np.abs(p_wac - lowest)) * EV_PER_HA <= 0.02, c
