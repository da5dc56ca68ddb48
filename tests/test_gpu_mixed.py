"""Mixed-precision Pi build (BF16X3, FP16X3, FP8) against the FP64 oracle / FP64 GPU path.

Targets for BF16X3 and FP16X3: |dE_QP| <= 10 meV and matched satellite peak
positions within 0.02 eV; Sigma^c errors are reported (max and median relative).
FP8 (e4m3, 4-bit significands) carries ~2^-7 relative error per product (hi and
lo each round to 2^-4 of what they represent, and lo*lo is dropped); the
factorisation's conditioning can amplify that a few times, so its bars are
|dSigma^c| <= 2^-4 max|Sigma^c| and |dE_QP| <= 2^-4 |Re Sigma^c(eps_n)|.
"""
import numpy as np
import pytest

import paper_2412_17132_amd as gwc
from oracle import sigma as OS
from spectra import satellite_peaks
from workloads import CONFIGS, EV_PER_HA, system_from_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EQP_TOL = 0.010 / EV_PER_HA
SAT_TOL = 0.02 / EV_PER_HA


def _run(d, precision, mode="full"):
    out = gwc.gwc_sigma_core(d["eps"], d["occ"], d["M_oo"], d["M_ov"], d["core_idx"],
                             d["omega_imag"], d["w_imag"], d["omega_real"], d["eta"],
                             mode=mode, precision=precision)
    torch.cuda.synchronize()
    return out


def _spectrum(d, s, out, c, n_t=2 ** 16, dw=0.01 / EV_PER_HA):
    n = int(s.core_idx[c])
    e_qp = float(out["e_qp"][c])
    w0 = e_qp - 30 / EV_PER_HA
    A, z = gwc.gwc_spectral_cumulant(d["omega_real"][c], out["im_sigma_dec"][c], float(s.eps[n]), e_qp,
                                     s.eta, n_t, dw, 3500, w0)
    return w0 + np.arange(3500) * dw, A.cpu().numpy(), e_qp, float(z[0])


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3", "fp8"])
def test_c1_mixed_vs_oracle(precision):
    s = system_from_config(CONFIGS["c1"])
    d = gwc.to_device(s, torch.device("cuda:0"))
    out = _run(d, precision)
    ref = OS.sigma_core_system(s)
    sc = out["sigma_c"].cpu().numpy()
    sc = sc[..., 0] + 1j * sc[..., 1]
    rel = np.abs(sc - ref["sigma_c"]) / np.max(np.abs(ref["sigma_c"]))
    print(f"{precision} c1: Sigma^c rel err max {rel.max():.3e} median {np.median(rel):.3e}; "
          f"dE_QP {abs(out['e_qp'].cpu().numpy()[0] - ref['e_qp'][0]) * EV_PER_HA * 1e3:.3f} meV")
    deq = abs(out["e_qp"].cpu().numpy()[0] - ref["e_qp"][0])
    if precision == "fp8":
        assert deq <= 2.0 ** -4 * abs(ref["sigma_c_eps"][0].real)
        assert rel.max() < 2.0 ** -4
    else:
        assert deq <= EQP_TOL
        assert rel.max() < (1e-3 if precision == "bf16x3" else 1e-4)


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3", "fp8"])
def test_c2_size_mixed_eqp_and_satellites(precision):
    """Benzene-sized system, DECOUPLED mode (the paper's production setting):
    E_QP of every core within 10 meV and satellite peaks of A(w) within 0.02 eV
    of the FP64 GPU path (itself at 1e-9 of the oracle)."""
    s = system_from_config(CONFIGS["c2"], n_real=400)
    d = gwc.to_device(s, torch.device("cuda:0"))
    ref = _run(d, "fp64", "decoupled")
    out = _run(d, precision, "decoupled")
    deq = np.abs(out["e_qp"].cpu().numpy() - ref["e_qp"].cpu().numpy())
    print(f"{precision} c2: max dE_QP {deq.max() * EV_PER_HA * 1e3:.3f} meV")
    if precision == "fp8":
        sc_ref = ref["sigma_c_eps"].cpu().numpy()[:, 0]
        assert np.all(deq <= 2.0 ** -4 * np.abs(sc_ref))
    else:
        assert deq.max() <= EQP_TOL
    worst = 0.0
    for c in range(s.n_core):
        w, A_ref, eq_ref, z_ref = _spectrum(d, s, ref, c)
        w2, A_mx, eq_mx, z_mx = _spectrum(d, s, out, c)
        p_ref = satellite_peaks(w, A_ref, eq_ref, z_ref, s.eta)
        p_mx = satellite_peaks(w2, A_mx, eq_mx, z_mx, s.eta)
        assert len(p_ref) > 0
        for p in p_ref:
            worst = max(worst, np.min(np.abs(np.asarray(p_mx) - p)))
    print(f"{precision} c2: worst satellite shift {worst * EV_PER_HA * 1e3:.3f} meV")
    if precision != "fp8":
        assert worst <= SAT_TOL
