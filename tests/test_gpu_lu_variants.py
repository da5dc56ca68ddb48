"""GPU parity of both factorisations of the bordered matrices at wide borders.

The default LDL^T (no pivoting) and the partial-pivoting LU
(GWC_FACTORIZATION=lu).  The batched LU keeps each panel row-block in
registers, with a register layout chosen by the bordered order n = N_aux + R
(R = N_basis border vectors on the imaginary axis).  A small N_aux with a wide
border reaches every layout up to the largest supported order at little
oracle cost (the oracle solves N_aux x N_aux systems); N_aux = 150 gives three
outer steps, the last one ragged, and for the LDL^T a border block of up to
190 tile rows whose off-diagonal tiles are skipped.  Orders above the largest
supported one are refused.
"""
import numpy as np
import pytest

import paper_2412_17132_amd as gwc
from oracle import sigma as OS
from workloads import system_from_config
from workloads.configs import small_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-9
N_AUX = 150
MAX_ORDER = 24 * 512

# n_virt such that n = N_AUX + n_occ + n_virt falls in each row-block range
VIRT = [1800, 2800, 3800, 5900, 7900, 12000]


@pytest.mark.parametrize("fact", ["ldlt", "lu"])
@pytest.mark.parametrize("n_virt", VIRT, ids=[f"order{N_AUX + 3 + v}" for v in VIRT])
def test_wide_border_orders(n_virt, fact, monkeypatch):
    assert N_AUX + 3 + n_virt <= MAX_ORDER
    monkeypatch.setenv("GWC_FACTORIZATION", fact)
    s = system_from_config(small_config(name="wide", n_occ=3, n_virt=n_virt, n_aux=N_AUX, n_core=1,
                                        n_imag=4, n_real=3, seed=300 + n_virt % 97))
    print(f"case {fact} n_aux={N_AUX} n_basis={s.n_basis} order={N_AUX + s.n_basis}", flush=True)
    dev = torch.device("cuda:0")
    d = gwc.to_device(s, dev)
    out = gwc.gwc_sigma_core(d["eps"], d["occ"], d["M_oo"], d["M_ov"], d["core_idx"],
                             d["omega_imag"], d["w_imag"], d["omega_real"], d["eta"], mode="full")
    torch.cuda.synchronize()
    sc = out["sigma_c"].cpu().numpy()
    sc = sc[..., 0] + 1j * sc[..., 1]
    ref = OS.sigma_core_system(s)
    scale = np.max(np.abs(ref["sigma_c"][0]))
    err = np.max(np.abs(sc[0] - ref["sigma_c"][0])) / scale
    assert err <= TOL, f"sigma_c rel err {err:.3e}"
    assert np.allclose(out["e_qp"].cpu().numpy(), ref["e_qp"], rtol=TOL, atol=0)


def test_order_above_maximum_is_refused():
    n_virt = MAX_ORDER - N_AUX  # order N_AUX + 3 + n_virt > MAX_ORDER
    s = system_from_config(small_config(name="too_wide", n_occ=3, n_virt=n_virt, n_aux=N_AUX,
                                        n_core=1, n_imag=2, n_real=1, seed=399))
    with pytest.raises(gwc.GwcError) as ei:
        gwc.gwc_sigma_core(s.eps, s.occ, s.M_oo, s.M_ov, s.core_idx, s.omega_imag, s.w_imag,
                           s.omega_real, s.eta, mode="full")
    assert ei.value.status == -8
