"""GPU parity of evGW0 (gwc_evgw0, Eq. ev_sigma_spectral) against the evGW0
oracle: every state's quasiparticle energy after the first iteration (G0W0)
and at self-consistency, the iteration counts, Sigma^x, and Sigma^c,ev and A of
the core states with the final energies.

Bar: 1e-9 relative to the largest magnitude of the energies.  Both sides run
the same bracketed Newton solves in the same order; they differ by the rounding
of the pole sums (and of the eigensolvers, see the analytic route's tests),
which the contracting outer iteration does not amplify.  Sigma^c,ev and A on
the grid depend on the final energies through poles eta away from the grid
points (|d Sigma / d e_m| <= max|Sigma| / eta), so their bar is
1e-9 + 2 max|Delta e| / eta relative, with Delta e the energies' measured
difference."""
import numpy as np
import pytest

import paper_2412_17132_amd as gwc
from oracle import evgw as EV
from workloads import CONFIGS, system_from_config, vv_block
from workloads.configs import small_config

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-9

CASES = [
    # n_occ, n_virt, n_aux, n_core, n_real, seed; one virtual state and one real point
    (3, 1, 10, 1, 1, 13),
    (4, 12, 30, 2, 5, 9),
    (5, 14, 40, 2, 9, 23),
    (12, 90, 300, 3, 17, 31),
]


def _cplx(a):
    return a[..., 0] + 1j * a[..., 1]


def _run(s, vv, vxc=None):
    dev = torch.device("cuda:0")
    d = gwc.to_device(s, dev)
    out = gwc.gwc_evgw0(d["eps"], d["occ"], d["M_oo"], d["M_ov"], torch.as_tensor(vv, device=dev),
                        d["core_idx"], d["omega_real"], d["eta"],
                        vxc=None if vxc is None else torch.as_tensor(vxc, device=dev))
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}


def _compare(out, ref, eta):
    rel = {k: np.max(np.abs(a - b)) / np.max(np.abs(b)) for k, a, b in (
        ("e_qp", out["e_qp"], ref["e_qp"]), ("e_first", out["e_first"], ref["e_first"]),
        ("sigma_c", _cplx(out["sigma_c"]), ref["sigma_c"]), ("a_ev", out["a_ev"], ref["a_ev"]))}
    print("  outer", int(out["outer"][0]), ref["outer"], "; " +
          ", ".join(f"{k} {v:.2e}" for k, v in rel.items()), flush=True)
    assert int(out["outer"][0]) == ref["outer"] and ref["outer"] > 0
    assert np.all(out["newton"] >= 0) and np.all(ref["newton"] >= 0)
    assert np.allclose(out["sigma_x"], ref["sigma_x"], rtol=1e-13, atol=0)
    assert rel["e_qp"] <= TOL and rel["e_first"] <= TOL
    grid_tol = TOL + 2 * np.max(np.abs(out["e_qp"] - ref["e_qp"])) / eta
    assert rel["sigma_c"] <= grid_tol and rel["a_ev"] <= grid_tol, (rel, grid_tol)


@pytest.mark.parametrize("case", CASES, ids=[f"nb{c[0] + c[1]}_ov{c[0] * c[1]}" for c in CASES])
def test_evgw0_parity(case):
    n_occ, n_virt, n_aux, n_core, n_real, seed = case
    s = system_from_config(small_config(n_occ=n_occ, n_virt=n_virt, n_aux=n_aux, n_core=n_core,
                                        n_real=n_real, seed=seed))
    vv = vv_block(s)
    print(f"case evgw0 {case}", flush=True)
    out = _run(s, vv)
    ref = EV.evgw0(s.eps, s.occ, s.M_oo, s.M_ov, vv, s.core_idx, s.omega_real, s.eta)
    _compare(out, ref, s.eta)


def test_evgw0_c1_with_vxc():
    s = system_from_config(CONFIGS["c1"])
    vv = vv_block(s)
    vxc = np.linspace(-0.4, 0.1, s.n_basis)
    print("case evgw0 c1 vxc", flush=True)
    out = _run(s, vv, vxc)
    ref = EV.evgw0(s.eps, s.occ, s.M_oo, s.M_ov, vv, s.core_idx, s.omega_real, s.eta, vxc=vxc)
    _compare(out, ref, s.eta)


def test_evgw0_rejects_nonfinite_vv():
    s = system_from_config(small_config(n_occ=3, n_virt=5, n_aux=8, seed=2))
    vv = vv_block(s)
    vv[0, 1, 2] = np.nan
    print("case evgw0 nan M_vv", flush=True)
    with pytest.raises(gwc.GwcError) as ei:
        _run(s, vv)
    assert ei.value.status_name == "GWC_ERR_NONFINITE"


@pytest.mark.blas_threads
def test_evgw0_c2_first_iteration_sampled():
    """Benzene-sized system (300 states, N_ov = 5859) at the size the bench
    times: the first iteration's energies (the G0W0 solutions from eps, each a
    function of its own state only) of the 6 cores and a sample of valence and
    virtual states, computed one by one by the oracle; the run converges."""
    s = system_from_config(CONFIGS["c2"])
    vv = vv_block(s)
    print("case evgw0 c2 sampled", flush=True)
    out = _run(s, vv)
    states = [0, 1, 2, 3, 4, 5, 10, 20, 21, 60, 150, 299]
    E, steps = EV.first_iteration(s.eps, s.occ, s.M_oo, s.M_ov, vv, states, s.eta)
    rel = np.max(np.abs(out["e_first"][states] - E)) / np.max(np.abs(E))
    print(f"  e_first sampled rel {rel:.2e}; outer {int(out['outer'][0])}", flush=True)
    assert np.all(steps >= 0)
    assert rel <= TOL
    assert int(out["outer"][0]) > 0 and np.all(out["newton"] >= 0)
