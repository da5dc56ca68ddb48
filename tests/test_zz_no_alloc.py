"""gwc_spectral_cumulant_noalloc (no device allocation; its temporaries live in
a library-owned device array) against gwc_spectral_cumulant, through the C ABI:
two calls in a row, the second with a smaller input, each to 1e-9 of the
allocating entry point's A(w) and Z (the two share their kernels, so they
agree bitwise); sizes above the array's limits are refused before any device
work."""
import numpy as np
import pytest

import paper_2412_17132_amd as gwc
from workloads import EV_PER_HA

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
TOL = 1e-9


def _case(seed, n_real):
    rng = np.random.default_rng(seed)
    eps_n = -10.65 + 0.01 * rng.standard_normal()
    e_qp = eps_n - 0.8
    w = np.linspace(eps_n - 25 / EV_PER_HA, eps_n, n_real)
    im = np.zeros(n_real)
    for _ in range(4):
        c0 = rng.uniform(-24, -3) / EV_PER_HA
        im -= rng.uniform(0.005, 0.05) * np.exp(-((w - eps_n - c0) / rng.uniform(0.01, 0.08)) ** 2)
    return w, im, eps_n, e_qp


@pytest.mark.parametrize("on_device", [True, False], ids=["device", "host"])
def test_noalloc_matches_allocating_entry_point(on_device):
    dev = torch.device("cuda:0")
    eta, dw = 0.1 / EV_PER_HA, 0.01 / EV_PER_HA
    for seed, n_real, n_t, n_out in ((7, 401, 2 ** 18, 2600), (8, 123, 2 ** 13, 700)):
        print(f"case noalloc seed={seed} n_real={n_real} n_t={n_t} n_out={n_out} "
              f"device={on_device}", flush=True)
        w, im, eps_n, e_qp = _case(seed, n_real)
        w0 = e_qp - 22 / EV_PER_HA
        if on_device:
            wt, it = torch.tensor(w, device=dev), torch.tensor(im, device=dev)
            A = torch.empty(n_out, dtype=torch.float64, device=dev)
            z = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            wt, it = w, im
            A, z = np.empty(n_out), np.empty(2)
        gwc.gwc_spectral_cumulant_noalloc(wt, it, eps_n, e_qp, eta, n_t, dw, n_out, w0, A, z)
        Ar, zr = gwc.gwc_spectral_cumulant(wt, it, eps_n, e_qp, eta, n_t, dw, n_out, w0)
        if on_device:
            torch.cuda.synchronize()
            A, z, Ar, zr = (x.cpu().numpy() for x in (A, z, Ar, zr))
        assert np.max(np.abs(A - Ar)) <= TOL * np.max(np.abs(Ar))
        assert np.max(np.abs(z - zr)) <= 1e-12
        assert abs(np.sum(A) * dw) <= 1.0 + 1e-9


def test_noalloc_refuses_sizes_above_its_limits():
    w, im, eps_n, e_qp = _case(9, 64)
    A, z = np.empty(16), np.empty(2)
    with pytest.raises(gwc.GwcError) as ei:
        gwc.gwc_spectral_cumulant_noalloc(w, im, eps_n, e_qp, 0.003, 2 ** 20, 1e-3, 16, e_qp - 1.0, A, z)
    assert ei.value.status == -2 and "no-allocation limit" in str(ei.value)
    wl = np.linspace(-11.0, -10.0, 2 ** 15 + 1)
    with pytest.raises(gwc.GwcError) as ei:
        gwc.gwc_spectral_cumulant_noalloc(wl, np.zeros_like(wl), eps_n, e_qp, 0.003, 2 ** 14, 1e-3, 16,
                                          e_qp - 1.0, A, z)
    assert ei.value.status == -2 and "no-allocation limit" in str(ei.value)
    wbad = w.copy()
    wbad[5] = wbad[4]
    with pytest.raises(gwc.GwcError) as ei:
        gwc.gwc_spectral_cumulant_noalloc(wbad, im, eps_n, e_qp, 0.003, 2 ** 10, 1e-3, 16, e_qp - 1.0, A, z)
    assert ei.value.status == -1
