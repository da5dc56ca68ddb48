"""Peak-rate probes return plausible device figures (diagnostics used by bench.py)."""
import pytest

import paper_2412_17132_amd as gwc

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_probe_peaks_plausible():
    assert torch.cuda.is_available()
    f64 = gwc.probe_peak("fp64_mfma")
    bf16 = gwc.probe_peak("bf16_mfma")
    f16 = gwc.probe_peak("fp16_mfma")
    hbm = gwc.probe_peak("hbm_copy")
    f8a = gwc.probe_peak("fp8_mfma_k32")
    f8b = gwc.probe_peak("fp8_mfma_k128")
    print(f"fp64 mfma {f64:.1f} TF, bf16 mfma {bf16:.0f} TF, fp16 mfma {f16:.0f} TF, copy {hbm:.0f} GB/s, "
          f"fp8 mfma K=32 {f8a:.0f} TF, K=128 {f8b:.0f} TF")
    # within a factor of the datasheet figures (78.6 TF, 2.5 PF, 2.5 PF, 8 TB/s)
    assert 20 < f64 < 100
    assert 400 < bf16 < 3000
    assert 400 < f16 < 3000
    assert 1000 < hbm < 9000
    assert 400 < f8a < 6000
    assert 800 < f8b < 6000
