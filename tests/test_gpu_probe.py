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
    print(f"fp64 mfma {f64:.1f} TF, bf16 mfma {bf16:.0f} TF, fp16 mfma {f16:.0f} TF, copy {hbm:.0f} GB/s")
    # within a factor of the datasheet figures (78.6 TF, 2.5 PF, 2.5 PF, 8 TB/s)
    assert 20 < f64 < 100
    assert 400 < bf16 < 3000
    assert 400 < f16 < 3000
    assert 1000 < hbm < 9000
