"""Host-side logic of bench.py (no GPU): its residue-task bookkeeping agrees with
the oracle's count (Eq. cd_prefactors), and a multi-GPU request is refused."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


@pytest.mark.parametrize("name", ["c1", "c2"])
@pytest.mark.parametrize("mode", ["full", "decoupled"])
def test_residue_task_count_matches_oracle(name, mode):
    import bench
    from oracle import sigma as OS
    from workloads import CONFIGS, system_from_config
    s = system_from_config(CONFIGS[name])
    assert (bench.residue_task_count(s.eps, s.occ, s.core_idx, s.omega_real, mode)
            == OS.count_residue_tasks(s.eps, s.occ, s.core_idx, s.omega_real, mode))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
