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


def test_jsonl_record_is_appended(tmp_path, capsys):
    """--jsonl appends each result line, time-stamped, to a JSON-lines log."""
    import json
    import bench
    log = tmp_path / "runs.jsonl"
    bench.emit({"metric": "m", "value": 1.0}, str(log))
    bench.emit({"metric": "m", "value": 2.0}, str(log))
    out = capsys.readouterr().out.strip().splitlines()
    assert [json.loads(x)["value"] for x in out] == [1.0, 2.0]
    recs = [json.loads(x) for x in log.read_text().splitlines()]
    assert [r["value"] for r in recs] == [1.0, 2.0]
    assert all("logged_utc" in r and "git_rev" in r for r in recs)
