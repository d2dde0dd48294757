"""bench.py behaviour that needs no GPU: the one-GPU guard and the rule that
counted HBM traffic is reported only for the kernel source it was taken
with."""
import json
import os
import shutil
import subprocess
import sys

from _hbi_util import ROOT

sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_only_for_the_source_it_was_counted_on(tmp_path, monkeypatch):
    # a copy of the committed record and kernel source under a scratch root
    for rel in ("profiles/k_wstage_f32_bump1024_traffic.json",
                "paper_2210_02698_amd/csrc/hbi_apply.hip"):
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        shutil.copy(os.path.join(ROOT, rel), tmp_path / rel)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = json.load(open(tmp_path / "profiles/k_wstage_f32_bump1024_traffic.json"))
    t = bench.measured_traffic("k_wstage")
    assert t is None or t == rec["traffic_bytes_per_launch"]
    assert bench.measured_traffic("k_final") is None   # another kernel's record
    with open(tmp_path / "paper_2210_02698_amd/csrc/hbi_apply.hip", "a") as f:
        f.write("\n// edited\n")
    assert bench.measured_traffic("k_wstage") is None
