"""Host-side parts of bench.py's contract (no GPU): the one-GPU guard, the
reading of committed rocprofv3 summaries behind the roofline figures, and the
roofline arithmetic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _summary(tmp_path, sha, traffic="123456789", cycles="1e9", td="2e8", workload="c2"):
    (tmp_path / f"k_back_{workload}.md").write_text(
        f"# k_back on {workload}\n\n## Recorded for bench.py\n\n"
        f"- `kernel_source_sha256`: `{sha}`\n"
        f"- `traffic_bytes_per_launch`: {traffic}\n"
        f"- `valu_issue_cycles_per_launch`: {cycles}\n"
        f"- `td_busy_cycles_per_launch`: {td}\n"
        f"- `l2_hit_rate`: 0.5\n")


@pytest.fixture
def bench(monkeypatch, tmp_path):
    import bench as b
    monkeypatch.setattr(b, "PROFILES", str(tmp_path))
    return b


def test_recorded_figures_are_read_when_the_sources_match(bench, tmp_path):
    _summary(tmp_path, bench.kernel_source_hash())
    assert bench.recorded_profile("k_back", "c2", "traffic_bytes_per_launch") == 123456789.0
    assert bench.recorded_profile("k_back", "c2", "valu_issue_cycles_per_launch") == 1e9
    assert bench.recorded_profile("k_back", "c2", "no_such_key") is None


def test_recorded_figures_are_dropped_once_the_kernels_change(bench, tmp_path):
    _summary(tmp_path, "0" * 64)
    assert bench.recorded_profile("k_back", "c2", "traffic_bytes_per_launch") is None


def test_missing_summary_gives_no_figure(bench):
    assert bench.recorded_profile("k_back", "c2", "traffic_bytes_per_launch") is None


def test_roofline_takes_the_resource_closer_to_its_peak(bench, tmp_path):
    """alu = recorded main-pipe VALU issue cycles / launch time / (1024 SIMDs x
    2.4 GHz), vmem = recorded texture-data busy cycles / launch time / (256 x 2.4
    GHz); the larger is the bound; HBM beside them; null when the sources differ."""
    _summary(tmp_path, bench.kernel_source_hash(), traffic="4e9", cycles="2.4576e9",
             td="9.8304e8", workload="c5")
    r = bench.roofline(("k_back", 2.0, 8e10), 10 ** 10, "c5")
    assert r["kernel"] == "k_back"
    assert abs(r["alu"]["frac"] - 0.5) < 1e-9       # 2.4576e9 cycles in 2 ms: half of 1024 SIMDs
    assert abs(r["vmem"]["frac"] - 0.8) < 1e-9      # 9.8304e8 in 2 ms: 0.8 of 256 units
    assert r["bound"] == "vmem" and r["frac"] == r["vmem"]["frac"]
    assert r["peak"] == 614.4 and r["achieved"] == 491.5
    assert r["traffic"] == 4e9
    assert abs(r["hbm"]["frac"] - 4e9 / 2e-3 / 8e12) < 1e-9
    assert r["effective_GBps"] == 40000.0 and r["l2_hit_rate"] == 0.5
    _summary(tmp_path, bench.kernel_source_hash(), cycles="4e9", td="1e8", workload="c5")
    assert bench.roofline(("k_back", 2.0, 8e10), 10 ** 10, "c5")["bound"] == "alu"
    _summary(tmp_path, "0" * 64, workload="c5")
    r = bench.roofline(("k_back", 2.0, 8e10), 10 ** 10, "c5")
    assert r["frac"] is None and r["traffic"] is None and r["bound"] is None


def test_committed_summaries_carry_the_recorded_keys():
    """Each committed projector summary names the source hash it was taken on and
    the per-launch figures bench.py reads (whether that hash is current is
    checked at run time, where a mismatch turns the figures to null)."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "k_*_c*.md")):
        text = open(path).read()
        for key in ("kernel_source_sha256", "traffic_bytes_per_launch",
                    "valu_issue_cycles_per_launch", "td_busy_cycles_per_launch"):
            assert f"- `{key}`:" in text, (path, key)
