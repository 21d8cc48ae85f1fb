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


def _summary(tmp_path, sha, traffic="123456789", cycles="1e9", workload="c2"):
    (tmp_path / f"k_back_{workload}.md").write_text(
        f"# k_back on {workload}\n\n## Recorded for bench.py\n\n"
        f"- `kernel_source_sha256`: `{sha}`\n"
        f"- `traffic_bytes_per_launch`: {traffic}\n"
        f"- `valu_issue_cycles_per_launch`: {cycles}\n"
        f"- `td_busy_fraction`: 0.9\n")


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


def test_roofline_is_issue_cycles_over_the_chips_capacity(bench, tmp_path):
    """frac = recorded VALU issue cycles per launch / launch time / (1024 SIMDs x
    2.4 GHz); HBM figures beside it; null when the profile does not match."""
    _summary(tmp_path, bench.kernel_source_hash(), traffic="4e9", cycles="2.4576e9",
             workload="c5")
    r = bench.roofline(("k_back", 2.0, 8e10), 10 ** 10, "c5")
    assert r["bound"] == "alu" and r["kernel"] == "k_back"
    assert r["peak"] == 2457.6
    assert abs(r["frac"] - 0.5) < 1e-9           # 2.4576e9 cycles in 2 ms: half the capacity
    assert abs(r["achieved"] - 1228.8) < 1e-6
    assert r["traffic"] == 4e9
    assert abs(r["hbm"]["frac"] - 4e9 / 2e-3 / 8e12) < 1e-9
    assert r["effective_GBps"] == 40000.0
    assert r["measured"]["texture_data_busy"] == 0.9
    _summary(tmp_path, "0" * 64, workload="c5")
    r = bench.roofline(("k_back", 2.0, 8e10), 10 ** 10, "c5")
    assert r["frac"] is None and r["traffic"] is None


def test_committed_summaries_carry_the_recorded_keys():
    """Each committed projector summary names the source hash it was taken on and
    the per-launch figures bench.py reads (whether that hash is current is
    checked at run time, where a mismatch turns the figures to null)."""
    import glob
    for path in glob.glob(os.path.join(ROOT, "profiles", "k_*_c*.md")):
        text = open(path).read()
        for key in ("kernel_source_sha256", "traffic_bytes_per_launch",
                    "valu_issue_cycles_per_launch"):
            assert f"- `{key}`:" in text, (path, key)
