"""Host-side parts of bench.py's contract (no GPU): the one-GPU guard and the
reading of committed rocprofv3 summaries behind `roofline.traffic`."""
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


def _summary(tmp_path, sha, traffic="123456789", valu="1e9"):
    (tmp_path / "k_back_c2.md").write_text(
        "# k_back on c2\n\n## Recorded for bench.py\n\n"
        f"- `kernel_source_sha256`: `{sha}`\n"
        f"- `traffic_bytes_per_launch`: {traffic}\n"
        f"- `valu_wave_instructions_per_launch`: {valu}\n")


@pytest.fixture
def bench(monkeypatch, tmp_path):
    import bench as b
    monkeypatch.setattr(b, "PROFILES", str(tmp_path))
    return b


def test_recorded_figures_are_read_when_the_sources_match(bench, tmp_path):
    _summary(tmp_path, bench.kernel_source_hash())
    assert bench.recorded_traffic("k_back", "c2") == 123456789.0
    assert bench.recorded_profile("k_back", "c2", "valu_wave_instructions_per_launch") == 1e9
    assert bench.recorded_profile("k_back", "c2", "no_such_key") is None


def test_recorded_figures_are_dropped_once_the_kernels_change(bench, tmp_path):
    _summary(tmp_path, "0" * 64)
    assert bench.recorded_traffic("k_back", "c2") is None


def test_missing_summary_gives_no_figure(bench):
    assert bench.recorded_traffic("k_back", "c2") is None


def test_committed_summaries_carry_the_recorded_keys():
    """Each committed projector summary names the source hash it was taken on and
    the per-launch figures bench.py reads (whether that hash is current is
    checked at run time, where a mismatch turns the figures to null)."""
    for k in ("k_back", "k_fwd"):
        text = open(os.path.join(ROOT, "profiles", f"{k}_c2.md")).read()
        for key in ("kernel_source_sha256", "traffic_bytes_per_launch",
                    "valu_wave_instructions_per_launch"):
            assert f"- `{key}`:" in text
