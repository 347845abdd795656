"""Host-side checks of the benchmark script (no GPU): the counter-derived
traffic of a profile summary is used only while the native sources hash to
the value recorded with it, and more than one GPU is refused with a message."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _profile(tmp_path, digest, traffic="123456789"):
    p = tmp_path / "traffic.md"
    p.write_text("# a summary\n\n"
                 f"- traffic_bytes_per_launch: `{traffic}`\n"
                 f"- sources_sha256: `{digest}`\n")
    return str(p)


def test_traffic_is_read_only_for_the_present_sources(tmp_path):
    assert bench.measured_traffic(_profile(tmp_path, bench.sources_digest())) == 123456789.0
    assert bench.measured_traffic(_profile(tmp_path, "0" * 64)) is None
    assert bench.measured_traffic(str(tmp_path / "missing.md")) is None


def test_committed_traffic_profiles_parse():
    """Every committed traffic summary names a positive byte count and a
    64-digit digest (whether it matches depends on the sources)."""
    for name in ("TRAFFIC_PROFILE", "RB_TRAFFIC_PROFILE", "RU_TRAFFIC_PROFILE",
                 "SHELL_TRAFFIC_PROFILE"):
        text = open(getattr(bench, name)).read()
        assert "traffic_bytes_per_launch: `" in text and "sources_sha256: `" in text, name
        digest = text.split("sources_sha256: `")[1].split("`")[0]
        assert len(digest) == 64 and all(c in "0123456789abcdef" for c in digest), name
        nbytes = float(text.split("traffic_bytes_per_launch: `")[1].split("`")[0])
        assert nbytes > 0, name


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
