"""bench.py's host-side contract: the counter-summary parser behind the
roofline's `traffic` field, and the one-GPU guard (no GPU needed)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def summary(path, digest, nbytes):
    with open(path, "w") as f:
        f.write("# counters\n\nsome text: with a colon\n\n")
        f.write(f"- sources_digest: `{digest}`\n- traffic_bytes_per_launch: `{nbytes}`\n")


def test_traffic_is_read_only_for_the_current_kernel_sources(tmp_path):
    p = str(tmp_path / "t.md")
    summary(p, bench.sources_digest(), 123456789)
    assert bench.measured_traffic(p) == 123456789.0
    # counters taken from other kernel sources do not apply
    summary(p, "0" * 16, 123456789)
    assert bench.measured_traffic(p) is None
    # missing file or field, unparsable value
    assert bench.measured_traffic(str(tmp_path / "absent.md")) is None
    with open(p, "w") as f:
        f.write(f"- sources_digest: `{bench.sources_digest()}`\n")
    assert bench.measured_traffic(p) is None
    summary(p, bench.sources_digest(), "many")
    assert bench.measured_traffic(p) is None


def test_digest_covers_every_frame_kernel_source():
    csrc = os.path.join(ROOT, "paper_2311_16121_amd", "csrc")
    for name in bench.FRAME_SOURCES:
        assert os.path.exists(os.path.join(csrc, name)), name
    assert len(bench.sources_digest()) == 16


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
