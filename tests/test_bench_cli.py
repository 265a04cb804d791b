"""bench.py's command line: the multi-GPU request is refused with a message
(one GPU only), before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_profile_figures_follow_the_kernel_sources(tmp_path, monkeypatch):
    """A figure taken from a committed counter summary is reported only while
    the kernel sources it was measured on are unchanged (their SHA-256 is in
    the summary); a missing summary or a changed source gives None."""
    import hashlib
    sys.path.insert(0, ROOT)
    import bench
    src_dir = tmp_path / "paper_2311_08946_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    (src_dir / "a.hip").write_text("kernel a\n")
    (src_dir / "b.h").write_text("header b\n")
    sha = hashlib.sha256(b"kernel a\nheader b\n").hexdigest()
    (tmp_path / "profiles" / "p.md").write_text(f"text\n\nbytes_per_step: 12345\n\nsource_sha256: {sha}\n")
    monkeypatch.setattr(bench.os.path, "abspath", lambda p: str(tmp_path / "bench.py"))
    assert bench._profile_value("p.md", "bytes_per_step", ["a.hip", "b.h"]) == 12345.0
    assert bench._profile_value("p.md", "bytes_per_step", ["b.h", "a.hip"]) is None
    assert bench._profile_value("missing.md", "bytes_per_step", ["a.hip"]) is None
    (src_dir / "a.hip").write_text("kernel a, changed\n")
    assert bench._profile_value("p.md", "bytes_per_step", ["a.hip", "b.h"]) is None

