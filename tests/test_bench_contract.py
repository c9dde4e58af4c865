"""Host-side checks of bench.py's contract (no GPU): more than one GPU is
refused with a message before anything touches a device, and the fingerprint
that ties the recorded HBM traffic to the kernel sources ignores comments but
not code."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_fingerprint_ignores_comments_not_code(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2411_09156_amd" / "csrc"
    csrc.mkdir(parents=True)
    (tmp_path / "include").mkdir()
    for f in ("paper_2411_09156_amd/csrc/gesr_render.hip", "paper_2411_09156_amd/csrc/gesr_device.h",
              "paper_2411_09156_amd/csrc/gesr_bin.hip", "paper_2411_09156_amd/csrc/gesr_project.hip",
              "paper_2411_09156_amd/csrc/gesr_kernels.h", "include/gesr.h"):
        with open(os.path.join(ROOT, f)) as fh:
            (tmp_path / f).write_text(fh.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_fingerprint()
    p = csrc / "gesr_bin.hip"
    text = p.read_text()
    p.write_text("// a new comment line\n" + text.replace("\n", "\n\n", 3) + "\n/* trailing\n   block */\n")
    assert bench.kernel_fingerprint() == base
    p.write_text(text.replace("IS_IPL = 2", "IS_IPL = 4", 1))
    assert bench.kernel_fingerprint() != base
    p.write_text(text)
    h = tmp_path / "include" / "gesr.h"
    h.write_text(h.read_text().replace("#define GESR_REC_FLOATS 16", "#define GESR_REC_FLOATS 12", 1))
    assert bench.kernel_fingerprint() != base
