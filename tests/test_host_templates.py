"""The structured operator application of the stability iteration (apply_row
for (a0 M~ + b0 L~) x) against the entry-by-entry system matrix (sys_entry),
compiled and run on the host."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)


@pytest.mark.skipif(HIPCC is None, reason="hipcc not available")
def test_apply_row_matches_sys_entry(tmp_path):
    exe = tmp_path / "templates_check"
    src = os.path.join(ROOT, "tests", "host", "templates_check.cpp")
    inc = os.path.join(ROOT, "paper_1905_10388_amd", "csrc")
    r = subprocess.run([HIPCC, "-O1", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", "-I", inc,
                        src, "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
