"""Host accuracy of the library's FP64 logarithm and Green's functions (the
code the pair kernels inline), against long-double evaluations of the
closed forms g_I = 2/d + log(2/d) - log(1 + d/2) and
g_E = 2/d - log(2/d) - log(1 + d/2) over chords d in [1e-6, 2]."""
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1906_04209_amd" / "csrc"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not Path(HIPCC).exists(), reason="hipcc not available")
def test_log64_and_green64_ulps(tmp_path):
    exe = tmp_path / "log_check"
    subprocess.check_call([HIPCC, "-O2", "-std=c++17", "-I", str(CSRC), str(ROOT / "tests" / "host" / "log_check.cpp"),
                           "-o", str(exe)], stderr=subprocess.DEVNULL)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
