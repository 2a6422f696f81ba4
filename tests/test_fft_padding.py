"""Index arithmetic of the padded LDS layout of the line transforms, checked on
the CPU: the shortcuts the Stockham passes take for padded indices
(read_split, write_split in csrc/fft.h) must equal the padded index computed
in full, for both element sizes (pad runs 16 and 8), every radix, line length
and stride.  Built from the library's own header with hipcc for the host only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1907_01194_amd", "csrc")


def test_padded_index_shortcuts(tmp_path):
    hipcc = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "pad_check")
    subprocess.run([hipcc, "-x", "hip", "--offload-host-only", "-std=c++20", "-iquote", CSRC,
                    os.path.join(ROOT, "tests", "native", "pad_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    assert "violations 0" in out, out
    assert "pad run 16" in out and "pad run 8" in out
