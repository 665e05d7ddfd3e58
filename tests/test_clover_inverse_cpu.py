"""Host build of the clover block inverse (csrc/clover_inv.h, the routine the
clover kernel runs per odd site and chirality): LDL^H on well-conditioned
blocks, the pivoted fallback on nonsingular indefinite blocks with a
vanishing pivot, and the singular report that becomes ENUMERIC.  Built with
g++ twice, plainly and under AddressSanitizer + UndefinedBehaviorSanitizer."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "clover_inv_check.cpp")
INC = os.path.join(ROOT, "paper_2503_16994_amd", "csrc")


@pytest.mark.parametrize("flags", [[], ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g"]],
                         ids=["plain", "asan_ubsan"])
def test_clover_block_inverse_host_build(tmp_path, flags):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no g++")
    exe = str(tmp_path / "clover_inv_check")
    subprocess.run([cxx, "-O2", "-std=c++17", "-Wall", "-Wno-unknown-pragmas", *flags, f"-I{INC}", SRC, "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("ok ") == 5
