"""The library's register FFT codelets, checked on the host: compiled from
paper_2505_03360_amd/csrc/fft.hpp by hipcc into a host program that compares
every length the collision kernels use (radix-2/3/4 mixed recursions with the
twiddles in scaled form) against a direct DFT summed in long double.

Bound: a Cooley-Tukey transform's relative L2 error grows like
eps * O(log2 N); the measured worst case over 50 Gaussian vectors per case is
about 1.2e-7 in float and 2.6e-16 in double for N <= 96, so the bounds below
(2.5e-7, 5e-16) leave 2x headroom and still fail a wrong twiddle, sign or
output order (those give O(1) errors)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2505_03360_amd", "csrc")


def _hipcc():
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("fftc") / "fft_codelets_host")
    cmd = [hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC, "-x", "hip",
           os.path.join(HERE, "fft_codelets_host.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, check=True).stdout
    rows = {}
    for line in out.split("\n"):
        if line.strip():
            n, sign, t, err = line.split()
            rows[(int(n), int(sign), t)] = float(err)
    return rows


def test_every_length_both_signs_and_types(results):
    lengths = (2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96)
    assert len(results) == 4 * len(lengths)
    for (n, sign, t), err in results.items():
        bound = 2.5e-7 if t == "f" else 5e-16
        assert err <= bound, (n, sign, t, err)
