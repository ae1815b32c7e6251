"""The register FFTs of the imaging engines, compiled for the host and
checked against a direct double-precision DFT (tests/host_fft/fft_reg_check.hip):
every size the engines use (8 to 64 points), both signs (the image transform
and its adjoint), random and sparse inputs.  The 64-point transform folds its
twiddles into fused multiply-adds, so this pins its scale bookkeeping."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_register_fft_matches_direct_dft(tmp_path):
    from paper_1603_02126_amd import build
    src = os.path.join(HERE, "host_fft", "fft_reg_check.hip")
    exe = str(tmp_path / "fft_reg_check")
    cmd = [build.hipcc(), f"--offload-arch={build.ARCH}", "-O2", "-std=c++17", "-I", build.CSRC, src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        pytest.fail(f"build failed:\n{r.stdout}\n{r.stderr}")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=dict(os.environ, HIP_VISIBLE_DEVICES=""))
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "fft_reg check passed" in r.stdout
