"""GPU parity of the split-precision DFT-GEMM imaging (FP16 hi+lo operands on
the matrix cores, FP32 accumulation) against the FP64 oracle, at the same
tolerances as the FP32 FFT path."""
import numpy as np
import pytest

from paper_1603_02126_amd import synth

from ._helpers import GAIN_RTOL, IMAGE_RTOL, gain_err, gpu_run, image_err, oracle_run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,efmt,kernel,na,n_samples,t_cal", [
    (32, synth.FMT_CI8, 2, 48, 230, 50),
    (64, synth.FMT_CI4, 2, 200, 301, 100),
    (32, synth.FMT_CF32, 1, 32, 64, 1),
    (64, synth.FMT_CI8, 2, 300, 90, 40),
])
def test_dft_gemm_run_matches_oracle(cuda, n, efmt, kernel, na, n_samples, t_cal):
    wl = synth.config_small(n=n, efmt=efmt, kernel=kernel, n_ant=na, n_samples=n_samples, t_cal=t_cal)
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda, transform=2)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    err = image_err(got["image"], ref["image"]).max()
    assert err <= IMAGE_RTOL, err


def test_dft_gemm_tiny_full(cuda):
    wl = synth.config_tiny()
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda, transform=2)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


def test_dft_gemm_lwa_full_size_sampled(cuda):
    wl = synth.config_lwa()
    packed = synth.make_efield(wl, threads=16)
    got = gpu_run(wl, packed, cuda, transform=2)
    fft = gpu_run(wl, packed, cuda, transform=1)
    chans = [5, 99]
    ref = oracle_run(wl, packed[:, chans], channels=chans)
    assert image_err(got["image"][chans], ref["image"]).max() <= IMAGE_RTOL
    assert image_err(got["image"], fft["image"]).max() <= 2 * IMAGE_RTOL
    np.testing.assert_array_equal(got["gains"], fft["gains"])   # same solve kernel
