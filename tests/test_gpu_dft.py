"""GPU parity of the split-precision DFT-GEMM imaging (16-bit split operands
on the matrix cores, FP32 accumulation) against the FP64 oracle, at the same
tolerances as the FP32 FFT path, for fp16 hi+lo (transform 2), bf16 hi+lo
(transform 3) and bf16 hi+mid+lo (transform 4): 32 x 32 and 64 x 64
directly, 128 x 128 and 256 x 256 as residue classes of 64 x 64
transforms."""
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
    (128, synth.FMT_CI8, 2, 150, 70, 30),     # residue classes of 64 x 64 DFT-GEMMs
    (256, synth.FMT_CI4, 2, 300, 33, 20),
    (128, synth.FMT_CF32, 1, 40, 25, 25),
])
@pytest.mark.parametrize("transform", [2, 3, 4])
def test_dft_gemm_run_matches_oracle(cuda, n, efmt, kernel, na, n_samples, t_cal, transform):
    wl = synth.config_small(n=n, efmt=efmt, kernel=kernel, n_ant=na, n_samples=n_samples, t_cal=t_cal)
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda, transform=transform)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    err = image_err(got["image"], ref["image"]).max()
    print(f"DFT-GEMM transform {transform}, {n}^2 {na} antennas: image error {err:.2e}", flush=True)
    assert err <= IMAGE_RTOL, err


# bf16 hi + lo keeps about 16 bits of every operand (each part's rounding
# 2^-9 relative, the dropped lo * lo term 2^-18); measured, its images stay
# within the 1e-5 tolerance (about 3e-6 on the cases above), which the
# parametrised test checks with the other two precisions.


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


def test_dft_gemm_hera_full_size_sampled(cuda):
    """HERA-shaped workload at full size through the residue-class DFT-GEMM
    (128 x 128, 350 antennas); the oracle checks one channel and the FFT path
    all of them."""
    wl = synth.config_hera()
    packed = synth.make_efield(wl, threads=16)
    got = gpu_run(wl, packed, cuda, transform=2)
    fft = gpu_run(wl, packed, cuda, transform=1)
    chans = [201]
    ref = oracle_run(wl, packed[:, chans], channels=chans)
    assert image_err(got["image"][chans], ref["image"]).max() <= IMAGE_RTOL
    assert image_err(got["image"], fft["image"]).max() <= 2 * IMAGE_RTOL
    np.testing.assert_array_equal(got["gains"], fft["gains"])
