"""GPU parity of EPICal from several tapped pixels (the multiple-pixel
correlations of Sec. 6; least squares over the pixels) against the FP64
oracle, through epical_set_model_pixels and epic_run."""
import numpy as np
import pytest

from oracle import epic_oracle as O
from paper_1603_02126_amd import synth

from ._helpers import GAIN_RTOL, IMAGE_RTOL, gain_err, gpu_run, image_err

pytestmark = pytest.mark.gpu


def _oracle_multi(wl, packed, pix):
    E = O.unpack(packed, wl.array.efmt)
    pb = O.Problem.from_workload(wl)
    pb.pix_lm = np.atleast_2d(pix)
    res = [O.run_channel_multi(E[:, c], pb, c, wl.g0[c]) for c in range(wl.array.n_chan)]
    return dict(image=np.stack([r["image"] for r in res]), gains=np.stack([r["gains"] for r in res], axis=1))


def _plan(wl, pix):
    from paper_1603_02126_amd import lib
    plan = lib.Plan([wl.array])
    plan.set_model_pixels(0, wl.model_lmS, pix, wl.gamma, wl.t_cal)
    return plan


@pytest.mark.parametrize("n,efmt,kernel,na,n_samples,t_cal,pix_idx", [
    (32, synth.FMT_CI8, 2, 48, 230, 50, [0, 3]),
    (64, synth.FMT_CI4, 2, 200, 301, 100, [0, 2, 5]),
    (128, synth.FMT_CI8, 2, 150, 120, 30, [0, 1, 4, 7]),
    (16, synth.FMT_CF32, 1, 30, 64, 7, [0, 6]),
])
def test_multi_pixel_run_matches_oracle(cuda, n, efmt, kernel, na, n_samples, t_cal, pix_idx):
    wl = synth.config_small(n=n, efmt=efmt, kernel=kernel, n_ant=na, n_samples=n_samples, t_cal=t_cal)
    packed = synth.make_efield(wl)
    pix = wl.src_lmS[pix_idx, :2]
    ref = _oracle_multi(wl, packed, pix)
    plan = _plan(wl, pix)
    got = gpu_run(wl, packed, cuda, plan=plan)
    plan.close()
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


def test_one_pixel_is_the_single_pixel_path(cuda):
    wl = synth.config_small(n=64, n_ant=180, n_samples=160, t_cal=40)
    packed = synth.make_efield(wl)
    plan = _plan(wl, wl.cal_lm)
    got = gpu_run(wl, packed, cuda, plan=plan)
    plan.close()
    ref = gpu_run(wl, packed, cuda)
    np.testing.assert_array_equal(got["hist"], ref["hist"])
    np.testing.assert_array_equal(got["image"], ref["image"])


def test_uneven_array_with_its_three_calibrators(cuda):
    """An array of the uneven workload (128 antennas, 64 x 64) calibrated on
    its three calibrators at once."""
    wl = synth.config_uneven(n_chan=3, n_samples=300)[1]
    packed = synth.make_efield(wl)
    pix = wl.src_lmS[:3, :2]
    ref = _oracle_multi(wl, packed, pix)
    plan = _plan(wl, pix)
    got = gpu_run(wl, packed, cuda, plan=plan)
    plan.close()
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


def test_stagewise_update_needs_one_pixel(cuda):
    import torch
    from paper_1603_02126_amd import lib
    wl = synth.config_small(n_chan=1, n_samples=20, t_cal=10)
    plan = _plan(wl, wl.src_lmS[:2, :2])
    a = wl.array
    e = torch.from_numpy(synth.make_efield(wl)).to(cuda)
    tap = torch.zeros((10, 1), dtype=torch.complex64, device=cuda)
    kq = torch.zeros((1, a.n_ant, 4), dtype=torch.float64, device=cuda)
    g = torch.ones((1, a.n_ant), dtype=torch.complex128, device=cuda)
    with pytest.raises(lib.EpicError):
        plan.epical_update(0, e, 0, 10, tap, kq, g, finalize=True)
    plan.close()


def _run_pixels(wl, packed, pix, overlap, dev):
    from paper_1603_02126_amd import lib
    plan = _plan(wl, pix)
    plan.set_option(lib.OPT_OVERLAP, overlap)
    plan.set_option(lib.OPT_TIMING, 1)
    got = gpu_run(wl, packed, dev, plan=plan)
    tim = plan.timing()
    plan.close()
    return got, tim


@pytest.mark.parametrize("n,efmt,na,n_samples,t_cal,pix_idx", [
    (64, synth.FMT_CI4, 200, 301, 100, [0, 2, 5]),        # paired engine, ragged last interval
    (64, synth.FMT_CI8, 256, 250, 7, [0, 1, 2, 3]),       # four pixels, many short intervals
    (128, synth.FMT_CI8, 512, 90, 40, [0, 4]),            # class-pair engine, the largest fused array
    (32, synth.FMT_CF32, 90, 120, 30, [0, 3]),            # eight-wave FFT engine, complex float
])
def test_fused_several_pixels_match_oracle_and_separate_launches(cuda, n, efmt, na, n_samples, t_cal, pix_idx):
    """Several tapped pixels in the fused run: the several-pixel solve runs as
    a task of the persistent launch at 512 threads and publishes u interval by
    interval.  Gains and images against the FP64 oracle, and the images
    against the separate launches (whose solve sums the same terms at 1024
    threads, in another order)."""
    from paper_1603_02126_amd import lib
    wl = synth.config_small(n=n, efmt=efmt, kernel=2, n_ant=na, n_chan=3, n_samples=n_samples, t_cal=t_cal)
    packed = synth.make_efield(wl)
    pix = wl.src_lmS[pix_idx, :2]
    ref = _oracle_multi(wl, packed, pix)
    fused, tf = _run_pixels(wl, packed, pix, 1, cuda)
    sep, ts = _run_pixels(wl, packed, pix, 0, cuda)
    assert tf[lib.TIMER_SOLVE][1] == 0 and tf[lib.TIMER_IMAGE][1] > 0     # one launch for both
    assert ts[lib.TIMER_SOLVE][1] == 1
    for got in (fused, sep):
        assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
        assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL
    assert gain_err(fused["hist"], sep["hist"]) <= 1e-8
    assert image_err(fused["image"], sep["image"]).max() <= 1e-5


def test_several_pixels_above_512_antennas_run_separately(cuda):
    """Above 512 antennas the several-pixel solve needs its own 1024-thread
    launch: the run keeps the separate launches with the fused option on and
    still matches the oracle."""
    from paper_1603_02126_amd import lib
    wl = synth.config_small(n=128, efmt=synth.FMT_CI4, kernel=2, n_ant=600, n_chan=2, n_samples=60, t_cal=20)
    packed = synth.make_efield(wl)
    pix = wl.src_lmS[[0, 3], :2]
    ref = _oracle_multi(wl, packed, pix)
    got, tim = _run_pixels(wl, packed, pix, 1, cuda)
    assert tim[lib.TIMER_SOLVE][1] == 1
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


def test_fused_several_pixels_graph_replays(cuda):
    """The fused several-pixel run captured in a hipGraph: replays with eager
    work in between, each equal to the eager fused run (gains bit for bit)."""
    import torch
    from paper_1603_02126_amd import lib
    wl = synth.config_small(n=64, efmt=synth.FMT_CI4, kernel=2, n_ant=200, n_chan=3, n_samples=160, t_cal=40)
    packed = synth.make_efield(wl)
    pix = wl.src_lmS[[0, 2, 5], :2]
    eager, te = _run_pixels(wl, packed, pix, 1, cuda)
    assert te[lib.TIMER_SOLVE][1] == 0
    plan = _plan(wl, pix)
    plan.set_option(lib.OPT_GRAPH, 1)
    for rep in range(3):
        got = gpu_run(wl, packed, cuda, plan=plan)
        torch.randn(1000, device=cuda).sum()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got["hist"], eager["hist"])
        assert image_err(got["image"], eager["image"]).max() <= 1e-6, rep
    plan.close()
