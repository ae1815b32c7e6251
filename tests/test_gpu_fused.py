"""GPU parity of the fused run (EPIC_OPT_OVERLAP): one launch for the
calibration solve and the imaging, the solve publishing each interval's u and
the imaging items waiting for the intervals they need.  Against the FP64
oracle, and against the separate launches (gains bit for bit: both run the
same single-pixel solve)."""
import numpy as np
import pytest

from paper_1603_02126_amd import synth

from ._helpers import GAIN_RTOL, IMAGE_RTOL, gain_err, gpu_run, image_err, oracle_run

pytestmark = pytest.mark.gpu


def _plan(wls, overlap, opts=None):
    from paper_1603_02126_amd import lib
    plan = lib.Plan([w.array for w in wls])
    for i, w in enumerate(wls):
        plan.set_model(i, w.model_lmS, w.cal_lm, w.gamma, w.t_cal)
    plan.set_option(lib.OPT_OVERLAP, overlap)
    for k, v in (opts or {}).items():
        plan.set_option(k, v)
    return plan


def _run(plan, wls, packs, dev):
    import torch
    es = [torch.from_numpy(p).to(dev) for p in packs]
    gs = [torch.from_numpy(w.g0.copy()).to(dev) for w in wls]
    imgs = [torch.zeros((w.array.n_chan, w.array.ny, w.array.nx), dtype=torch.float32, device=dev) for w in wls]
    hs = [torch.zeros((-(-w.n_samples // w.t_cal) + 1, w.array.n_chan, w.array.n_ant), dtype=torch.complex128,
                      device=dev) for w in wls]
    plan.run(es, wls[0].n_samples, gs, imgs, gain_hist=hs)
    torch.cuda.synchronize()
    return [h.cpu().numpy() for h in hs], [i.cpu().numpy() for i in imgs]


@pytest.mark.parametrize("n,efmt,na,n_samples,t_cal", [
    (64, synth.FMT_CI4, 200, 301, 100),      # paired engine, ragged last interval
    (64, synth.FMT_CI8, 100, 250, 7),        # many short intervals
    (32, synth.FMT_CF32, 90, 120, 30),       # eight-wave FFT engine
    (128, synth.FMT_CI8, 350, 60, 20),       # class-pair engine
    (256, synth.FMT_CI4, 700, 40, 9),        # dense class engine, two solve slots per thread
])
def test_fused_run_matches_oracle_and_separate_launches(cuda, n, efmt, na, n_samples, t_cal):
    wl = synth.config_small(n=n, efmt=efmt, kernel=2, n_ant=na, n_chan=3, n_samples=n_samples, t_cal=t_cal)
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    fused = _plan([wl], 1)
    (hf,), (imf,) = _run(fused, [wl], [packed], cuda)
    fused.close()
    sep = _plan([wl], 0)
    (hs,), (ims,) = _run(sep, [wl], [packed], cuda)
    sep.close()
    assert gain_err(hf, ref["gains"]) <= GAIN_RTOL
    assert image_err(imf, ref["image"]).max() <= IMAGE_RTOL
    np.testing.assert_array_equal(hf, hs)
    assert image_err(imf, ims).max() <= 1e-6


def test_fused_batch_of_uneven_arrays(cuda):
    """Four arrays of uneven size in one fused launch (solve tasks of every
    array first, then their imaging items), against the oracle and the
    separate launches."""
    wls = synth.config_uneven(n_chan=2, n_samples=70, n_ants=(40, 200, 160, 600), grids=(32, 64, 128, 256))
    packs = [synth.make_efield(w) for w in wls]
    hf, imf = _run(_plan(wls, 1), wls, packs, cuda)
    hs, ims = _run(_plan(wls, 0), wls, packs, cuda)
    for w, p, h1, h0, i1, i0 in zip(wls, packs, hf, hs, imf, ims):
        ref = oracle_run(w, p)
        assert gain_err(h1, ref["gains"]) <= GAIN_RTOL, w.name
        assert image_err(i1, ref["image"]).max() <= IMAGE_RTOL, w.name
        np.testing.assert_array_equal(h1, h0)
        assert image_err(i1, i0).max() <= 1e-6


def test_fused_graph_replays(cuda):
    """The fused launch captured in a hipGraph: several replays with eager
    work in between, each equal to the eager fused run."""
    import torch
    from paper_1603_02126_amd import lib
    wls = synth.config_uneven(n_chan=2, n_samples=50, n_ants=(40, 200), grids=(32, 64))
    packs = [synth.make_efield(w) for w in wls]
    he, ie = _run(_plan(wls, 1), wls, packs, cuda)
    graph = _plan(wls, 1, {lib.OPT_GRAPH: 1})
    for rep in range(3):
        hg, ig = _run(graph, wls, packs, cuda)
        torch.randn(1000, device=cuda).sum()
        torch.cuda.synchronize()
        for k in range(len(wls)):
            np.testing.assert_array_equal(hg[k], he[k])
            assert image_err(ig[k], ie[k]).max() <= 1e-6, (rep, k)
    graph.close()


def test_ineligible_plan_runs_separately(cuda):
    """A tiny array (one-wave solve) or a band model keeps the separate
    launches; the run still matches the oracle with the option on."""
    from paper_1603_02126_amd import lib
    wl = synth.config_tiny()
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL
    with lib.Plan([wl.array]) as plan:
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        plan.set_option(lib.OPT_TIMING, 1)
        gpu_run(wl, packed, cuda, plan=plan)
        tim = plan.timing()
        assert tim[lib.TIMER_SOLVE][1] == 1      # its own solve launch


def test_fused_wait_bound_gives_nan_images_not_a_hang(cuda):
    """The imaging's bounded wait for the calibration, forced short from the
    host: every kernel still ends, the gains are those of the separate
    launches bit for bit, and the images are either the right ones (every wait
    ended in time) or NaN throughout (a wait gave up), never a silent mix."""
    from paper_1603_02126_amd import lib
    wl = synth.config_small(n=64, efmt=synth.FMT_CI4, kernel=2, n_ant=200, n_chan=3, n_samples=301, t_cal=100)
    packed = synth.make_efield(wl)
    sep = _plan([wl], 0)
    (hs,), (ims,) = _run(sep, [wl], [packed], cuda)
    sep.close()
    short = _plan([wl], 1, {lib.OPT_WAIT_POLLS: 1})
    (hf,), (imf,) = _run(short, [wl], [packed], cuda)
    np.testing.assert_array_equal(hf, hs)
    assert np.isnan(imf).all() or image_err(imf, ims).max() <= 1e-6
    # back to the default bound: the same plan runs clean again
    short.set_option(lib.OPT_WAIT_POLLS, 0)
    (hf,), (imf,) = _run(short, [wl], [packed], cuda)
    np.testing.assert_array_equal(hf, hs)
    assert image_err(imf, ims).max() <= 1e-6
    with pytest.raises(lib.EpicError):
        short.set_option(lib.OPT_WAIT_POLLS, (1 << 23) + 1)
    short.close()
