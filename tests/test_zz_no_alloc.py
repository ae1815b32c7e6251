"""epic_run_noalloc: the calibrated loop with every intermediate in the
library's static device scratch.  Through the C ABI, two calls in a row on
one plan (the second with fewer samples and channels' worth of work) against
epic_run on the same inputs, and against the FP64 oracle; then a run too
large for the static scratch is rejected before anything is enqueued."""
import numpy as np
import pytest

from paper_1603_02126_amd import synth

from ._helpers import GAIN_RTOL, IMAGE_RTOL, gain_err, image_err, oracle_run

pytestmark = pytest.mark.gpu


def _buffers(wls, T, dev):
    import torch
    gs = [torch.from_numpy(w.g0.copy()).to(dev) for w in wls]
    imgs = [torch.full((w.array.n_chan, w.array.ny, w.array.nx), -1.0, dtype=torch.float32, device=dev)
            for w in wls]
    hs = [torch.zeros((-(-T // w.t_cal) + 1, w.array.n_chan, w.array.n_ant), dtype=torch.complex128, device=dev)
          for w in wls]
    st = [torch.zeros((w.array.n_chan, w.array.n_ant), dtype=torch.int32, device=dev) for w in wls]
    return gs, imgs, hs, st


def _np(ts):
    return [t.cpu().numpy() for t in ts]


def test_noalloc_run_matches_epic_run_twice(cuda):
    import torch
    from paper_1603_02126_amd import lib
    wls = [synth.config_small(n=64, efmt=synth.FMT_CI4, n_ant=256, n_chan=6, n_samples=400, t_cal=100, seed=21),
           synth.config_small(n=128, efmt=synth.FMT_CI8, n_ant=150, n_chan=3, n_samples=400, t_cal=50, seed=22),
           synth.config_small(n=32, efmt=synth.FMT_CF32, n_ant=40, n_chan=2, n_samples=400, t_cal=7, seed=23)]
    packs = [synth.make_efield(w) for w in wls]
    es = [torch.from_numpy(p).to(cuda) for p in packs]
    with lib.Plan([w.array for w in wls]) as plan:
        for i, w in enumerate(wls):
            plan.set_model(i, w.model_lmS, w.cal_lm, w.gamma, w.t_cal)
        plan.set_option(lib.OPT_BATCH, 2)
        for T, hist in ((400, True), (130, False)):          # the second call: a smaller input
            ref_b = _buffers(wls, T, cuda)
            plan.run(es, T, ref_b[0], ref_b[1], gain_hist=ref_b[2], status=ref_b[3])
            got_b = _buffers(wls, T, cuda)
            plan.run_noalloc(es, T, got_b[0], got_b[1], gain_hist=got_b[2] if hist else None, status=got_b[3])
            torch.cuda.synchronize()
            rg, ri, rh, rs = (_np(x) for x in ref_b)
            gg, gi, gh, gs = (_np(x) for x in got_b)
            for k, w in enumerate(wls):
                assert gain_err(gg[k], rg[k]) <= 1e-12, (T, k)
                assert image_err(gi[k], ri[k]).max() <= 1e-6, (T, k)
                np.testing.assert_array_equal(gs[k], rs[k])
                if hist:
                    assert gain_err(gh[k], rh[k]) <= 1e-12, (T, k)
                ref = oracle_run(w.replace(n_samples=T), packs[k][:T])
                assert gain_err(gg[k], ref["gains"][-1]) <= GAIN_RTOL, (T, k)
                assert image_err(gi[k], ref["image"]).max() <= IMAGE_RTOL, (T, k)


def test_noalloc_run_too_large_is_rejected(cuda):
    """The LWA shape without a caller gain history needs more than the static
    scratch even with one time split: EPIC_ERR_ARG, outputs untouched."""
    import torch
    from paper_1603_02126_amd import lib
    wl = synth.config_lwa(n_chan=128, n_samples=10000)
    a = wl.array
    e = torch.zeros((wl.n_samples, a.n_chan, a.n_ant), dtype=torch.uint8, device=cuda)
    g = torch.ones((a.n_chan, a.n_ant), dtype=torch.complex128, device=cuda)
    img = torch.full((a.n_chan, a.ny, a.nx), 3.0, dtype=torch.float32, device=cuda)
    with lib.Plan([a]) as plan:
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        with pytest.raises(lib.EpicError, match="static scratch"):
            plan.run_noalloc([e], wl.n_samples, [g], [img])
    torch.cuda.synchronize()
    assert float(img.min()) == 3.0 and float(img.max()) == 3.0
