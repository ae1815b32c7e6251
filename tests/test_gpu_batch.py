"""GPU parity of the batched form: several arrays of uneven antenna count and
grid size in one launch per stage (persistent imaging kernel over a work
queue), its hipGraph capture and replay, and the autotuner -- each against the
FP64 oracle or the plain per-array path."""
import numpy as np
import pytest

from paper_1603_02126_amd import synth

from ._helpers import GAIN_RTOL, IMAGE_RTOL, gain_err, image_err, oracle_run

pytestmark = pytest.mark.gpu


def _run(plan, wls, packs, dev, n_repeat=1):
    import torch
    es = [torch.from_numpy(p).to(dev) for p in packs]
    outs = []
    for _ in range(n_repeat):
        gs = [torch.from_numpy(w.g0.copy()).to(dev) for w in wls]
        imgs = [torch.zeros((w.array.n_chan, w.array.ny, w.array.nx), dtype=torch.float32, device=dev) for w in wls]
        plan.run(es, wls[0].n_samples, gs, imgs)
        torch.cuda.synchronize()
        outs.append(([g.cpu().numpy() for g in gs], [i.cpu().numpy() for i in imgs]))
    return outs


def _plan(wls, opts=None):
    from paper_1603_02126_amd import lib
    plan = lib.Plan([w.array for w in wls])
    for i, w in enumerate(wls):
        plan.set_model(i, w.model_lmS, w.cal_lm, w.gamma, w.t_cal)
    for k, v in (opts or {}).items():
        plan.set_option(k, v)
    return plan


def _small_uneven(n_chan=3, n_samples=60):
    return synth.config_uneven(n_chan=n_chan, n_samples=n_samples, n_ants=(40, 200, 160, 600),
                               grids=(32, 64, 128, 256))


def test_batched_uneven_arrays_match_oracle(cuda):
    wls = _small_uneven()
    packs = [synth.make_efield(w) for w in wls]
    plan = _plan(wls)           # several arrays: batched by default
    (gs, imgs), = _run(plan, wls, packs, cuda)
    for w, p, g, img in zip(wls, packs, gs, imgs):
        ref = oracle_run(w, p)
        assert gain_err(g, ref["gains"][-1]) <= GAIN_RTOL, w.name
        assert image_err(img, ref["image"]).max() <= IMAGE_RTOL, w.name
    plan.close()


def test_batched_equals_per_array(cuda):
    from paper_1603_02126_amd import lib
    wls = _small_uneven(n_chan=2, n_samples=70)
    packs = [synth.make_efield(w) for w in wls]
    a = _plan(wls, {lib.OPT_BATCH: 1})
    b = _plan(wls, {lib.OPT_BATCH: 2})
    (ga, ia), = _run(a, wls, packs, cuda)
    (gb, ib), = _run(b, wls, packs, cuda)
    for k in range(len(wls)):
        np.testing.assert_array_equal(ga[k], gb[k])
        assert image_err(ia[k], ib[k]).max() <= 1e-6
    a.close()
    b.close()


def test_graph_replays_match_eager(cuda):
    """Capture once, replay several times with eager work and synchronisation
    in between; every replay equals the eager result."""
    import torch
    from paper_1603_02126_amd import lib
    wls = _small_uneven(n_chan=2, n_samples=50)
    packs = [synth.make_efield(w) for w in wls]
    eager = _plan(wls, {lib.OPT_BATCH: 1})
    (ge, ie), = _run(eager, wls, packs, cuda)
    graph = _plan(wls, {lib.OPT_BATCH: 1, lib.OPT_GRAPH: 1})
    es = [torch.from_numpy(p).to(cuda) for p in packs]
    gs = [torch.zeros((w.array.n_chan, w.array.n_ant), dtype=torch.complex128, device=cuda) for w in wls]
    imgs = [torch.zeros((w.array.n_chan, w.array.ny, w.array.nx), dtype=torch.float32, device=cuda) for w in wls]
    for rep in range(4):
        for g, w in zip(gs, wls):
            g.copy_(torch.from_numpy(w.g0))
        for img in imgs:
            img.fill_(float(rep) - 7.0)          # eager work between replays
        graph.run(es, wls[0].n_samples, gs, imgs)
        torch.cuda.synchronize()
        x = torch.randn(1000, device=cuda).sum()   # more eager work
        torch.cuda.synchronize()
        for k in range(len(wls)):
            np.testing.assert_array_equal(gs[k].cpu().numpy(), ge[k])
            assert image_err(imgs[k].cpu().numpy(), ie[k]).max() <= 1e-6, (rep, k)
    eager.close()
    graph.close()


def test_autotune_then_run_matches_oracle(cuda):
    import torch
    wls = _small_uneven(n_chan=2, n_samples=80)
    packs = [synth.make_efield(w) for w in wls]
    plan = _plan(wls)
    es = [torch.from_numpy(p).to(cuda) for p in packs]
    tuning = plan.autotune(es, wls[0].n_samples)
    assert len(tuning) == len(wls) and all(t[0] in (1, 2, 3, 4) and t[1] >= 1 and t[2] in (0, 2, 4) for t in tuning)
    (gs, imgs), = _run(plan, wls, packs, cuda)
    for w, p, g, img in zip(wls, packs, gs, imgs):
        ref = oracle_run(w, p)
        assert gain_err(g, ref["gains"][-1]) <= GAIN_RTOL, w.name
        assert image_err(img, ref["image"]).max() <= IMAGE_RTOL, w.name
    plan.close()


def test_graph_follows_option_changes_and_new_inputs(cuda):
    """With graph replay on, changing the time splits or the transform, or the
    number of samples, between two calls (no synchronisation in between)
    re-records the graph: each call matches the FP64 oracle on fresh E-field
    contents."""
    import torch
    from paper_1603_02126_amd import lib
    wls = _small_uneven(n_chan=2, n_samples=90)
    packs = [synth.make_efield(w) for w in wls]
    alt = [synth.make_efield(w.replace(seed=w.seed + 77)) for w in wls]
    plan = _plan(wls, {lib.OPT_BATCH: 1, lib.OPT_GRAPH: 1})
    es = [torch.from_numpy(p).to(cuda) for p in packs]
    calls = [({lib.OPT_SPLITS: 3}, packs, 90), ({lib.OPT_SPLITS: 1}, alt, 90), ({lib.OPT_TRANSFORM: 2}, packs, 90),
             ({lib.OPT_TRANSFORM: 1, lib.OPT_SPLITS: 5}, alt, 61)]
    outs = []
    for opts, src, T in calls:
        for k, v in opts.items():
            plan.set_option(k, v)
        for e, p in zip(es, src):
            e.copy_(torch.from_numpy(p), non_blocking=False)
        gs = [torch.from_numpy(w.g0.copy()).to(cuda) for w in wls]
        imgs = [torch.zeros((w.array.n_chan, w.array.ny, w.array.nx), dtype=torch.float32, device=cuda) for w in wls]
        plan.run(es, T, gs, imgs)
        outs.append(([g.clone() for g in gs], [i.clone() for i in imgs]))
    torch.cuda.synchronize()
    for (opts, src, T), (gs, imgs) in zip(calls, outs):
        for w, p, g, img in zip(wls, src, gs, imgs):
            w2 = w.replace(n_samples=T)
            ref = oracle_run(w2, p[:T])
            assert gain_err(g.cpu().numpy(), ref["gains"][-1]) <= GAIN_RTOL, (opts, w.name)
            assert image_err(img.cpu().numpy(), ref["image"]).max() <= IMAGE_RTOL, (opts, w.name)
    plan.close()


def test_autotune_cache_round_trip(cuda, tmp_path):
    """The tuning cache: a first autotune writes one entry per array, a
    second plan takes them without timing (same choices), and a run with the
    cached tuning matches the FP64 oracle."""
    import json
    import torch
    wls = _small_uneven(n_chan=2, n_samples=60)
    packs = [synth.make_efield(w) for w in wls]
    es = [torch.from_numpy(p).to(cuda) for p in packs]
    path = str(tmp_path / "tune.json")
    a = _plan(wls)
    ta = a.autotune(es, 60, cache=path)
    a.close()
    entries = json.load(open(path))
    assert len(entries) == len(wls) and all("|N=" in k for k in entries)
    b = _plan(wls)
    tb = b.autotune(es, 60, cache=path)
    assert [t[:3] for t in tb] == [t[:3] for t in ta]
    (gs, imgs), = _run(b, wls, packs, cuda)
    for w, p, g, img in zip(wls, packs, gs, imgs):
        ref = oracle_run(w, p)
        assert gain_err(g, ref["gains"][-1]) <= GAIN_RTOL, w.name
        assert image_err(img, ref["image"]).max() <= IMAGE_RTOL, w.name
    b.close()
