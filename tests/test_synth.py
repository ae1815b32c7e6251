"""The seeded input generators: determinism, channel independence, formats."""
import numpy as np

from paper_1603_02126_amd import synth


def test_same_seed_same_bytes():
    a = synth.make_efield(synth.config_small(n_samples=64))
    b = synth.make_efield(synth.config_small(n_samples=64))
    assert a.dtype == np.int8 and np.array_equal(a, b)
    c = synth.make_efield(synth.config_small(seed=12, n_samples=64))
    assert not np.array_equal(a, c)


def test_channel_subsets_regenerate_identically():
    wl = synth.config_lwa(n_chan=6, n_samples=50)
    full = synth.make_efield(wl)
    sub = synth.make_efield(wl, channels=[4, 1])
    assert full.shape == (50, 6, 256) and full.dtype == np.uint8
    assert np.array_equal(sub[:, 0], full[:, 4]) and np.array_equal(sub[:, 1], full[:, 1])
    thr = synth.make_efield(wl, threads=3)
    assert np.array_equal(thr, full)


def test_quantiser_rounds_half_up_and_clips():
    x = np.array([-9.0, -8.5, -0.5, -0.49, 0.5, 6.49, 6.5, 7.6, 100.0])
    assert synth.quantise(x, 1.0, -8, 7).tolist() == [-8, -8, 0, 0, 1, 6, 7, 7, 7]


def test_ci4_levels_and_rms():
    wl = synth.config_lwa(n_chan=2, n_samples=400)
    p = synth.make_efield(wl)
    hi = (p.astype(np.int16) >> 4)
    hi = np.where(hi >= 8, hi - 16, hi)
    rms = np.sqrt(np.mean(hi.astype(np.float64) ** 2))
    assert 1.5 < rms < 2.6, rms


def test_layouts():
    hexa = synth.layout_hex(350, 14.0)
    assert hexa.shape == (350, 2)
    d = np.hypot(*(hexa[:, None, :] - hexa[None, :, :]).transpose(2, 0, 1))
    np.fill_diagonal(d, np.inf)
    np.testing.assert_allclose(d.min(), 14.0, rtol=1e-12)
    disk = synth.layout_uniform_disk(np.random.default_rng(0), 256, 50.0)
    assert disk.shape == (256, 2) and np.all(np.hypot(disk[:, 0], disk[:, 1]) <= 50.0)


def test_configs_fit_their_grids():
    for name in ("lwa", "hera", "diff"):
        wl = synth.CONFIGS[name](n_chan=2, n_samples=10)
        a = wl.array
        px = (a.ant_xy[:, 0] - a.x0) / a.dx
        py = (a.ant_xy[:, 1] - a.y0) / a.dy
        assert px.min() >= 1 and px.max() < a.nx - 2 and py.min() >= 1 and py.max() < a.ny - 2, name
