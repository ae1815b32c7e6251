"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and its host-side plan logic (grid cells, calibrator pixel,
pixel response, model denominator, argument checks) agrees with the oracle.
No device work is done here."""
import ctypes
import dataclasses

import numpy as np
import pytest

from oracle import epic_oracle as O
from paper_1603_02126_amd import lib, synth


def test_library_exports_every_header_function():
    L = lib.load()
    names = lib.header_functions()
    assert len(names) >= 14, names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(lib._SIGS), set(names) ^ set(lib._SIGS)
    assert L.epic_abi_version() == 2


@pytest.mark.parametrize("cfg", ["tiny", "small", "lwa", "hera"])
def test_grid_cells_bit_exact(cfg):
    wl = synth.CONFIGS[cfg](n_chan=2) if cfg in ("lwa", "hera", "small") else synth.CONFIGS[cfg]()
    a = wl.array
    ixy, w = lib.host_grid_cells(a)
    c = O.grid_cells(a.ant_xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    assert np.array_equal(ixy[..., 0], c.ix) and np.array_equal(ixy[..., 1], c.iy)
    assert np.array_equal(w, c.w)


def test_grid_cells_ties_and_wrap():
    spec = synth.ArraySpec(ant_xy=np.array([[1.25, 0.0], [-0.25, 15.8], [-0.3, 0.74], [7.75, 7.75]]),
                           freq_hz=np.array([1e8]), nx=32, ny=32, dx=0.5, dy=0.5, x0=0.0, y0=0.0,
                           kernel=1, efmt=0)
    ixy, w = lib.host_grid_cells(spec)
    c = O.grid_cells(spec.ant_xy, 0.5, 0.5, 0.0, 0.0, 32, 32, 1)
    assert ixy[:, 0, 0].tolist() == c.ix[:, 0].tolist() == [3, 0, 31, 16]
    assert ixy[:, 0, 1].tolist() == c.iy[:, 0].tolist() == [0, 0, 1, 16]


@pytest.mark.parametrize("cfg", ["tiny", "small", "lwa"])
def test_calibrator_tables_match_oracle(cfg):
    wl = synth.CONFIGS[cfg](n_chan=3) if cfg in ("lwa", "small") else synth.CONFIGS[cfg]()
    flags = np.zeros(wl.array.n_ant, np.uint8)
    flags[[1, 5]] = 1
    arr = synth.dataclasses.replace(wl.array, ant_flag=flags)
    wl = wl.replace(array=arr)
    k0, A, D = lib.host_calibrator(arr, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
    pb = O.Problem.from_workload(wl)
    for f in range(arr.n_chan):
        s = O.channel_setup(pb, f)
        assert tuple(k0[f]) == s["k0"]
        np.testing.assert_allclose(A[f], s["A"], rtol=0, atol=1e-13)
        scale = np.abs(s["D"]).max()
        np.testing.assert_allclose(D[f], s["D"], rtol=0, atol=1e-11 * scale)


def test_offcentre_calibrator_pixel():
    wl = synth.config_hera(n_chan=4)
    k0, A, D = lib.host_calibrator(wl.array, wl.model_lmS, wl.cal_lm)
    for f in range(4):
        assert tuple(k0[f]) == O.pixel_of_direction(wl.cal_lm[0], wl.cal_lm[1], wl.array.freq_hz[f],
                                                    128, 128, 2.5, 2.5)
    assert not np.all(k0 == 0)


@pytest.mark.parametrize("field,value,code", [
    ("n_ant", 0, lib.EPIC_ERR_ARG), ("nx", 48, lib.EPIC_ERR_ARG), ("kernel", 3, lib.EPIC_ERR_ARG),
    ("efmt", 7, lib.EPIC_ERR_ARG), ("dx", -1.0, lib.EPIC_ERR_ARG), ("dx", float("nan"), lib.EPIC_ERR_ARG)])
def test_descriptor_errors(field, value, code):
    wl = synth.config_tiny()
    h = lib._DescHolder(wl.array)
    setattr(h.desc, field, value)
    ixy = np.zeros((64, 4, 2), np.int32)
    w = np.zeros((64, 4))
    rc = lib.load().epic_host_grid_cells(ctypes.byref(h.desc), ixy.ctypes.data, w.ctypes.data)
    assert rc == code
    assert lib.last_error()


@pytest.mark.parametrize("gamma,t_cal,n_src", [(1.0, 1, 1), (-0.1, 1, 1), (0.5, 0, 1), (0.5, 1, 0)])
def test_model_errors(gamma, t_cal, n_src):
    wl = synth.config_tiny()
    h = lib._DescHolder(wl.array)
    m = lib._ModelHolder(wl.model_lmS, wl.cal_lm, gamma, t_cal)
    m.desc.n_src = n_src
    rc = lib.load().epic_host_calibrator(ctypes.byref(h.desc), ctypes.byref(m.desc), None, None, None)
    assert rc == lib.EPIC_ERR_ARG
    assert "gamma" in lib.last_error() or "t_cal" in lib.last_error() or "source" in lib.last_error()


def test_null_pointers_rejected():
    L = lib.load()
    assert L.epic_host_grid_cells(None, None, None) == lib.EPIC_ERR_ARG
    assert L.epic_plan_create(None, 1, ctypes.byref(ctypes.c_void_p())) == lib.EPIC_ERR_ARG
    assert L.epic_plan_destroy(None) == lib.EPIC_OK
    assert L.epic_grid(None, 0, None, 0, 0, None, None, None) == lib.EPIC_ERR_ARG
    assert L.epic_run(None, None, 1, None, None, None, None, None) == lib.EPIC_ERR_ARG


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    monkeypatch.setattr(lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        lib.load()


def test_pixel_tables_match_oracle():
    """Tables of several tapped pixels (k_p, A_p, D_p) against the oracle."""
    wl = synth.config_small(n_chan=2)
    flags = np.zeros(wl.array.n_ant, np.uint8)
    flags[[2, 9]] = 1
    arr = synth.dataclasses.replace(wl.array, ant_flag=flags)
    wl = wl.replace(array=arr)
    pix = wl.src_lmS[[0, 3, 6], :2]
    k, A, D = lib.host_calibrator_pixels(arr, wl.model_lmS, pix, wl.gamma, wl.t_cal)
    pb = O.Problem.from_workload(wl)
    pb.pix_lm = pix
    for f in range(arr.n_chan):
        s = O.pixel_setup(pb, f)
        np.testing.assert_array_equal(k[:, f], s["k"])
        np.testing.assert_allclose(A[:, f], s["A_p"], rtol=0, atol=1e-13)
        scale = np.abs(s["D_p"]).max()
        np.testing.assert_allclose(D[:, f], s["D_p"], rtol=0, atol=1e-11 * scale)
    # one pixel at the calibrator is the single-pixel table
    k1, A1, D1 = lib.host_calibrator_pixels(arr, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
    k0, A0, D0 = lib.host_calibrator(arr, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
    np.testing.assert_array_equal(k1[0], k0)
    np.testing.assert_array_equal(A1[0], A0)
    np.testing.assert_array_equal(D1[0], D0)


@pytest.mark.parametrize("n_pix", [0, 5])
def test_pixel_count_errors(n_pix):
    wl = synth.config_small(n_chan=1)
    pix = np.zeros((max(n_pix, 1), 2))
    with pytest.raises(lib.EpicError):
        d = lib._DescHolder(wl.array)
        m = lib._ModelHolder(wl.model_lmS, wl.cal_lm, 0.5, 10)
        lib._check(lib.load().epic_host_calibrator_pixels(ctypes.byref(d.desc), ctypes.byref(m.desc),
                                                          pix.ctypes.data, n_pix, None, None, None))


@pytest.mark.parametrize("b0,b1", [(0, 5), (1, 4), (2, 3)])
def test_band_coordinate_matches_oracle(b0, b1):
    """The library's band coordinate (epical_set_band) against the oracle's."""
    wl = synth.config_small(n_chan=5)
    got = lib.host_band_coordinate(wl.array, b0, b1)
    want = np.zeros(5)
    want[b0:b1] = O.band_coordinate(wl.array.freq_hz, b0, b1)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-15)


def test_band_coordinate_reversed_frequencies():
    wl = synth.config_small(n_chan=4)
    arr = dataclasses.replace(wl.array, freq_hz=wl.array.freq_hz[::-1].copy())
    got = lib.host_band_coordinate(arr, 0, 4)
    np.testing.assert_allclose(got, O.band_coordinate(arr.freq_hz, 0, 4), atol=1e-15)
    assert got[0] == -1.0 and got[-1] == 1.0


@pytest.mark.parametrize("b0,b1", [(-1, 2), (2, 2), (3, 1), (0, 6)])
def test_band_range_errors(b0, b1):
    wl = synth.config_small(n_chan=5)
    with pytest.raises(lib.EpicError):
        lib.host_band_coordinate(wl.array, b0, b1)
