"""GPU checks of the boundary calls that expose the plan's device state: the
imaging engines' integer unpacking (epic_debug_unpack, bit-exact for every
code), the read-back gridding tables (epic_plan_get_cells, equal to the
oracle's cells of eq. gridding), a caller-supplied model denominator
(epical_set_denominator, eq. cal_solution) against the oracle run with the
same D, and the 256-byte alignment rule for caller buffers."""
import numpy as np
import pytest

from oracle import epic_oracle as O
from paper_1603_02126_amd import synth

from ._helpers import GAIN_RTOL, IMAGE_RTOL, gain_err, gpu_run, image_err

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1603_02126_amd import lib
    return lib


def _one_cell_array(efmt, n_ant=64):
    xy = np.stack([np.arange(n_ant) % 16 * 1.0, np.arange(n_ant) // 16 * 1.0], axis=1)
    return synth.ArraySpec(ant_xy=xy, freq_hz=np.array([5e7]), nx=16, ny=16, dx=1.0, dy=1.0, x0=0.0, y0=0.0,
                           kernel=1, efmt=efmt)


def test_debug_unpack_ci4_every_code(cuda):
    import torch
    codes = np.arange(256, dtype=np.uint8)
    with _lib().Plan([_one_cell_array(synth.FMT_CI4)]) as plan:
        got = plan.debug_unpack(0, torch.from_numpy(codes).to(cuda)).cpu().numpy()
    want = O.unpack(codes, O.FMT_CI4)
    np.testing.assert_array_equal(got[:, 0].astype(np.float64), want.real)
    np.testing.assert_array_equal(got[:, 1].astype(np.float64), want.imag)


def test_debug_unpack_ci8_every_pair(cuda):
    import torch
    v = np.arange(-128, 128)
    re, im = np.meshgrid(v, v, indexing="ij")
    packed = np.stack([re.ravel(), im.ravel()], -1).astype(np.int8)      # 65,536 (re, im) pairs
    with _lib().Plan([_one_cell_array(synth.FMT_CI8)]) as plan:
        got = plan.debug_unpack(0, torch.from_numpy(packed).to(cuda)).cpu().numpy()
    want = O.unpack(packed, O.FMT_CI8)
    np.testing.assert_array_equal(got[:, 0].astype(np.float64), want.real)
    np.testing.assert_array_equal(got[:, 1].astype(np.float64), want.imag)


def test_debug_unpack_float_format_is_unsupported(cuda):
    import torch
    lib = _lib()
    with lib.Plan([_one_cell_array(synth.FMT_CF32)]) as plan:
        with pytest.raises(lib.EpicError, match="UNSUPPORTED"):
            plan.debug_unpack(0, torch.zeros((4, 2), dtype=torch.float32, device=cuda))


@pytest.mark.parametrize("n,kernel,na,flagged", [(32, 2, 48, ()), (64, 1, 300, ()), (256, 2, 700, (0, 5, 699)),
                                                 (16, 2, 30, (3,))])
def test_plan_cells_match_oracle(cuda, n, kernel, na, flagged):
    """The device tables read back equal the oracle's cells and weights
    (indices bit-exact, weights rounded once to float32; flagged antennas
    carry weight zero)."""
    wl = synth.config_small(n=n, kernel=kernel, n_ant=na, n_chan=1, n_samples=4)
    a = wl.array
    if flagged:
        flags = np.zeros(na, np.uint8)
        flags[list(flagged)] = 1
        a = synth.dataclasses.replace(a, ant_flag=flags)
    with _lib().Plan([a]) as plan:
        ixy, w = plan.get_cells(0)
    c = O.grid_cells(a.ant_xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    np.testing.assert_array_equal(ixy[..., 0], np.asarray(c.ix))
    np.testing.assert_array_equal(ixy[..., 1], np.asarray(c.iy))
    want_w = np.asarray(c.w, np.float64).astype(np.float32)
    if flagged:
        want_w[list(flagged)] = 0
    np.testing.assert_array_equal(w, want_w)


def _oracle_with_denominator(wl, packed, D):
    """The oracle loop with the model denominator replaced by D [F, Na]."""
    pb = O.Problem.from_workload(wl)
    E = O.unpack(packed, wl.array.efmt)
    res = []
    for f in range(wl.array.n_chan):
        s = O.channel_setup(pb, f)
        s = dict(s, D=np.asarray(D[f], np.complex128))
        res.append(O.run_channel(E[:, f], pb, f, wl.g0[f], setup=s))
    return dict(image=np.stack([r["image"] for r in res]), gains=np.stack([r["gains"] for r in res], axis=1),
                held=np.stack([r["held"] for r in res], axis=1))


def test_set_denominator_of_the_same_model_changes_nothing(cuda):
    """D computed by the library for the plan's own model, handed back through
    epical_set_denominator, gives bit-identical gains and images."""
    lib = _lib()
    wl = synth.config_small(n=32, n_ant=60, n_chan=3, n_samples=150, t_cal=50)
    packed = synth.make_efield(wl)
    base = gpu_run(wl, packed, cuda)
    _, _, D = lib.host_calibrator(wl.array, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
    with lib.Plan([wl.array]) as plan:
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        plan.set_denominator(0, D)
        got = gpu_run(wl, packed, cuda, plan=plan)
    np.testing.assert_array_equal(got["hist"], base["hist"])
    np.testing.assert_array_equal(got["image"], base["image"])


def test_set_denominator_from_another_model_matches_oracle(cuda):
    """A caller-held model (here: the calibrator alone, scaled by 1.3, and one
    antenna whose D is zeroed) replaces the plan's D; the oracle runs the loop
    with the same D.  The zeroed antenna is held (EPIC_ANT_D_ZERO)."""
    lib = _lib()
    wl = synth.config_small(n=64, efmt=synth.FMT_CI4, n_ant=160, n_chan=2, n_samples=200, t_cal=50)
    packed = synth.make_efield(wl)
    _, _, D = lib.host_calibrator(wl.array, wl.model_lmS[:1] * np.array([1.0, 1.0, 1.3]), wl.cal_lm, wl.gamma,
                                  wl.t_cal)
    D[:, 17] = 0.0
    with lib.Plan([wl.array]) as plan:
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        plan.set_denominator(0, D)
        got = gpu_run(wl, packed, cuda, plan=plan)
    ref = _oracle_with_denominator(wl, packed, D)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL
    assert np.all(ref["held"][:, :, 17])
    assert np.all(got["status"][:, 17] == lib.ANT_D_ZERO)
    np.testing.assert_array_equal(got["gains"][:, 17], wl.g0[:, 17])


def test_set_denominator_errors(cuda):
    lib = _lib()
    wl = synth.config_small(n=32, n_ant=40, n_chan=2, n_samples=10)
    D = np.ones((2, 40), np.complex128)
    with lib.Plan([wl.array]) as plan:
        with pytest.raises(lib.EpicError, match="EPIC_ERR_STATE"):
            plan.set_denominator(0, D)                  # no model yet
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        D[1, 3] = np.nan
        with pytest.raises(lib.EpicError, match="finite"):
            plan.set_denominator(0, D)


def test_misaligned_buffers_are_rejected(cuda):
    """A device buffer that does not start on a 256-byte boundary is an
    EPIC_ERR_ARG before anything is enqueued."""
    import torch
    lib = _lib()
    wl = synth.config_small(n=32, n_ant=40, n_chan=2, n_samples=30, t_cal=10)
    a = wl.array
    e = torch.from_numpy(synth.make_efield(wl)).to(cuda)
    with lib.Plan([a]) as plan:
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        g = torch.from_numpy(wl.g0).to(cuda)
        img_store = torch.zeros(a.n_chan * a.ny * a.nx + 1, dtype=torch.float32, device=cuda)
        img = img_store[1:].view(a.n_chan, a.ny, a.nx)           # starts 4 bytes into its allocation
        with pytest.raises(lib.EpicError, match="image.*256-byte"):
            plan.run([e], 30, [g], [img])
        g_store = torch.zeros(a.n_chan * a.n_ant + 1, dtype=torch.complex128, device=cuda)
        g_off = g_store[1:].view(a.n_chan, a.n_ant)
        g_off.copy_(g)
        with pytest.raises(lib.EpicError, match="gains.*256-byte"):
            plan.run([e], 30, [g_off], [torch.zeros((a.n_chan, a.ny, a.nx), device=cuda)])
        assert float(img_store.abs().max()) == 0.0               # nothing ran
