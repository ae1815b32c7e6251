"""GPU parity: every entry point of the C ABI against the FP64 oracle on the
same seeded inputs.  Integer work (unpacking, cell indices) is bit-exact;
images agree within 1e-5 of the per-channel peak and gains within 1e-4
relative (FP32 hot path vs FP64 oracle)."""
import numpy as np
import pytest

from oracle import epic_oracle as O
from paper_1603_02126_amd import synth

from ._helpers import GAIN_RTOL, IMAGE_RTOL, gain_err, gpu_run, image_err, oracle_run

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _lib():
    from paper_1603_02126_amd import lib
    return lib


def _codes_array(n_ant, n, efmt, kernel=1):
    """n_ant antennas each on its own cell of an n x n grid (cell = index)."""
    a = np.arange(n_ant)
    xy = np.stack([(a % n) * 1.0, (a // n) * 1.0], axis=1)
    return synth.ArraySpec(ant_xy=xy, freq_hz=np.array([5e7]), nx=n, ny=n, dx=1.0, dy=1.0, x0=0.0, y0=0.0,
                           kernel=kernel, efmt=efmt)


# ---------------------------------------------------------------------------
# stage-wise entry points
# ---------------------------------------------------------------------------

def test_unpack_ci4_all_codes_bit_exact(cuda):
    torch = _torch()
    spec = _codes_array(256, 32, synth.FMT_CI4)
    codes = np.arange(256, dtype=np.uint8).reshape(1, 1, 256)
    with _lib().Plan([spec]) as plan:
        u = torch.ones((1, 256), dtype=torch.complex64, device=cuda)
        g = plan.grid(0, torch.from_numpy(codes).to(cuda), 0, 1, u).cpu().numpy()
    want = O.unpack(codes[0, 0], O.FMT_CI4)
    got = g[0, 0].reshape(-1)[:256]
    assert np.array_equal(got.real.astype(np.float64), want.real)
    assert np.array_equal(got.imag.astype(np.float64), want.imag)


def test_unpack_ci8_all_pairs_bit_exact(cuda):
    torch = _torch()
    spec = _codes_array(256, 32, synth.FMT_CI8)
    v = np.arange(-128, 128)
    re, im = np.meshgrid(v, v, indexing="ij")             # [256 t, 256 a]
    packed = np.stack([re, im], -1).astype(np.int8)[:, None]   # [T=256][F=1][Na=256][2]
    with _lib().Plan([spec]) as plan:
        u = torch.ones((1, 256), dtype=torch.complex64, device=cuda)
        g = plan.grid(0, torch.from_numpy(packed).to(cuda), 0, 256, u).cpu().numpy()
    got = g[:, 0].reshape(256, -1)[:, :256]
    assert np.array_equal(got.real, re.astype(np.float32)) and np.array_equal(got.imag, im.astype(np.float32))


@pytest.mark.parametrize("n,efmt,kernel,na", [(32, synth.FMT_CI8, 2, 48), (64, synth.FMT_CI4, 2, 256),
                                               (16, synth.FMT_CF32, 1, 20), (32, synth.FMT_CF32, 2, 100),
                                               (64, synth.FMT_CI8, 1, 300)])
def test_grid_matches_oracle(cuda, n, efmt, kernel, na):
    torch = _torch()
    wl = synth.config_small(n=n, efmt=efmt, kernel=kernel, n_ant=na, n_chan=3, n_samples=37)
    packed = synth.make_efield(wl)
    u = synth.random_gains(99, 3, na).astype(np.complex64)
    t0, nt = 5, 29
    with _lib().Plan([wl.array]) as plan:
        g = plan.grid(0, torch.from_numpy(packed).to(cuda), t0, nt, torch.from_numpy(u).to(cuda)).cpu().numpy()
    a = wl.array
    cells = O.grid_cells(a.ant_xy, a.dx, a.dy, a.x0, a.y0, n, n, kernel)
    E = O.unpack(packed[t0:t0 + nt], efmt)
    for f in range(3):
        ref = O.grid(E[:, f] * u[f].astype(np.complex128), cells, n, n)
        scale = np.abs(ref).max()
        assert np.abs(g[:, f] - ref).max() <= 2e-6 * scale


@pytest.mark.parametrize("n", [16, 32, 64])
def test_image_accumulate_and_tap(cuda, n):
    torch = _torch()
    wl = synth.config_small(n=n, n_chan=2, n_ant=min(40, 8 * n))
    rng = np.random.default_rng(17)
    nt = 23
    grid = ((rng.standard_normal((nt, 2, n, n)) + 1j * rng.standard_normal((nt, 2, n, n))) * 3).astype(np.complex64)
    img0 = rng.uniform(0, 1, size=(2, n, n)).astype(np.float32)
    with _lib().Plan([wl.array]) as plan:
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        img = torch.from_numpy(img0).to(cuda)
        tap = torch.zeros((nt, 2), dtype=torch.complex64, device=cuda)
        plan.image_accumulate(0, torch.from_numpy(grid).to(cuda), img, tap)
        img, tap = img.cpu().numpy(), tap.cpu().numpy()
    na = float(wl.array.n_ant)
    X = O.dft2(grid.astype(np.complex128), na)
    ref = img0 + (np.abs(X) ** 2).sum(0)
    assert image_err(img, ref).max() <= IMAGE_RTOL
    pb = O.Problem.from_workload(wl)
    for f in range(2):
        kx, ky = O.channel_setup(pb, f)["k0"]
        p = X[:, f, ky, kx]
        assert np.abs(tap[:, f] - p).max() <= 1e-5 * np.abs(X[:, f]).max()


def test_epical_update_matches_oracle(cuda):
    torch = _torch()
    wl = synth.config_small(n_chan=3, n_samples=90)
    a = wl.array
    packed = synth.make_efield(wl)
    rng = np.random.default_rng(5)
    tap = ((rng.standard_normal((90, 3)) + 1j * rng.standard_normal((90, 3))) * 2).astype(np.complex64)
    g0 = synth.random_gains(7, 3, a.n_ant)
    with _lib().Plan([a]) as plan:
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        e = torch.from_numpy(packed).to(cuda)
        kq = torch.zeros((3, a.n_ant, 4), dtype=torch.float64, device=cuda)
        g = torch.from_numpy(g0.copy()).to(cuda)
        tp = torch.from_numpy(tap).to(cuda)
        plan.epical_update(0, e, 0, 40, tp[:40], kq, g, finalize=False)   # accumulate in two calls
        plan.epical_update(0, e, 40, 50, tp[40:].clone(), kq, g, finalize=True)   # own allocation: 256-byte aligned
        got = g.cpu().numpy()
        assert float(kq.abs().max()) == 0.0
    pb = O.Problem.from_workload(wl)
    E = O.unpack(packed, a.efmt)
    for f in range(3):
        s = O.channel_setup(pb, f)
        K, Q = O.correlate(E[:, f], tap[:, f].astype(np.complex128))
        want, _ = O.gain_update(K / 90, Q / 90, s["A"], s["D"], g0[f], s["na"], wl.gamma)
        assert np.abs(got[f] - want).max() <= 1e-9 * np.abs(want).max()


# ---------------------------------------------------------------------------
# the fused loop
# ---------------------------------------------------------------------------

def test_run_tiny_full(cuda):
    """32 antennas, 32x32 nearest-cell grid, complex float input, a gain
    update after every sample for 400 samples."""
    wl = synth.config_tiny()
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


@pytest.mark.parametrize("n,efmt,kernel,na,n_samples,t_cal", [
    (32, synth.FMT_CI8, 2, 48, 230, 50),      # ragged last interval
    (64, synth.FMT_CI4, 2, 200, 301, 100),
    (16, synth.FMT_CF32, 2, 30, 64, 7),
    (64, synth.FMT_CI8, 1, 130, 40, 500),     # one interval shorter than t_cal
    (128, synth.FMT_CI8, 2, 150, 120, 50),    # residue-class engine, 2 x 2 classes
    (256, synth.FMT_CI4, 2, 300, 45, 20),     # residue-class engine, 4 x 4 classes
    (128, synth.FMT_CF32, 1, 40, 30, 30),
    (256, synth.FMT_CI8, 2, 700, 30, 15),     # dense-array variant (Na > 512, slot table in memory)
])
def test_run_small(cuda, n, efmt, kernel, na, n_samples, t_cal):
    wl = synth.config_small(n=n, efmt=efmt, kernel=kernel, n_ant=na, n_samples=n_samples, t_cal=t_cal)
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


@pytest.mark.parametrize("n,efmt,kernel,na,n_samples,t_cal", [
    (16, synth.FMT_CI8, 2, 128, 40, 20),     # 8 N antennas: the FFT engines' limit
    (64, synth.FMT_CI4, 1, 512, 30, 16),     # 8 N at 64 x 64 (the 2 x 2 kernel's schedule would not fit)
    (256, synth.FMT_CI8, 2, 2048, 12, 6),    # the residue-class engines' limit
])
def test_run_maximum_antennas(cuda, n, efmt, kernel, na, n_samples, t_cal):
    wl = synth.config_small(n=n, efmt=efmt, kernel=kernel, n_ant=na, n_chan=2, n_samples=n_samples, t_cal=t_cal)
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


@pytest.mark.parametrize("n,efmt,na,n_samples,t_cal", [
    (256, synth.FMT_CI8, 513, 37, 10),       # just past the class-pair engine
    (256, synth.FMT_CI4, 1500, 29, 8),
    (128, synth.FMT_CI8, 1000, 41, 20),      # two frames per step, odd sample count
    (128, synth.FMT_CI4, 700, 8, 3),
    (128, synth.FMT_CI8, 350, 23, 10),       # class-pair arrays, dense engine chosen
    (256, synth.FMT_CI4, 60, 19, 7),
])
@pytest.mark.parametrize("batch", [0, 4])
def test_dense_class_engine(cuda, n, efmt, na, n_samples, t_cal, batch):
    """The dense residue-class engine with two waves per SIMD (513..2048
    antennas at 256 x 256, up to 1024 at 128 x 128 by default; any integer
    array when chosen), gridding 2 or 4 schedule entries per batch from slot
    tables read from memory."""
    wl = synth.config_small(n=n, efmt=efmt, kernel=2, n_ant=na, n_chan=2, n_samples=n_samples, t_cal=t_cal)
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda, cls_engine=batch if na > 512 else (batch or 2))
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


def test_dense_64_grid_with_2x2_kernel_is_an_error(cuda):
    """512 antennas with the 2 x 2 kernel give a 64 x 64 gridding schedule
    longer than the LDS slot table: a clean EPIC_ERR_UNSUPPORTED."""
    lib = _lib()
    wl = synth.config_small(n=64, efmt=synth.FMT_CI4, kernel=2, n_ant=512, n_chan=2, n_samples=30, t_cal=16)
    with pytest.raises(lib.EpicError, match="slots per lane"):
        gpu_run(wl, synth.make_efield(wl), cuda)


@pytest.mark.parametrize("n,efmt,kernel,na,n_samples,t_cal,flagged", [
    (32, synth.FMT_CI4, 2, 64, 203, 1, ()),         # all 64 lanes own an antenna; four 64-row blocks, the last partial
    (16, synth.FMT_CI8, 1, 17, 130, 8, (0, 16)),    # flagged antennas at both ends
    (32, synth.FMT_CF32, 2, 40, 71, 3, (5,)),       # ragged last interval
])
def test_single_wave_solve(cuda, n, efmt, kernel, na, n_samples, t_cal, flagged):
    """Arrays of at most 64 antennas with intervals of at most 8 samples are
    solved by one wave per channel (DPP tap sums, no workgroup barriers)."""
    wl = synth.config_small(n=n, efmt=efmt, kernel=kernel, n_ant=na, n_chan=3, n_samples=n_samples, t_cal=t_cal)
    if flagged:
        flags = np.zeros(na, np.uint8)
        flags[list(flagged)] = 1
        wl = wl.replace(array=synth.dataclasses.replace(wl.array, ant_flag=flags))
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL
    if flagged:
        f = np.array(flagged)
        assert np.all(got["status"][:, f] & 1)
        np.testing.assert_array_equal(got["gains"][:, f], wl.g0[:, f])


def test_run_flagged_antennas(cuda):
    wl = synth.config_small(n_samples=150, t_cal=50)
    flags = np.zeros(wl.array.n_ant, np.uint8)
    flags[[0, 7, 33]] = 1
    wl = wl.replace(array=synth.dataclasses.replace(wl.array, ant_flag=flags))
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL
    assert np.all(got["status"][:, flags == 1] & 1)
    np.testing.assert_array_equal(got["gains"][:, flags == 1], wl.g0[:, flags == 1])


@pytest.mark.parametrize("layout", ["one_half", "edges"])
def test_paired_engine_half_frame_edges(cuda, layout):
    """The 64 x 64 two-waves-per-SIMD engine grids a frame in two halves of 32
    columns.  'one_half': every cell lies in columns 0..31, so the second
    half's schedule is empty.  'edges': 2 x 2 kernels that straddle columns
    31/32, or wrap around the last column and row (cell indices mod N)."""
    wl = synth.config_small(n=64, efmt=synth.FMT_CI4, n_ant=160, n_chan=2, n_samples=120, t_cal=40)
    a = wl.array
    rng = np.random.default_rng(5)
    if layout == "one_half":
        p = np.column_stack([rng.uniform(1.0, 30.0, 160), rng.uniform(1.0, 62.0, 160)])
    else:
        px = np.concatenate([rng.uniform(31.0, 32.0, 60), rng.uniform(63.0, 64.0, 50), rng.uniform(5.0, 58.0, 50)])
        py = np.concatenate([rng.uniform(3.0, 60.0, 60), rng.uniform(3.0, 60.0, 50), rng.uniform(63.0, 64.0, 50)])
        p = np.column_stack([px, py])
    xy = np.column_stack([a.x0 + p[:, 0] * a.dx, a.y0 + p[:, 1] * a.dy])
    wl = wl.replace(array=synth.dataclasses.replace(a, ant_xy=xy))
    cells = O.grid_cells(xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    ix = np.asarray(cells.ix)[np.asarray(cells.w) > 0]
    if layout == "one_half":
        assert ix.max() < 32
    else:
        assert {31, 32, 63, 0} <= set(ix.tolist())
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


def _half_schedule_length(cells, nx, half, fold=False):
    """Longest lane of a half-frame gridding schedule: the cells of the half
    (columns 32*half .. 32*half+31), largest first, each to the least-loaded of
    64 lanes, a cell costing one slot per antenna that touches it.  With fold,
    the residue-class engines' schedule: cells taken modulo 64 in x and y."""
    ix, iy, w = (np.asarray(v).ravel() for v in (cells.ix, cells.iy, cells.w))
    if fold:
        ix, iy, nx = ix % 64, iy % 64, 64
    keep = (w != 0) & (ix // 32 == half)
    flat = iy[keep] * nx + ix[keep]
    ids, counts = np.unique(flat, return_counts=True)
    load = np.zeros(64, np.int64)
    for k in np.argsort(-counts, kind="stable"):
        load[np.argmin(load)] += counts[k]
    return int(load.max())


@pytest.mark.parametrize("na,lo,hi", [(129, 9, 10), (176, 11, 12), (250, 13, 20), (140, 1, 8)])
def test_paired_engine_gridding_batch_lengths(cuda, na, lo, hi):
    """The 64 x 64 paired engine grids each half in batches sized to the
    half's schedule (8, 10 or 12 slots, batches of 8 beyond 12).  Antennas
    packed into columns 0..31 give first-half schedules in each range; the
    last case spreads them over both halves."""
    wl = synth.config_small(n=64, efmt=synth.FMT_CI8, n_ant=na, n_chan=2, n_samples=100, t_cal=50)
    a = wl.array
    rng = np.random.default_rng(na)
    xmax = 62.0 if hi <= 8 else 30.0
    p = np.column_stack([rng.uniform(1.0, xmax, na), rng.uniform(1.0, 62.0, na)])
    xy = np.column_stack([a.x0 + p[:, 0] * a.dx, a.y0 + p[:, 1] * a.dy])
    wl = wl.replace(array=synth.dataclasses.replace(a, ant_xy=xy))
    cells = O.grid_cells(xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    s0 = _half_schedule_length(cells, a.nx, 0)
    print(f"paired gridding: Na={na} first-half schedule {s0}", flush=True)
    assert lo <= s0 <= hi
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


@pytest.mark.parametrize("n,na,left,lo,hi", [(128, 60, False, 1, 4), (128, 200, False, 5, 8), (128, 340, False, 9, 12),
                                            (128, 250, True, 13, 20), (256, 340, False, 9, 12)])
def test_class_pair_engine_gridding_batch_lengths(cuda, n, na, left, lo, hi):
    """The residue-class engine with two waves per SIMD grids each half of a
    class in batches sized to the half's schedule (4, 8 or 12 slots, batches
    of 4 beyond 12).  'left' puts every antenna in folded columns 0..31."""
    wl = synth.config_small(n=n, efmt=synth.FMT_CI8, kernel=2, n_ant=na, n_chan=2, n_samples=60, t_cal=30)
    a = wl.array
    rng = np.random.default_rng(na + n)
    if left:
        px = rng.uniform(1.0, 30.0, na) + 64.0 * rng.integers(0, n // 64, na)
    else:
        px = rng.uniform(1.0, n - 2.0, na)
    p = np.column_stack([px, rng.uniform(1.0, n - 2.0, na)])
    xy = np.column_stack([a.x0 + p[:, 0] * a.dx, a.y0 + p[:, 1] * a.dy])
    wl = wl.replace(array=synth.dataclasses.replace(a, ant_xy=xy))
    cells = O.grid_cells(xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    s0, s1 = (_half_schedule_length(cells, a.nx, h, fold=True) for h in (0, 1))
    print(f"class-pair gridding: N={n} Na={na} half schedules {s0}, {s1}", flush=True)
    assert lo <= s0 <= hi and s0 + s1 <= 26
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL


@pytest.mark.parametrize("splits", [1, 3, 64])
def test_run_split_counts_agree(cuda, splits):
    """Any time split of the imaging launch gives the same answer."""
    wl = synth.config_small(n=64, efmt=synth.FMT_CI4, n_ant=256, n_chan=2, n_samples=200, t_cal=100)
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda, splits=splits)
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL


def test_run_lwa_full_size_sampled_channels(cuda):
    """The LWA-shaped workload at full size (256 antennas, 4+4-bit, 128
    channels, 64x64, 10,000 samples, update every 100) in the launch
    configuration the benchmark times; the oracle checks three channels."""
    wl = synth.config_lwa()
    packed = synth.make_efield(wl, threads=8)
    got = gpu_run(wl, packed, cuda)
    chans = [0, 77, 127]
    ref = oracle_run(wl, packed[:, chans], channels=chans)
    assert gain_err(got["hist"][:, chans], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"][chans], ref["image"]).max() <= IMAGE_RTOL
    assert np.all(np.isfinite(got["image"])) and np.all(got["status"] == 0)


@pytest.mark.parametrize("n,na", [(32, 48), (64, 180), (128, 48)])
def test_fixed_gain_image(cuda, n, na):
    torch = _torch()
    wl = synth.config_small(n=n, n_ant=na, n_chan=2, n_samples=77)
    a = wl.array
    packed = synth.make_efield(wl)
    g = synth.random_gains(3, 2, a.n_ant)
    with _lib().Plan([a]) as plan:
        img = plan.image(0, torch.from_numpy(packed).to(cuda), 77, torch.from_numpy(g).to(cuda)).cpu().numpy()
    cells = O.grid_cells(a.ant_xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    E = O.unpack(packed, a.efmt)
    u32 = (1 / g).astype(np.complex64).astype(np.complex128)
    for f in range(2):
        ref = O.image_fixed_gains(E[:, f], 1 / u32[f], cells, a.nx, a.ny, float(a.n_ant))
        assert image_err(img[f:f + 1], ref[None]).max() <= IMAGE_RTOL


def test_run_hera_full_size_sampled_channels(cuda):
    """The HERA-shaped workload at full size (350 antennas on a hexagonal
    lattice, 8+8-bit, 512 channels, 128 x 128, 2000 samples, update every
    100, off-centre calibrator); the oracle checks two channels."""
    wl = synth.config_hera()
    packed = synth.make_efield(wl, threads=16)
    got = gpu_run(wl, packed, cuda)
    chans = [3, 400]
    ref = oracle_run(wl, packed[:, chans], channels=chans)
    assert gain_err(got["hist"][:, chans], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"][chans], ref["image"]).max() <= IMAGE_RTOL
    assert np.all(np.isfinite(got["image"]))


def test_stagewise_equals_fused(cuda):
    """epic_grid + epic_image_accumulate + epical_update, interval by
    interval, reproduce epic_run."""
    torch = _torch()
    lib = _lib()
    wl = synth.config_small(n=32, n_chan=2, n_samples=120, t_cal=40)
    a = wl.array
    packed = synth.make_efield(wl)
    fused = gpu_run(wl, packed, cuda)
    with lib.Plan([a]) as plan:
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        e = torch.from_numpy(packed).to(cuda)
        g = torch.from_numpy(wl.g0.copy()).to(cuda)
        img = torch.zeros((2, a.ny, a.nx), dtype=torch.float32, device=cuda)
        kq = torch.zeros((2, a.n_ant, 4), dtype=torch.float64, device=cuda)
        for t0 in range(0, 120, 40):
            u = (1.0 / g).to(torch.complex64)
            grid = plan.grid(0, e, t0, 40, u)
            tap = torch.zeros((40, 2), dtype=torch.complex64, device=cuda)
            plan.image_accumulate(0, grid, img, tap)
            plan.epical_update(0, e, t0, 40, tap, kq, g, finalize=True)
        img = (img / 120).cpu().numpy()
        g = g.cpu().numpy()
    assert gain_err(g, fused["gains"]) <= GAIN_RTOL
    assert image_err(img, fused["image"]).max() <= IMAGE_RTOL


# ---------------------------------------------------------------------------
# edge cases and errors
# ---------------------------------------------------------------------------

def test_single_sample_and_errors(cuda):
    torch = _torch()
    lib = _lib()
    wl = synth.config_small(n_samples=1, t_cal=50)
    packed = synth.make_efield(wl)
    ref = oracle_run(wl, packed)
    got = gpu_run(wl, packed, cuda)
    assert gain_err(got["hist"], ref["gains"]) <= GAIN_RTOL
    assert image_err(got["image"], ref["image"]).max() <= IMAGE_RTOL
    a = wl.array
    with lib.Plan([a]) as plan:
        e = torch.from_numpy(packed).to(cuda)
        g = torch.from_numpy(wl.g0).to(cuda)
        img = torch.zeros((a.n_chan, a.ny, a.nx), dtype=torch.float32, device=cuda)
        with pytest.raises(lib.EpicError, match="EPIC_ERR_STATE"):
            plan.run([e], 1, [g], [img])                       # no model yet
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        with pytest.raises(lib.EpicError, match="EPIC_ERR_ARG"):
            plan.run([e], 0, [g], [img])                       # no samples
        with pytest.raises(lib.EpicError, match="gamma"):
            plan.set_model(0, wl.model_lmS, wl.cal_lm, 1.0, 10)


def test_unsupported_grid_is_an_error(cuda):
    lib = _lib()
    import torch
    wl = synth.config_small(n=32, n_ant=300)      # more than 8 antennas per lane
    with lib.Plan([wl.array]) as plan:
        with pytest.raises(lib.EpicError, match="UNSUPPORTED"):
            plan.grid(0, torch.from_numpy(synth.make_efield(wl)).to(cuda), 0, 1,
                      torch.ones((wl.array.n_chan, 300), dtype=torch.complex64, device=cuda))
    wl = synth.config_small(n=128, n_ant=40, n_samples=4)   # stage-wise calls stop at 64 x 64
    with lib.Plan([wl.array]) as plan:
        with pytest.raises(lib.EpicError, match="UNSUPPORTED"):
            plan.grid(0, torch.from_numpy(synth.make_efield(wl)).to(cuda), 0, 1,
                      torch.ones((wl.array.n_chan, 40), dtype=torch.complex64, device=cuda))
