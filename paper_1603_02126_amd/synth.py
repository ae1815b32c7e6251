"""Seeded synthetic inputs for the EPIC / EPICal hot path.

This module produces the *inputs* of the method and nothing else: antenna
layouts, channel frequencies, true complex gains, a sky of point sources, the
antenna E-field stream and its integer packing.  It holds none of the method's
arithmetic (no calibration, gridding, Fourier transform, squaring, correlation,
model denominator or gain update), so it can feed both the FP64 CPU oracle and
the HIP library without coupling them.

Signal model (Sec. 2.1, the antenna-measurement equation and eq. apply_gain):

    E_a(f, t) = g_a(f) * sum_s eps_s(f, t) * exp(-2 pi i f r_a . s_s / c) + n_a(f, t)

with an isotropic antenna pattern (W = 1), eps_s ~ CN(0, S_s) i.i.d. over
source, channel and time (the stochastic point sources of Sec. 3), and
receiver noise n ~ CN(0, sigma_r) with E|n|^2 = sigma_r (Sec. 4 defines the
noise level as the mean squared noise amplitude).

Random streams: numpy PCG64 seeded by a SeedSequence(seed); independent child
streams are spawned for layout, gains, sky, and then one per channel for the
source amplitudes and the receiver noise, so any subset of channels can be
regenerated on its own and gives the same bytes.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

C_LIGHT = 299792458.0

FMT_CF32 = 0
FMT_CI8 = 1
FMT_CI4 = 2
FMT_NAMES = {FMT_CF32: "cf32", FMT_CI8: "ci8", FMT_CI4: "ci4"}
FMT_BYTES = {FMT_CF32: 8, FMT_CI8: 2, FMT_CI4: 1}


@dataclass
class ArraySpec:
    """One antenna array and its aperture grid (positions and grid in metres)."""
    ant_xy: np.ndarray            # [Na, 2] float64, metres
    freq_hz: np.ndarray           # [F] float64
    nx: int
    ny: int
    dx: float
    dy: float
    x0: float                     # grid origin (position of cell 0), metres
    y0: float
    kernel: int                   # 1 = nearest cell, 2 = 2x2 bilinear
    efmt: int                     # FMT_*
    ant_flag: Optional[np.ndarray] = None   # [Na] uint8, 1 = flagged

    @property
    def n_ant(self) -> int:
        return int(self.ant_xy.shape[0])

    @property
    def n_chan(self) -> int:
        return int(self.freq_hz.shape[0])

    def flags(self) -> np.ndarray:
        if self.ant_flag is None:
            return np.zeros(self.n_ant, np.uint8)
        return np.asarray(self.ant_flag, np.uint8)


@dataclass
class Workload:
    """A complete seeded problem: array, sky, truth, calibration settings."""
    name: str
    seed: int
    array: ArraySpec
    src_lmS: np.ndarray           # [Ns, 3] true sky (l, m, flux)
    model_lmS: np.ndarray         # [Nm, 3] calibration sky model, flux in data units
    cal_lm: np.ndarray            # [2] calibrator direction
    g_true: np.ndarray            # [F, Na] complex128
    g0: np.ndarray                # [F, Na] complex128 initial gain estimate
    gamma: float
    t_cal: int
    n_samples: int
    sigma_r: float
    quant_scale: float            # data = round(E / quant_scale) for integer formats
    amp_model: str = "gaussian"   # gaussian | constmod | orthogonal
    noise: bool = True
    ortho_m: Optional[np.ndarray] = None   # [Ns] integer tones for amp_model=orthogonal

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# random streams
# --------------------------------------------------------------------------

_STREAM_LAYOUT, _STREAM_GAINS, _STREAM_SKY, _STREAM_CHAN = 0, 1, 2, 3


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(4)
    return kids


def _rng(child: np.random.SeedSequence) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(child))


def _chan_rngs(seed: int, n_chan: int):
    """Per-channel (amplitude, noise) generators."""
    chan_root = _streams(seed)[_STREAM_CHAN]
    per_chan = chan_root.spawn(n_chan)
    out = []
    for c in per_chan:
        a, n = c.spawn(2)
        out.append((_rng(a), _rng(n)))
    return out


# --------------------------------------------------------------------------
# layouts
# --------------------------------------------------------------------------

def layout_uniform_square(rng, n_ant, side):
    return rng.uniform(0.0, side, size=(n_ant, 2))


def layout_uniform_disk(rng, n_ant, radius, centre=(0.0, 0.0)):
    pts = []
    while len(pts) < n_ant:
        p = rng.uniform(-radius, radius, size=(4 * n_ant, 2))
        keep = p[(p ** 2).sum(1) <= radius * radius]
        pts.extend(keep.tolist())
    pts = np.array(pts[:n_ant], dtype=np.float64)
    return pts + np.asarray(centre, np.float64)


def layout_hex(n_ant, spacing):
    """The n_ant hexagonal-lattice points nearest the origin, ties broken by
    (radius, angle)."""
    r = int(np.ceil(np.sqrt(n_ant))) + 2
    pts = []
    for i in range(-r, r + 1):
        for j in range(-r, r + 1):
            x = spacing * (i + 0.5 * j)
            y = spacing * (np.sqrt(3.0) / 2.0) * j
            pts.append((x, y))
    pts = np.array(pts)
    rad = np.round(np.hypot(pts[:, 0], pts[:, 1]), 9)
    ang = np.round(np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2 * np.pi), 9)
    order = np.lexsort((ang, rad))
    return pts[order[:n_ant]].copy()


# --------------------------------------------------------------------------
# gains and sky
# --------------------------------------------------------------------------

def draw_gains(rng, n_chan, n_ant, amp_lo=0.8, amp_hi=1.2):
    amp = rng.uniform(amp_lo, amp_hi, size=(n_chan, n_ant))
    ph = rng.uniform(0.0, 2 * np.pi, size=(n_chan, n_ant))
    return amp * np.exp(1j * ph)


def bandpass_gains(rng, freq_hz, n_ant, amp_deg=0, phase_deg=0, turns=0.0, amp_lo=0.8, amp_hi=1.2):
    """Gains that vary smoothly over frequency: per antenna an amplitude
    a0 (1 + sum_k alpha_k x^k) and a phase phi0 + sum_k beta_k x^k, k >= 1,
    with x the frequency mapped linearly onto [-1, 1] over all channels.
    alpha_k ~ U[-0.1, 0.1]; beta_1 ~ U[-turns pi, turns pi] (a delay-like
    slope: the phase winds up to `turns` times across the channels); higher
    beta_k ~ U[-0.5, 0.5].  Degree 0 gives gains constant over the channels
    (the narrow-band assumption of Sec. 5).  [F, Na] complex128."""
    nu = np.asarray(freq_hz, np.float64)
    span = nu.max() - nu.min()
    x = (2.0 * (nu - nu.min()) / span - 1.0) if span > 0 else np.zeros_like(nu)
    a0 = rng.uniform(amp_lo, amp_hi, size=n_ant)
    ph0 = rng.uniform(0.0, 2 * np.pi, size=n_ant)
    amp = np.ones((nu.size, n_ant))
    ph = np.zeros((nu.size, n_ant))
    for k in range(1, amp_deg + 1):
        amp += rng.uniform(-0.1, 0.1, size=n_ant)[None, :] * x[:, None] ** k
    for k in range(1, phase_deg + 1):
        lim = turns * np.pi if k == 1 else 0.5
        ph += rng.uniform(-lim, lim, size=n_ant)[None, :] * x[:, None] ** k
    return a0[None, :] * amp * np.exp(1j * (ph0[None, :] + ph))


def powerlaw_flux(rng, n, s_min, s_max):
    """dN/dS proportional to S^-2 on [s_min, s_max] (inverse CDF)."""
    u = rng.uniform(0.0, 1.0, size=n)
    return 1.0 / (1.0 / s_min - u * (1.0 / s_min - 1.0 / s_max))


def random_disk_lm(rng, n, rmax):
    out = []
    while len(out) < n:
        p = rng.uniform(-rmax, rmax, size=(4 * n, 2))
        keep = p[(p ** 2).sum(1) < rmax * rmax]
        out.extend(keep.tolist())
    return np.array(out[:n])


# --------------------------------------------------------------------------
# E-field stream
# --------------------------------------------------------------------------

def geometric_phase(ant_xy, freq, lm):
    """exp(-2 pi i f r_a . s / c) for a coplanar array: [Na, Ns]."""
    arg = (ant_xy[:, 0:1] * lm[None, :, 0] + ant_xy[:, 1:2] * lm[None, :, 1]) * (freq / C_LIGHT)
    return np.exp(-2j * np.pi * arg)


def _amplitudes(wl: Workload, rng, n_t, t0, dtype):
    S = wl.src_lmS[:, 2]
    ns = S.shape[0]
    if wl.amp_model == "gaussian":
        re = rng.standard_normal((n_t, ns), dtype=np.float64 if dtype == np.complex128 else np.float32)
        im = rng.standard_normal((n_t, ns), dtype=re.dtype)
        return ((re + 1j * im) * np.sqrt(S / 2.0)[None, :]).astype(dtype)
    if wl.amp_model == "constmod":
        th = rng.uniform(0.0, 2 * np.pi, size=(n_t, ns))
        return (np.sqrt(S)[None, :] * np.exp(1j * th)).astype(dtype)
    if wl.amp_model == "orthogonal":
        t = np.arange(t0, t0 + n_t, dtype=np.float64)[:, None]
        m = np.asarray(wl.ortho_m, np.float64)[None, :]
        return (np.sqrt(S)[None, :] * np.exp(2j * np.pi * m * t / wl.t_cal)).astype(dtype)
    raise ValueError(wl.amp_model)


def efield_channel(wl: Workload, ch: int, dtype=np.complex128):
    """Complex E-field of one channel, [T, Na] (before quantisation)."""
    arr = wl.array
    rng_a, rng_n = _chan_rngs(wl.seed, arr.n_chan)[ch]
    T = wl.n_samples
    phase = geometric_phase(arr.ant_xy, arr.freq_hz[ch], wl.src_lmS[:, :2]).astype(dtype)
    eps = _amplitudes(wl, rng_a, T, 0, dtype)
    E = eps @ phase.T                                  # [T, Na]
    E *= wl.g_true[ch][None, :].astype(dtype)
    if wl.noise and wl.sigma_r > 0:
        rdt = np.float64 if dtype == np.complex128 else np.float32
        nre = rng_n.standard_normal((T, arr.n_ant), dtype=rdt)
        nim = rng_n.standard_normal((T, arr.n_ant), dtype=rdt)
        E += (nre + 1j * nim) * np.sqrt(wl.sigma_r / 2.0)
    return E


def loss_target_sky(wl: Workload, n_src: int = 50):
    """The loss target's sky of the differentiable workload: the n_src
    brightest sources of the calibration model (data units) and the receiver
    noise power in data units, sigma_r / quant_scale^2."""
    order = np.argsort(-wl.model_lmS[:, 2], kind="stable")[:n_src]
    return wl.model_lmS[order].copy(), wl.sigma_r / (wl.quant_scale * wl.quant_scale)


def tone_efield(ant_xy, freq_hz, src_lmS, sigma: float) -> np.ndarray:
    """A noiseless stand-in for a sky with receiver noise, as a float32
    stream [T, F, Na, 2] with T = n_src + Na: source s radiates
    sqrt(S_s) exp(2 pi i s t / T) and antenna a adds its own tone
    sqrt(sigma) exp(2 pi i (n_src + a) t / T), with unit gains:

        E_a(f, t) = sum_s sqrt(S_s) e^{2 pi i s t / T} exp(-2 pi i f r_a . s_s / c)
                    + sqrt(sigma) e^{2 pi i (n_src + a) t / T}.

    All T tones are distinct over the T samples, so every product of two
    different tones averages to zero over the stream: time averages of
    second moments equal those of the stochastic sky of the signal model."""
    ant_xy = np.asarray(ant_xy, np.float64)
    src = np.asarray(src_lmS, np.float64)
    ns, na = src.shape[0], ant_xy.shape[0]
    T = ns + na
    t = np.arange(T, dtype=np.float64)[:, None]
    amp_s = np.sqrt(src[:, 2])[None, :] * np.exp(2j * np.pi * np.arange(ns)[None, :] * t / T)     # [T, Ns]
    amp_n = np.sqrt(sigma) * np.exp(2j * np.pi * (ns + np.arange(na))[None, :] * t / T)           # [T, Na]
    out = np.empty((T, len(freq_hz), na, 2), np.float32)
    for c, f in enumerate(np.asarray(freq_hz, np.float64)):
        E = amp_s @ geometric_phase(ant_xy, f, src[:, :2]).T + amp_n
        out[:, c, :, 0] = E.real
        out[:, c, :, 1] = E.imag
    return out


def quantise(x: np.ndarray, scale: float, lo: int, hi: int) -> np.ndarray:
    """Round half up then clip: the digitiser's integer code for x / scale."""
    return np.clip(np.floor(x / scale + 0.5), lo, hi).astype(np.int8)


def pack_ci4(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """4+4-bit two's complement: real part in the high nibble."""
    return (((re.astype(np.int16) & 0xF) << 4) | (im.astype(np.int16) & 0xF)).astype(np.uint8)


def pack_channel(wl: Workload, E: np.ndarray) -> np.ndarray:
    """Pack one channel [T, Na] into the array's format.

    Returns uint8 [T, Na] (ci4), int8 [T, Na, 2] (ci8) or float32 [T, Na, 2] (cf32).
    """
    fmt = wl.array.efmt
    if fmt == FMT_CF32:
        out = np.empty(E.shape + (2,), np.float32)
        out[..., 0] = E.real
        out[..., 1] = E.imag
        return out
    if fmt == FMT_CI8:
        out = np.empty(E.shape + (2,), np.int8)
        out[..., 0] = quantise(E.real, wl.quant_scale, -128, 127)
        out[..., 1] = quantise(E.imag, wl.quant_scale, -128, 127)
        return out
    if fmt == FMT_CI4:
        return pack_ci4(quantise(E.real, wl.quant_scale, -8, 7), quantise(E.imag, wl.quant_scale, -8, 7))
    raise ValueError(fmt)


def packed_shape(wl: Workload, n_t: Optional[int] = None, n_chan: Optional[int] = None):
    T = wl.n_samples if n_t is None else n_t
    F = wl.array.n_chan if n_chan is None else n_chan
    Na = wl.array.n_ant
    fmt = wl.array.efmt
    if fmt == FMT_CI4:
        return (T, F, Na), np.uint8
    if fmt == FMT_CI8:
        return (T, F, Na, 2), np.int8
    return (T, F, Na, 2), np.float32


def make_efield(wl: Workload, channels: Optional[Sequence[int]] = None, dtype=None, threads: int = 0):
    """Packed E-field stream [T, F_sel, Na(, 2)] for the selected channels.

    Channels are generated independently (own random streams), optionally in
    a thread pool; the bytes do not depend on the thread count.
    """
    arr = wl.array
    chans = list(range(arr.n_chan)) if channels is None else list(channels)
    if dtype is None:
        dtype = np.complex128 if arr.efmt == FMT_CF32 else np.complex64
    shape, pdt = packed_shape(wl, n_chan=len(chans))
    out = np.empty(shape, pdt)

    def work(i_c):
        i, c = i_c
        out[:, i] = pack_channel(wl, efield_channel(wl, c, dtype))

    items = list(enumerate(chans))
    if threads and threads > 1 and len(items) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, items))
    else:
        for it in items:
            work(it)
    return out


# --------------------------------------------------------------------------
# the configurations
# --------------------------------------------------------------------------

def _grid_for_disk(radius, n, dx, offset_cells=0.0):
    """Grid origin such that a disk of `radius` centred at 0 sits in the middle."""
    x0 = -0.5 * n * dx + offset_cells * dx
    return x0


def config_tiny(seed: int = 1, **over) -> Workload:
    """32 antennas in a 16-wavelength square, 1 channel, 32x32 grid, nearest
    cell, 400 samples, calibrator (100) at the phase centre plus 10 sources
    (U[1,5]) on random physical pixels, sigma_r = 1, gains updated every
    sample with gamma = 0.5.  Positions in wavelengths: the single channel is
    at f = c, so one metre is one wavelength."""
    s_lay, s_g, s_sky, _ = (_rng(k) for k in _streams(seed))
    Na, N = 32, 32
    ant = layout_uniform_square(s_lay, Na, 16.0)
    freq = np.array([C_LIGHT])
    arr = ArraySpec(ant_xy=ant, freq_hz=freq, nx=N, ny=N, dx=0.5, dy=0.5, x0=0.0, y0=0.0,
                    kernel=1, efmt=FMT_CF32)
    # random physical pixels (l, m) = kappa / 16, excluding the phase centre
    pix = set()
    srcs = []
    while len(srcs) < 10:
        k = s_sky.integers(-16, 16, size=2)
        l, m = k[0] / 16.0, k[1] / 16.0
        if (k[0], k[1]) == (0, 0) or l * l + m * m >= 1.0 or (k[0], k[1]) in pix:
            continue
        pix.add((k[0], k[1]))
        srcs.append((l, m, s_sky.uniform(1.0, 5.0)))
    src = np.array([(0.0, 0.0, 100.0)] + srcs)
    g = draw_gains(s_g, 1, Na)
    wl = Workload(name="tiny", seed=seed, array=arr, src_lmS=src, model_lmS=src.copy(),
                  cal_lm=np.array([0.0, 0.0]), g_true=g, g0=np.ones((1, Na), np.complex128),
                  gamma=0.5, t_cal=1, n_samples=400, sigma_r=1.0, quant_scale=1.0)
    return wl.replace(**over) if over else wl


def _quant_scale(src_S, sigma_r, g, rms_levels):
    """Scale giving `rms_levels` of per-component rms for the mean power."""
    p = float(np.mean(np.abs(g) ** 2)) * float(np.sum(src_S)) + sigma_r
    return np.sqrt(p / 2.0) / rms_levels


def config_lwa(seed: int = 2, n_chan: int = 128, n_samples: int = 10000, **over) -> Workload:
    """LWA-station shape: 256 antennas uniform in a 50 m radius disk, 4+4-bit
    E-fields, channels across 30-80 MHz, 64x64 grid of 1.875 m cells with the
    2x2 kernel, a zenith calibrator plus 100 power-law sources, receiver
    noise dominated, gains updated every 100 samples (gamma = 0.5)."""
    s_lay, s_g, s_sky, _ = (_rng(k) for k in _streams(seed))
    Na, N, dx = 256, 64, 1.875
    ant = layout_uniform_disk(s_lay, Na, 50.0)
    F_full = 128
    freq_full = (30.0 + (np.arange(F_full) + 0.5) * 50.0 / F_full) * 1e6
    freq = freq_full[:n_chan] if n_chan <= F_full else \
        (30.0 + (np.arange(n_chan) + 0.5) * 50.0 / n_chan) * 1e6
    x0 = _grid_for_disk(50.0, N, dx)
    arr = ArraySpec(ant_xy=ant, freq_hz=freq, nx=N, ny=N, dx=dx, dy=dx, x0=x0, y0=x0,
                    kernel=2, efmt=FMT_CI4)
    lm = random_disk_lm(s_sky, 100, 0.95)
    S = powerlaw_flux(s_sky, 100, 1.0, 100.0)
    src = np.concatenate([np.array([[0.0, 0.0, 1000.0]]), np.column_stack([lm, S])])
    g = draw_gains(s_g, F_full if n_chan <= F_full else n_chan, Na)[:n_chan]
    sigma_r = 1000.0
    qs = _quant_scale(src[:, 2], sigma_r, g, 2.0)
    model = src.copy()
    model[:, 2] /= qs * qs
    wl = Workload(name="lwa", seed=seed, array=arr, src_lmS=src, model_lmS=model,
                  cal_lm=np.array([0.0, 0.0]), g_true=g, g0=np.ones((n_chan, Na), np.complex128),
                  gamma=0.5, t_cal=100, n_samples=n_samples, sigma_r=sigma_r, quant_scale=qs)
    return wl.replace(**over) if over else wl


def config_lwa_band(seed: int = 2, n_chan: int = 128, n_samples: int = 10000, **over) -> Workload:
    """The lwa shape with the choices of the LWA demonstration of Sec. 5:
    gains constant over the band (one complex gain per antenna), initial
    gains 0.25, gamma = 0.7.  Calibrated with every channel sharing the band's
    mean solution."""
    base = config_lwa(seed, n_chan, n_samples)
    s_g = _rng(_streams(seed + 1000)[1])
    g = bandpass_gains(s_g, base.array.freq_hz, base.array.n_ant)
    qs = _quant_scale(base.src_lmS[:, 2], base.sigma_r, g, 2.0)
    model = base.src_lmS.copy()
    model[:, 2] /= qs * qs
    wl = base.replace(name="lwa_band", g_true=g, quant_scale=qs, model_lmS=model,
                      g0=np.full((n_chan, base.array.n_ant), 0.25, np.complex128), gamma=0.7)
    return wl.replace(**over) if over else wl


def config_noise(seed: int = 9, sigma_r: float = 10.0, t_cal: int = 100, n_iter: int = 10, n_chan: int = 64,
                 model: str = "full", **over) -> Workload:
    """The noise-trend study of Sec. 4: 51 antennas uniform in a 48 m square
    (a stand-in for the inner MWA layout of Sec. 3), n_chan channels over
    140-160 MHz with fluxes constant over frequency, complex float samples in
    Jy.  Sky: a 5 Jy calibrator at the phase centre and 49 sources of
    0.2-0.5 Jy uniform within 0.5 of it (about 22 Jy in total; the
    calibrator carries about 22%).  True gains 1 and g(0) = 1, gamma = 0.35,
    receiver noise sigma_r, n_iter updates of t_cal samples.  model "full"
    puts every source in the calibration model, "single" the calibrator only.
    64 x 64 grid of 1 m cells, 2x2 kernel."""
    s_lay, _, s_sky, _ = (_rng(k) for k in _streams(seed))
    Na, N, dx = 51, 64, 1.0
    ant = s_lay.uniform(-24.0, 24.0, size=(Na, 2))
    freq = (140.0 + 20.0 * (np.arange(n_chan) + 0.5) / n_chan) * 1e6
    x0 = _grid_for_disk(24.0 * np.sqrt(2.0), N, dx)
    arr = ArraySpec(ant_xy=ant, freq_hz=freq, nx=N, ny=N, dx=dx, dy=dx, x0=x0, y0=x0, kernel=2, efmt=FMT_CF32)
    lm = random_disk_lm(s_sky, 49, 0.5)
    S = s_sky.uniform(0.2, 0.5, size=49)
    src = np.concatenate([np.array([[0.0, 0.0, 5.0]]), np.column_stack([lm, S])])
    mdl = src.copy() if model == "full" else src[:1].copy()
    g = np.ones((n_chan, Na), np.complex128)
    wl = Workload(name=f"noise_{model}", seed=seed, array=arr, src_lmS=src, model_lmS=mdl,
                  cal_lm=np.array([0.0, 0.0]), g_true=g, g0=g.copy(), gamma=0.35, t_cal=t_cal,
                  n_samples=t_cal * n_iter, sigma_r=sigma_r, quant_scale=1.0)
    return wl.replace(**over) if over else wl


def config_hera(seed: int = 3, n_chan: int = 512, n_samples: int = 2000, **over) -> Workload:
    """HERA shape: 350 antennas on a 14 m hexagonal lattice, 8+8-bit E-fields,
    channels across 100-200 MHz, 128x128 grid of 2.5 m cells (origin offset a
    quarter cell), 2x2 kernel, calibrator carrying 10% of the sky power plus
    100 power-law sources (fluxes 1..10, over the visible sky, all fainter
    than the calibrator), receiver noise equal to the sky power, gains every
    100 samples."""
    s_lay, s_g, s_sky, _ = (_rng(k) for k in _streams(seed))
    Na, N, dx = 350, 128, 2.5
    ant = layout_hex(Na, 14.0)
    F_full = 512
    freq = (100.0 + (np.arange(F_full) + 0.5) * 100.0 / F_full)[:n_chan] * 1e6
    x0 = _grid_for_disk(140.0, N, dx, 0.25)
    arr = ArraySpec(ant_xy=ant, freq_hz=freq, nx=N, ny=N, dx=dx, dy=dx, x0=x0, y0=x0,
                    kernel=2, efmt=FMT_CI8)
    lm = random_disk_lm(s_sky, 100, 0.9)
    S = powerlaw_flux(s_sky, 100, 1.0, 10.0)
    cal = 0.1 / 0.9 * S.sum()
    cal_lm = random_disk_lm(s_sky, 1, 0.1)[0]
    src = np.concatenate([np.array([[cal_lm[0], cal_lm[1], cal]]), np.column_stack([lm, S])])
    g = draw_gains(s_g, F_full, Na)[:n_chan]
    sigma_r = float(src[:, 2].sum())
    qs = _quant_scale(src[:, 2], sigma_r, g, 32.0)
    model = src.copy()
    model[:, 2] /= qs * qs
    wl = Workload(name="hera", seed=seed, array=arr, src_lmS=src, model_lmS=model,
                  cal_lm=cal_lm.copy(), g_true=g, g0=np.ones((n_chan, Na), np.complex128),
                  gamma=0.5, t_cal=100, n_samples=n_samples, sigma_r=sigma_r, quant_scale=qs)
    return wl.replace(**over) if over else wl


def config_diff(seed: int = 4, n_chan: int = 64, n_samples: int = 1000, **over) -> Workload:
    """Differentiable-imaging case: the LWA-shaped layout with 8+8-bit data,
    64 channels, 1000 samples; gains perturbed 5% from the truth."""
    base = config_lwa(seed=seed, n_chan=n_chan, n_samples=n_samples)
    s_g = _rng(_streams(seed + 1000)[_STREAM_GAINS])
    arr = dataclasses.replace(base.array, efmt=FMT_CI8)
    qs = _quant_scale(base.src_lmS[:, 2], base.sigma_r, base.g_true, 32.0)
    model = base.src_lmS.copy()
    model[:, 2] /= qs * qs
    pert = 0.05 * (s_g.standard_normal(base.g_true.shape) + 1j * s_g.standard_normal(base.g_true.shape)) / np.sqrt(2)
    wl = base.replace(name="diff", array=arr, quant_scale=qs, model_lmS=model,
                      g0=base.g_true * (1.0 + pert))
    return wl.replace(**over) if over else wl


def config_small(seed: int = 11, n_ant: int = 48, n: int = 32, n_chan: int = 3, n_samples: int = 250,
                 efmt: int = FMT_CI8, kernel: int = 2, t_cal: int = 50, **over) -> Workload:
    """A small multi-channel case for parity tests: several tiles of antennas
    per lane group, a ragged last interval, off-centre calibrator."""
    s_lay, s_g, s_sky, _ = (_rng(k) for k in _streams(seed))
    dx = 1.5
    radius = 0.4 * n * dx
    ant = layout_uniform_disk(s_lay, n_ant, radius)
    freq = (40.0 + 20.0 * np.arange(n_chan) / max(1, n_chan)) * 1e6
    x0 = _grid_for_disk(radius, n, dx, 0.3)
    arr = ArraySpec(ant_xy=ant, freq_hz=freq, nx=n, ny=n, dx=dx, dy=dx, x0=x0, y0=x0,
                    kernel=kernel, efmt=efmt)
    lm = random_disk_lm(s_sky, 12, 0.9)
    S = powerlaw_flux(s_sky, 12, 1.0, 20.0)
    cal_lm = np.array([0.21, -0.13])
    src = np.concatenate([np.array([[cal_lm[0], cal_lm[1], 200.0]]), np.column_stack([lm, S])])
    g = draw_gains(s_g, n_chan, n_ant)
    sigma_r = 50.0
    qs = _quant_scale(src[:, 2], sigma_r, g, 24.0 if efmt == FMT_CI8 else 2.0) if efmt != FMT_CF32 else 1.0
    model = src.copy()
    model[:, 2] /= qs * qs
    wl = Workload(name="small", seed=seed, array=arr, src_lmS=src, model_lmS=model,
                  cal_lm=cal_lm, g_true=g, g0=np.ones((n_chan, n_ant), np.complex128),
                  gamma=0.5, t_cal=t_cal, n_samples=n_samples, sigma_r=sigma_r, quant_scale=qs)
    return wl.replace(**over) if over else wl


CONFIGS = {
    "tiny": config_tiny,
    "lwa": config_lwa,
    "lwa_band": config_lwa_band,
    "hera": config_hera,
    "diff": config_diff,
    "small": config_small,
}


def unit_gains(n_chan, n_ant):
    return np.ones((n_chan, n_ant), np.complex128)


def random_gains(seed, n_chan, n_ant, amp_lo=0.8, amp_hi=1.2):
    """Seeded gain estimates for stage-wise tests (not drawn from any workload)."""
    return draw_gains(_rng(np.random.SeedSequence(seed)), n_chan, n_ant, amp_lo, amp_hi)


def config_uneven(seed: int = 5, n_chan: int = 256, n_samples: int = 500,
                  n_ants=(64, 128, 256, 512, 1024, 1024, 2048, 2048),
                  grids=(32, 64, 64, 128, 128, 256, 256, 256)):
    """Several arrays of uneven size observed together: antennas uniform in a
    disk of diameter 0.8 N dx on an N x N grid (dx = half a wavelength at the
    top of the band), 8+8-bit E-fields, channels across 50-100 MHz, three
    calibrators (100, 50, 25) plus 50 power-law sources per array, gains every
    100 samples.  Returns one Workload per array; the brightest calibrator is
    the tapped pixel and all three are in the model."""
    out = []
    for i, (na, n) in enumerate(zip(n_ants, grids)):
        s_lay, s_g, s_sky, _ = (_rng(k) for k in _streams(seed * 1000 + i))
        dx = 1.5
        radius = 0.4 * n * dx
        ant = layout_uniform_disk(s_lay, na, radius)
        freq = (50.0 + (np.arange(n_chan) + 0.5) * 50.0 / n_chan) * 1e6
        x0 = _grid_for_disk(radius, n, dx, 0.25)
        arr = ArraySpec(ant_xy=ant, freq_hz=freq, nx=n, ny=n, dx=dx, dy=dx, x0=x0, y0=x0,
                        kernel=2, efmt=FMT_CI8)
        cal = random_disk_lm(s_sky, 3, 0.3)
        lm = random_disk_lm(s_sky, 50, 0.5)
        S = powerlaw_flux(s_sky, 50, 1.0, 10.0)
        src = np.concatenate([np.column_stack([cal, [100.0, 50.0, 25.0]]), np.column_stack([lm, S])])
        g = draw_gains(s_g, n_chan, na)
        sigma_r = float(src[:, 2].sum())
        qs = _quant_scale(src[:, 2], sigma_r, g, 32.0)
        model = src.copy()
        model[:, 2] /= qs * qs
        out.append(Workload(name=f"uneven{i}", seed=seed * 1000 + i, array=arr, src_lmS=src, model_lmS=model,
                            cal_lm=cal[0].copy(), g_true=g, g0=np.ones((n_chan, na), np.complex128),
                            gamma=0.5, t_cal=100, n_samples=n_samples, sigma_r=sigma_r, quant_scale=qs))
    return out
