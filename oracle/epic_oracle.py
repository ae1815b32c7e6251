"""FP64 CPU oracle for the EPIC direct-imaging loop with EPICal calibration.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
statement of what the hot path computes, written from Beardsley et al. (2016),
"An Efficient Feedback Calibration Algorithm for Direct Imaging Radio
Telescopes" (arXiv:1603.02126).  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import it; the library never does, and the
two share no code.  Everything is float64 / complex128.

Notation follows the paper: E_a(t) antenna E-field (uncalibrated), g_a gain
estimate, E'_a = E_a / g_a (calibrated), W_a gridding kernel, E'_j gridded
aperture field, script-E'(s_k, t) the instantaneous electric-field image,
I'(s_k) the time-averaged squared image, K / C the antenna-pixel correlation
and its autocorrelation-subtracted form, V^M model visibilities, gamma the
damping factor.

Readings of places where the paper is silent or loose (each one is also
listed with its reason in the design notes of the repository):

* The 2D transform uses the +2 pi i sign and the 1/Na factor of the MOFF
  summary equation (Sec. 2.1), no 1/Ng, natural (unshifted) pixel order.
* Grid cell j sits at r_j = (x0 + jx dx, y0 + jy dy); cell indices wrap
  modulo the grid size (the discrete transform is periodic).  A grid origin
  only multiplies every pixel by a common phase, which cancels in C / D and in
  |.|^2.
* Kernels: nearest cell (jx = floor(p + 0.5), p = (x - x0) / dx) or the 2x2
  bilinear kernel = area overlap of a one-cell tophat (i0 = floor(p),
  phi = p - i0, weights (1 - phi), phi per axis).
* The calibrator pixel k0 is the pixel nearest the calibrator direction:
  kappa = floor(l f Nx dx / c + 0.5) modulo Nx (likewise for m).
* The direction-dependent factor W*_b(s0) exp(-2 pi i f s0 . r_b / c) that
  multiplies the model in eq. (Cna) and eq. (cal_solution) is taken as the
  exact response of the *gridded* antenna at the tapped pixel,
  conj(A_b(k0)) with A_b(k) = sum_j W_b(r_j - r_b) exp(+2 pi i j . k / N):
  this is what the tapped pixel of the gridded transform really contains, it
  equals the paper's factor at the phase centre, and with it exact gains are
  an exact fixed point (the eq. (epix) approximation breaks that off-centre).
* <.> over a calibration interval is a mean (divide by the number of
  samples in the interval); a short last interval is averaged over its own
  length.
* Na is the number of unflagged antennas.  Flagged antennas are neither
  gridded nor correlated nor updated, and are left out of the model sum.
* An antenna whose model denominator is (numerically) zero, or whose update is
  not finite, keeps its previous gain.
* The gain recursion follows eq. (damping) exactly, so the single-source
  limit of Sec. 2.2 comes out as (Na - 1) S_src in the denominator (the sum
  excludes b = a), not Na S_src.
* Several tapped pixels (Sec. 6): the gain is the least-squares solution over
  the pixels of Na C_ap = g_a D_ap, damped (gain_update_multi).
* The visibility-based comparison calibrator of Sec. 4 minimises eq.
  (vis_cal) by alternating least squares (StEFCal); sigma_g of eq.
  (gain_error) is taken after removing each channel's unobservable global
  phase.
* Gains shared over a band of channels (Sec. 5 averaging, Sec. 6 gain-model
  fitting): the undamped per-channel solutions Na C/D of the band's channels
  are averaged, or fitted by polynomials in amplitude and unwrapped phase over
  a frequency coordinate mapped onto [-1, 1]; every channel of the band is
  then damped towards the model (run_band).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

C_LIGHT = 299792458.0

FMT_CF32, FMT_CI8, FMT_CI4 = 0, 1, 2


# --------------------------------------------------------------------------
# Input decoding (the digitised E-field stream, Sec. 2.1 "F-engine")
# --------------------------------------------------------------------------

def nibble_to_int(v: np.ndarray) -> np.ndarray:
    """A 4-bit two's complement code (0..15) as a signed integer in [-8, 7]."""
    v = np.asarray(v).astype(np.int64) & 0xF
    return np.where(v >= 8, v - 16, v)


def unpack(packed: np.ndarray, fmt: int) -> np.ndarray:
    """Packed E-field samples -> complex128.

    ci4: one byte per sample, real part in the high nibble, imaginary part in
    the low nibble, each 4-bit two's complement.  ci8: int8 (re, im) pairs.
    cf32: float32 (re, im) pairs.
    """
    if fmt == FMT_CI4:
        b = np.asarray(packed).astype(np.int64)
        return nibble_to_int(b >> 4).astype(np.float64) + 1j * nibble_to_int(b).astype(np.float64)
    if fmt == FMT_CI8 or fmt == FMT_CF32:
        p = np.asarray(packed)
        return p[..., 0].astype(np.float64) + 1j * p[..., 1].astype(np.float64)
    raise ValueError(f"unknown format {fmt}")


# --------------------------------------------------------------------------
# Plan: gridding kernel, pixel directions, model (Sec. 2.1 eq. gridding,
# Sec. 2.2 eq. cal_solution)
# --------------------------------------------------------------------------

@dataclass
class GridCells:
    ix: np.ndarray   # [Na, K2] int64, column index (mod nx)
    iy: np.ndarray   # [Na, K2] int64, row index (mod ny)
    w: np.ndarray    # [Na, K2] float64 kernel weight


def grid_cells(ant_xy, dx, dy, x0, y0, nx, ny, kernel) -> GridCells:
    """Grid cells touched by each antenna and the kernel weights W_a(r_j - r_a)
    (eq. gridding).  kernel 1: nearest cell; kernel 2: 2x2 bilinear."""
    ant_xy = np.asarray(ant_xy, np.float64)
    px = (ant_xy[:, 0] - x0) / dx
    py = (ant_xy[:, 1] - y0) / dy
    if kernel == 1:
        ix = np.floor(px + 0.5).astype(np.int64)[:, None]
        iy = np.floor(py + 0.5).astype(np.int64)[:, None]
        w = np.ones_like(ix, dtype=np.float64)
    elif kernel == 2:
        fx, fy = np.floor(px), np.floor(py)
        ax, ay = px - fx, py - fy
        i0, j0 = fx.astype(np.int64), fy.astype(np.int64)
        # cell order: (i0, j0), (i0+1, j0), (i0, j0+1), (i0+1, j0+1)
        ix = np.stack([i0, i0 + 1, i0, i0 + 1], axis=1)
        iy = np.stack([j0, j0, j0 + 1, j0 + 1], axis=1)
        w = np.stack([(1 - ax) * (1 - ay), ax * (1 - ay), (1 - ax) * ay, ax * ay], axis=1)
    else:
        raise ValueError("kernel must be 1 or 2")
    return GridCells(ix=np.mod(ix, nx), iy=np.mod(iy, ny), w=w)


def pixel_of_direction(l, m, freq, nx, ny, dx, dy):
    """Pixel nearest the direction (l, m) at frequency freq.

    The transform dual of r f / c is (l, m) (Sec. 2.1): pixel kappa of an
    N-cell grid with spacing d sits at l = kappa c / (f N d).  Ties round half
    up on the signed index; the result is taken modulo N (natural order)."""
    kx = math.floor(l * freq * nx * dx / C_LIGHT + 0.5)
    ky = math.floor(m * freq * ny * dy / C_LIGHT + 0.5)
    return int(kx % nx), int(ky % ny)


def direction_of_pixel(kx, ky, freq, nx, ny, dx, dy):
    """(l, m) of pixel (kx, ky), using the signed index in [-N/2, N/2)."""
    sx = kx - nx if kx >= nx // 2 else kx
    sy = ky - ny if ky >= ny // 2 else ky
    return sx * C_LIGHT / (freq * nx * dx), sy * C_LIGHT / (freq * ny * dy)


def pixel_response(cells: GridCells, kx, ky, nx, ny) -> np.ndarray:
    """A_a(k) = sum_j W_a(r_j - r_a) exp(+2 pi i (jx kx / Nx + jy ky / Ny)):
    the contribution of antenna a's gridded field to pixel k of the
    (un-normalised) transform."""
    ph = 2.0 * np.pi * (np.mod(cells.ix * kx, nx) / nx + np.mod(cells.iy * ky, ny) / ny)
    return (cells.w * np.exp(1j * ph)).sum(axis=1)


def model_visibilities(ant_xy, freq, model_lmS) -> np.ndarray:
    """V^M_ab = sum_s S_s exp(-2 pi i f (r_a - r_b) . s_s / c) for a coplanar
    array and isotropic antennas (point-source model, Sec. 2.2)."""
    ant_xy = np.asarray(ant_xy, np.float64)
    Na = ant_xy.shape[0]
    V = np.zeros((Na, Na), np.complex128)
    for l, m, S in np.asarray(model_lmS, np.float64):
        e = np.exp(-2j * np.pi * freq * (ant_xy[:, 0] * l + ant_xy[:, 1] * m) / C_LIGHT)
        V += S * np.outer(e, np.conj(e))
    return V


def denominator(A: np.ndarray, V: np.ndarray, flags: Optional[np.ndarray] = None) -> np.ndarray:
    """D_a = sum over unflagged b != a of conj(A_b(k0)) V^M_ab: the model side
    of eq. (cal_solution), by the direct double sum."""
    Na = A.shape[0]
    ok = np.ones(Na, bool) if flags is None else (np.asarray(flags) == 0)
    D = np.zeros(Na, np.complex128)
    for a in range(Na):
        s = 0.0 + 0.0j
        for b in range(Na):
            if b != a and ok[b]:
                s += np.conj(A[b]) * V[a, b]
        D[a] = s
    return D


# --------------------------------------------------------------------------
# The per-sample (fast, "gray box") steps, Sec. 2.1 and Fig. schematic
# --------------------------------------------------------------------------

def calibrate(E: np.ndarray, g: np.ndarray, flags: Optional[np.ndarray] = None) -> np.ndarray:
    """E'_a = E_a / g'_a (Sec. 2.1); flagged antennas contribute nothing."""
    Ec = E / g
    if flags is not None:
        Ec = np.where(np.asarray(flags) == 0, Ec, 0.0)
    return Ec


def grid(Ecal: np.ndarray, cells: GridCells, nx, ny) -> np.ndarray:
    """E'_j = sum_a W_a(r_j - r_a) E'_a (eq. gridding) for a batch of samples:
    Ecal [nt, Na] -> G [nt, ny, nx]."""
    Ecal = np.atleast_2d(Ecal)
    nt, Na = Ecal.shape
    G = np.zeros((nt, ny, nx), np.complex128)
    for a in range(Na):
        for k in range(cells.w.shape[1]):
            G[:, cells.iy[a, k], cells.ix[a, k]] += cells.w[a, k] * Ecal[:, a]
    return G


def dft_matrix(n: int, sign: int = +1) -> np.ndarray:
    """W[k, j] = exp(sign 2 pi i j k / n), phases reduced modulo n exactly."""
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * (np.outer(j, j) % n) / n)


def dft2(G: np.ndarray, na: float, sign: int = +1) -> np.ndarray:
    """script-E'(s_k) = (1/Na) sum_j E'_j exp(+2 pi i r_j . s_k f / c) on the
    grid (the MOFF summary equation, Sec. 2.1): a naive separable DFT,
    rows then columns, no FFT.  G [..., ny, nx] -> X [..., ny, nx]."""
    ny, nx = G.shape[-2:]
    Wy, Wx = dft_matrix(ny, sign), dft_matrix(nx, sign)
    return (Wy @ G @ Wx.T) / na


def correlate(E: np.ndarray, P: np.ndarray):
    """Interval sums for eq. (Kna_def) and eq. (Cna): K_a = sum_t E_a(t) P*(t)
    with the *uncalibrated* E_a, and Q_a = sum_t |E_a(t)|^2."""
    K = (E * np.conj(P)[:, None]).sum(axis=0)
    Q = (np.abs(E) ** 2).sum(axis=0)
    return K, Q


def gain_update(Kbar, Qbar, A, D, g, na, gamma, flags=None, d_tiny=1e-12):
    """One EPICal update.

    C_a = K_a - conj(A_a) <|E_a|^2> / (Na conj(g_a))       (eq. Cna)
    g_a <- (1 - gamma) C_a Na / D_a + gamma g_a             (eq. damping;
                                                            gamma = 0 gives
                                                            eq. cal_solution)
    Antennas that are flagged, whose |D_a| is below d_tiny * max|D|, or whose
    update is not finite keep g_a.  Returns (g_new, held_mask).
    """
    C = Kbar - np.conj(A) * Qbar / (na * np.conj(g))
    with np.errstate(all="ignore"):
        g_new = (1.0 - gamma) * C * na / D + gamma * g
    dmax = np.max(np.abs(D)) if D.size else 0.0
    held = (np.abs(D) <= d_tiny * dmax) | ~np.isfinite(g_new)
    if flags is not None:
        held |= np.asarray(flags) != 0
    return np.where(held, g, g_new), held


def gain_update_multi(Kbar, Qbar, A, D, g, na, gamma, flags=None, d_tiny=1e-12):
    """EPICal update from several tapped pixels (the multiple-pixel extension
    named in Sec. 6; the paper gives no formula, this is the reading used).

    Each pixel p gives its own autocorrelation-subtracted correlation
      C_ap = K_ap - conj(A_ap) <|E_a|^2> / (Na conj(g_a))        (eq. Cna per pixel)
    whose expectation is g_a D_ap / Na (eq. cal_solution per pixel).  The gain
    is the least-squares solution over the pixels of Na C_ap = g_a D_ap,
      g_a = Na sum_p conj(D_ap) C_ap / sum_p |D_ap|^2,
    damped as in eq. (damping).  With one pixel this is Na C_a / D_a.
    Kbar, A, D: [n_pix, Na].  Antennas that are flagged, whose
    sum_p |D_ap|^2 is below d_tiny^2 times its largest value, or whose update
    is not finite keep g_a.  Returns (g_new, held_mask).
    """
    Kbar, A, D = np.atleast_2d(Kbar), np.atleast_2d(A), np.atleast_2d(D)
    C = Kbar - np.conj(A) * Qbar[None, :] / (na * np.conj(g))[None, :]
    num = np.sum(np.conj(D) * C, axis=0)
    den = np.sum(np.abs(D) ** 2, axis=0)
    with np.errstate(all="ignore"):
        g_new = (1.0 - gamma) * na * num / den + gamma * g
    dmax = np.max(den) if den.size else 0.0
    held = (den <= d_tiny * d_tiny * dmax) | ~np.isfinite(g_new)
    if flags is not None:
        held |= np.asarray(flags) != 0
    return np.where(held, g, g_new), held


# --------------------------------------------------------------------------
# The whole loop (Fig. schematic; Sec. 2.2 feedback schedule)
# --------------------------------------------------------------------------

@dataclass
class Problem:
    """Everything the loop needs for one array (channels independent)."""
    ant_xy: np.ndarray
    freq_hz: np.ndarray
    nx: int
    ny: int
    dx: float
    dy: float
    x0: float
    y0: float
    kernel: int
    model_lmS: np.ndarray
    cal_lm: np.ndarray
    gamma: float
    t_cal: int
    flags: Optional[np.ndarray] = None
    pix_lm: Optional[np.ndarray] = None   # [n_pix, 2] tapped directions (None: the calibrator only)

    @staticmethod
    def from_workload(wl) -> "Problem":
        a = wl.array
        return Problem(ant_xy=a.ant_xy, freq_hz=a.freq_hz, nx=a.nx, ny=a.ny, dx=a.dx, dy=a.dy,
                       x0=a.x0, y0=a.y0, kernel=a.kernel, model_lmS=wl.model_lmS, cal_lm=wl.cal_lm,
                       gamma=wl.gamma, t_cal=wl.t_cal,
                       flags=None if a.ant_flag is None else np.asarray(a.ant_flag))


def channel_setup(pb: Problem, ch: int):
    """Per-channel plan: cells, k0, A(k0), V^M, D, Na."""
    cells = grid_cells(pb.ant_xy, pb.dx, pb.dy, pb.x0, pb.y0, pb.nx, pb.ny, pb.kernel)
    f = float(pb.freq_hz[ch])
    k0 = pixel_of_direction(pb.cal_lm[0], pb.cal_lm[1], f, pb.nx, pb.ny, pb.dx, pb.dy)
    A = pixel_response(cells, k0[0], k0[1], pb.nx, pb.ny)
    V = model_visibilities(pb.ant_xy, f, pb.model_lmS)
    D = denominator(A, V, pb.flags)
    flags = np.zeros(pb.ant_xy.shape[0], np.uint8) if pb.flags is None else np.asarray(pb.flags)
    na = float(np.sum(flags == 0))
    return dict(cells=cells, k0=k0, A=A, V=V, D=D, na=na, flags=flags)


def pixel_setup(pb: Problem, ch: int, s=None):
    """Per-channel tables of every tapped pixel: k_p, A_p, D_p ([n_pix, ...])."""
    s = channel_setup(pb, ch) if s is None else s
    lms = np.atleast_2d(pb.cal_lm if pb.pix_lm is None else pb.pix_lm)
    f = float(pb.freq_hz[ch])
    ks, As, Ds = [], [], []
    for l, m in lms:
        k = pixel_of_direction(l, m, f, pb.nx, pb.ny, pb.dx, pb.dy)
        A = pixel_response(s["cells"], k[0], k[1], pb.nx, pb.ny)
        ks.append(k)
        As.append(A)
        Ds.append(denominator(A, s["V"], pb.flags))
    return dict(s, k=np.array(ks), A_p=np.array(As), D_p=np.array(Ds))


def intervals(n_samples: int, t_cal: int):
    return [(t0, min(t0 + t_cal, n_samples)) for t0 in range(0, n_samples, t_cal)]


def run_channel(E: np.ndarray, pb: Problem, ch: int, g0: np.ndarray, setup=None, keep_taps=False):
    """The calibrated EPIC loop for one channel.

    E [T, Na] complex128 (uncalibrated).  For each calibration interval n the
    current estimate g^(n) calibrates, grids and images every sample; the
    squared images are accumulated; the unsquared image is tapped at k0 and
    correlated with the uncalibrated E-fields; at the end of the interval the
    damped update gives g^(n+1), used for the next interval.

    Returns dict(image = time-averaged I' [ny, nx], gains = [n_int + 1, Na]
    (g^(0) .. g^(n_int)), held = [n_int, Na], taps = [T] if keep_taps).
    """
    s = channel_setup(pb, ch) if setup is None else setup
    cells, (kx0, ky0), A, D, na, flags = s["cells"], s["k0"], s["A"], s["D"], s["na"], s["flags"]
    T = E.shape[0]
    g = np.array(g0, np.complex128).copy()
    I = np.zeros((pb.ny, pb.nx), np.float64)
    hist = [g.copy()]
    held_hist = []
    taps = np.zeros(T, np.complex128) if keep_taps else None
    for (t0, t1) in intervals(T, pb.t_cal):
        Ec = calibrate(E[t0:t1], g, flags)
        X = dft2(grid(Ec, cells, pb.nx, pb.ny), na)
        I += (np.abs(X) ** 2).sum(axis=0)
        P = X[:, ky0, kx0]
        if keep_taps:
            taps[t0:t1] = P
        Eu = np.where(flags == 0, E[t0:t1], 0.0)
        K, Q = correlate(Eu, P)
        nt = t1 - t0
        g, held = gain_update(K / nt, Q / nt, A, D, g, na, pb.gamma, flags)
        hist.append(g.copy())
        held_hist.append(held)
    out = dict(image=I / T, gains=np.array(hist), held=np.array(held_hist))
    if keep_taps:
        out["taps"] = taps
    return out


def run_channel_snapshots(E: np.ndarray, pb: Problem, ch: int, g0: np.ndarray, t_acc: int, setup=None):
    """The calibrated loop of run_channel, imaged in windows: window w holds
    the mean of |script-E'(t)|^2 over the samples w t_acc .. (w+1) t_acc - 1
    (the last window may be short) instead of one mean over the run --
    short-timescale images for transient science (Sec. 1).  The gains follow
    the same recursion as run_channel.  Returns dict(images [n_win, ny, nx],
    gains [n_int + 1, Na])."""
    s = channel_setup(pb, ch) if setup is None else setup
    cells, (kx0, ky0), A, D, na, flags = s["cells"], s["k0"], s["A"], s["D"], s["na"], s["flags"]
    T = E.shape[0]
    n_win = -(-T // t_acc)
    sums = np.zeros((n_win, pb.ny, pb.nx), np.float64)
    g = np.array(g0, np.complex128).copy()
    hist = [g.copy()]
    for (t0, t1) in intervals(T, pb.t_cal):
        X = dft2(grid(calibrate(E[t0:t1], g, flags), cells, pb.nx, pb.ny), na)
        for k in range(t1 - t0):
            sums[(t0 + k) // t_acc] += np.abs(X[k]) ** 2
        K, Q = correlate(np.where(flags == 0, E[t0:t1], 0.0), X[:, ky0, kx0])
        g, _ = gain_update(K / (t1 - t0), Q / (t1 - t0), A, D, g, na, pb.gamma, flags)
        hist.append(g.copy())
    lens = np.array([min(t_acc, T - w * t_acc) for w in range(n_win)], np.float64)
    return dict(images=sums / lens[:, None, None], gains=np.array(hist))


def run_channel_multi(E: np.ndarray, pb: Problem, ch: int, g0: np.ndarray, setup=None):
    """The calibrated loop with several tapped pixels (gain_update_multi).

    Identical to run_channel except that every pixel p of pb.pix_lm is tapped,
    P_p(t) = script-E'(s_p, t), correlated with the uncalibrated E-fields, and
    the update combines the pixels.  Returns dict(image, gains, held).
    """
    s = pixel_setup(pb, ch) if setup is None else setup
    cells, ks, A, D, na, flags = s["cells"], s["k"], s["A_p"], s["D_p"], s["na"], s["flags"]
    T = E.shape[0]
    g = np.array(g0, np.complex128).copy()
    I = np.zeros((pb.ny, pb.nx), np.float64)
    hist = [g.copy()]
    held_hist = []
    for (t0, t1) in intervals(T, pb.t_cal):
        Ec = calibrate(E[t0:t1], g, flags)
        X = dft2(grid(Ec, cells, pb.nx, pb.ny), na)
        I += (np.abs(X) ** 2).sum(axis=0)
        Eu = np.where(flags == 0, E[t0:t1], 0.0)
        nt = t1 - t0
        Ks = []
        for (kx, ky) in ks:
            K, Q = correlate(Eu, X[:, ky, kx])
            Ks.append(K / nt)
        g, held = gain_update_multi(np.array(Ks), Q / nt, A, D, g, na, pb.gamma, flags)
        hist.append(g.copy())
        held_hist.append(held)
    return dict(image=I / T, gains=np.array(hist), held=np.array(held_hist))


def run(E: np.ndarray, pb: Problem, g0: np.ndarray, channels=None):
    """All (or the selected) channels; E [T, F_sel, Na] matches `channels`."""
    chans = list(range(len(pb.freq_hz))) if channels is None else list(channels)
    res = [run_channel(E[:, i], pb, c, g0[c]) for i, c in enumerate(chans)]
    return dict(image=np.stack([r["image"] for r in res]),
                gains=np.stack([r["gains"] for r in res], axis=1),
                held=np.stack([r["held"] for r in res], axis=1))


# --------------------------------------------------------------------------
# Gain solutions shared over a band of channels: the per-channel solutions
# averaged across channels (Sec. 5, LWA demonstration) or fitted by low-order
# polynomials in amplitude and phase over frequency (Sec. 6, fitting gain
# models).  The paper gives no formulas; this is the reading used.
# --------------------------------------------------------------------------

def raw_solution(Kbar, Qbar, A, D, g, na, flags=None, d_tiny=1e-12):
    """The undamped per-channel solution s_a = Na C_a / D_a (eq. Cna and
    eq. cal_solution) and whether it is usable: not flagged, |D_a| above
    d_tiny * max|D|, finite.  Returns (s, ok)."""
    C = Kbar - np.conj(A) * Qbar / (na * np.conj(g))
    with np.errstate(all="ignore"):
        s = C * na / D
    dmax = np.max(np.abs(D)) if D.size else 0.0
    ok = (np.abs(D) > d_tiny * dmax) & np.isfinite(s)
    if flags is not None:
        ok &= np.asarray(flags) == 0
    return s, ok


def band_coordinate(freq_hz, b0: int, b1: int) -> np.ndarray:
    """Frequency coordinate of the channels b0..b1-1 of a band, mapped
    linearly onto [-1, 1] (first channel -1 for increasing frequencies; all
    zero for a band of one channel)."""
    nu = np.asarray(freq_hz[b0:b1], np.float64)
    mid, half = 0.5 * (nu[0] + nu[-1]), 0.5 * (nu[-1] - nu[0])
    return (nu - mid) / half if half != 0 else np.zeros_like(nu)


def band_fit(sol, ok, x, mode: str, deg_amp: int = 0, deg_phase: int = 0):
    """Model of the per-channel solutions of each antenna across a band.

    sol, ok [Fb, Na]: solutions and usability (raw_solution) of the band's
    channels in frequency order; x [Fb]: band_coordinate.
      mode "mean": the mean of the usable solutions (Sec. 5);
      mode "poly": |s| fitted by a polynomial of degree deg_amp in x, and the
        phase, unwrapped along the usable channels in order, by one of degree
        deg_phase (Sec. 6); the model is amp(x) exp(i phase(x)).  A solution
        of exactly zero has no phase and is not usable here.
    Least squares with equal weights.  An antenna needs at least one usable
    channel (mean) or max(deg_amp, deg_phase) + 1 of them (poly).
    Returns (model [Fb, Na] at every channel of the band, fit_ok [Na])."""
    Fb, Na = sol.shape
    model = np.zeros((Fb, Na), np.complex128)
    fit_ok = np.zeros(Na, bool)
    P = np.polynomial.polynomial
    for a in range(Na):
        v = ok[:, a]
        if mode == "mean":
            if v.sum() >= 1:
                model[:, a] = sol[v, a].mean()
                fit_ok[a] = True
        elif mode == "poly":
            v = v & (sol[:, a] != 0)
            if v.sum() < max(deg_amp, deg_phase) + 1:
                continue
            xs, s = x[v], sol[v, a]
            ca = np.linalg.lstsq(np.vander(xs, deg_amp + 1, increasing=True), np.abs(s), rcond=None)[0]
            cp = np.linalg.lstsq(np.vander(xs, deg_phase + 1, increasing=True), np.unwrap(np.angle(s)),
                                 rcond=None)[0]
            model[:, a] = P.polyval(x, ca) * np.exp(1j * P.polyval(x, cp))
            fit_ok[a] = True
        else:
            raise ValueError(mode)
    return model, fit_ok


def run_band(E: np.ndarray, pb: Problem, g0: np.ndarray, band, mode: str = "mean",
             deg_amp: int = 0, deg_phase: int = 0):
    """The calibrated loop of all channels of one array, interval by interval,
    with the gains of the channels band = (b0, b1) taken from the band model.

    E [T, F, Na] uncalibrated.  Every channel is imaged, tapped and correlated
    as in run_channel; at the end of an interval each channel's undamped
    solution s_fa is formed (raw_solution).  Channels outside the band update
    from their own s_fa; the band's channels from the band model m_fa
    (band_fit), both damped as in eq. (damping):
        g_fa <- (1 - gamma) target_fa + gamma g_fa.
    A gain is held when its target is not usable (flagged antenna, no usable
    solution, too few usable channels for the fit) or the update is not
    finite.  Returns dict(image [F, ny, nx], gains [n_int + 1, F, Na],
    held [n_int, F, Na])."""
    F = len(pb.freq_hz)
    b0, b1 = band
    T = E.shape[0]
    st = [channel_setup(pb, c) for c in range(F)]
    x = band_coordinate(pb.freq_hz, b0, b1)
    g = np.array(g0, np.complex128).copy()
    Na = g.shape[1]
    I = np.zeros((F, pb.ny, pb.nx), np.float64)
    hist, held_hist = [g.copy()], []
    for (t0, t1) in intervals(T, pb.t_cal):
        nt = t1 - t0
        sol = np.zeros((F, Na), np.complex128)
        ok = np.zeros((F, Na), bool)
        for c in range(F):
            s = st[c]
            Ec = calibrate(E[t0:t1, c], g[c], s["flags"])
            X = dft2(grid(Ec, s["cells"], pb.nx, pb.ny), s["na"])
            I[c] += (np.abs(X) ** 2).sum(axis=0)
            P = X[:, s["k0"][1], s["k0"][0]]
            K, Q = correlate(np.where(s["flags"] == 0, E[t0:t1, c], 0.0), P)
            sol[c], ok[c] = raw_solution(K / nt, Q / nt, s["A"], s["D"], g[c], s["na"], s["flags"])
        target, use = sol.copy(), ok.copy()
        if b1 > b0:
            model, fit_ok = band_fit(sol[b0:b1], ok[b0:b1], x, mode, deg_amp, deg_phase)
            target[b0:b1] = model
            use[b0:b1] = fit_ok[None, :] & (st[0]["flags"] == 0)[None, :]
        with np.errstate(all="ignore"):
            g_new = (1.0 - pb.gamma) * target + pb.gamma * g
        held = ~use | ~np.isfinite(g_new)
        g = np.where(held, g, g_new)
        hist.append(g.copy())
        held_hist.append(held)
    return dict(image=I / T, gains=np.array(hist), held=np.array(held_hist))


# --------------------------------------------------------------------------
# The visibility-based comparison calibrator and the gain error of Sec. 4
# --------------------------------------------------------------------------

def visibilities(E: np.ndarray) -> np.ndarray:
    """V_ab = <E_a E_b*> over the samples of E [T, Na]: every antenna pair
    correlated over the window (Sec. 4 correlates for the effective
    integration time of the EPICal loop)."""
    E = np.asarray(E, np.complex128)
    return (E.T @ np.conj(E)) / E.shape[0]


def vis_chi2(V, VM, g) -> float:
    """chi^2 = sum_a sum_{b != a} |V_ab - g_a g_b* V^M_ab|^2 (eq. vis_cal)."""
    R = V - np.outer(g, np.conj(g)) * VM
    np.fill_diagonal(R, 0.0)
    return float(np.sum(np.abs(R) ** 2))


def vis_chi2_gains(V, VM, g0, n_iter: int = 2000, tol: float = 1e-14):
    """Gains that minimise eq. (vis_cal), by alternating least squares in the
    form of StEFCal (Salvini & Wijnholds 2014).  With the other gains fixed,
    chi^2 is quadratic in g_a (V and V^M are Hermitian, so the b-a terms
    repeat the a-b ones): with z_ab = g_b* V^M_ab it is minimised by
        g_a = sum_{b != a} conj(z_ab) V_ab / sum_{b != a} |z_ab|^2.
    Every antenna is updated from the previous iterate and every second
    update is averaged with it (which makes the iteration converge).  Stops
    when the largest relative change is below tol.  The global phase is not
    determined by chi^2; it is whatever the iteration from g0 reaches."""
    g = np.array(g0, np.complex128).copy()
    off = ~np.eye(V.shape[0], dtype=bool)
    for it in range(n_iter):
        Z = VM * np.conj(g)[None, :] * off
        g_new = np.sum(np.conj(Z) * V, axis=1) / np.sum(np.abs(Z) ** 2, axis=1)
        if it % 2 == 1:
            g_new = 0.5 * (g_new + g)
        done = np.max(np.abs(g_new - g)) <= tol * np.max(np.abs(g_new))
        g = g_new
        if done:
            break
    return g


def gain_error(g_est: np.ndarray, g_true: np.ndarray) -> float:
    """sigma_g of eq. (gain_error): the rms over channels and antennas of
    |g_est - g_true| / |g_true|.  g [F, Na].  The global phase of a channel's
    gains is unobservable (every calibrator here fixes it only through its
    starting point), so each channel's estimate is first rotated by the
    common phase that minimises its error."""
    g_est = np.atleast_2d(g_est)
    g_true = np.atleast_2d(g_true)
    w = 1.0 / np.abs(g_true) ** 2
    c = np.sum(w * np.conj(g_est) * g_true, axis=1)
    rot = np.where(np.abs(c) > 0, c / np.where(np.abs(c) > 0, np.abs(c), 1.0), 1.0)
    err = np.abs(g_est * rot[:, None] - g_true) ** 2 * w
    return float(np.sqrt(np.mean(err)))


def effective_time(t_cal: float, gamma: float) -> float:
    """t_eff = t_cal (1 + gamma) / (1 - gamma) (eq. teff)."""
    return t_cal * (1.0 + gamma) / (1.0 - gamma)


def epical_gains(E: np.ndarray, pb: Problem, ch: int, g0: np.ndarray, setup=None):
    """The EPICal recursion of run_channel without forming images: the tap of
    each sample is the beamformed sum P = (1/Na) sum_a A_a(k0) E_a / g_a (the
    transform evaluated at k0; the identity is pinned against the imaged
    tap), then eq. (Kna_def), eq. (Cna) and eq. (damping) as in run_channel.
    Returns the gains [n_int + 1, Na]."""
    s = channel_setup(pb, ch) if setup is None else setup
    A, D, na, flags = s["A"], s["D"], s["na"], s["flags"]
    g = np.array(g0, np.complex128).copy()
    hist = [g.copy()]
    for (t0, t1) in intervals(E.shape[0], pb.t_cal):
        Ec = calibrate(E[t0:t1], g, flags)
        P = (Ec @ A) / na
        K, Q = correlate(np.where(flags == 0, E[t0:t1], 0.0), P)
        g, _ = gain_update(K / (t1 - t0), Q / (t1 - t0), A, D, g, na, pb.gamma, flags)
        hist.append(g.copy())
    return np.array(hist)


# --------------------------------------------------------------------------
# Fixed-gain imaging and its gradient (differentiable form)
# --------------------------------------------------------------------------

def image_fixed_gains(E: np.ndarray, g: np.ndarray, cells: GridCells, nx, ny, na, flags=None):
    """I' = <|script-E'|^2>_t with one fixed set of gains: E [T, Na]."""
    X = dft2(grid(calibrate(E, g, flags), cells, nx, ny), na)
    return (np.abs(X) ** 2).mean(axis=0)


def model_image(cells: GridCells, nx, ny, na, ant_xy, freq, src_lmS, sigma: float) -> np.ndarray:
    """The expected time-averaged image (Sec. 2.1, squared and averaged in
    time) of a point-source sky with receiver noise, at exact gains:
    <E'_a E'*_b> = V^M_ab + sigma delta_ab gives

        M_k = sum_s S_s |(1/Na) sum_a A_a(k) e_a(s)|^2 + (sigma / Na^2) sum_a |A_a(k)|^2,

    e_a(s) = exp(-2 pi i f r_a . s_s / c), A_a(k) the gridded antenna's
    response at pixel k.  (1/Na) sum_a A_a(k) e_a(s) is the transform of the
    grid of e(s), and A_a(k) / Na that of antenna a's grid alone."""
    ant_xy = np.asarray(ant_xy, np.float64)
    n_ant = ant_xy.shape[0]
    M = np.zeros((ny, nx), np.float64)
    for l, m, S in np.asarray(src_lmS, np.float64):
        e = np.exp(-2j * np.pi * freq * (ant_xy[:, 0] * l + ant_xy[:, 1] * m) / C_LIGHT)
        M += S * np.abs(dft2(grid(e[None, :], cells, nx, ny), na)[0]) ** 2
    X = dft2(grid(np.eye(n_ant, dtype=np.complex128), cells, nx, ny), na)
    return M + sigma * (np.abs(X) ** 2).sum(axis=0)


def image_gain_gradient(E, g, cells: GridCells, nx, ny, na, R, flags=None):
    """Gradient of a real loss L(I') with respect to the complex gains, given
    R = dL/dI' [ny, nx].

    With X_t = (1/Na) DFT+(grid(u E_t)), u = 1/g and I' = (1/T) sum_t |X_t|^2:
      dL/dX*_t  = (1/T) R X_t
      dL/dG*_t  = (1/Na) DFT-(dL/dX*_t)          (adjoint of the + transform)
      dL/dE'*_a = sum_j W_a(r_j - r_a) dL/dG*_j   (degridding)
      dL/du*_a  = sum_t conj(E_a(t)) dL/dE'*_a(t)
      dL/dg*_a  = conj(-1 / g_a^2) dL/du*_a
    Returned in the convention dL/dRe g + i dL/dIm g = 2 dL/dg*.
    """
    T = E.shape[0]
    Ec = calibrate(E, g, flags)
    X = dft2(grid(Ec, cells, nx, ny), na)
    Z = R[None] * X / T
    Gbar = dft2(Z, na, sign=-1)
    Ebar = np.zeros_like(Ec)
    for a in range(E.shape[1]):
        for k in range(cells.w.shape[1]):
            Ebar[:, a] += cells.w[a, k] * Gbar[:, cells.iy[a, k], cells.ix[a, k]]
    if flags is not None:
        Ebar = np.where(np.asarray(flags) == 0, Ebar, 0.0)
    du = (np.conj(E) * Ebar).sum(axis=0)
    dg = np.conj(-1.0 / g ** 2) * du
    return 2.0 * dg
