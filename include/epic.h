/*
 * epic.h -- C ABI of the MI355X (gfx950) EPIC / EPICal library.
 *
 * The library runs the direct-imaging correlator loop with in-loop feedback
 * calibration of Beardsley et al. (2016), "An Efficient Feedback Calibration
 * Algorithm for Direct Imaging Radio Telescopes" (arXiv:1603.02126):
 * per channel and time sample, calibrate the antenna E-fields with the
 * current gains, grid them with the antenna kernel, take the 2D spatial
 * transform, square and accumulate the image, correlate each antenna with the
 * tapped calibrator pixel, and update the gains once per calibration interval
 * with the damped solution -- without ever forming visibilities.
 *
 * Conventions used by every call
 *   - Return value: EPIC_OK (0) or a negative epic_status.  Nothing aborts or
 *     throws; epic_last_error() gives a message for the calling thread.
 *   - "host" pointers are read during the call and may be freed afterwards.
 *     "device" pointers are caller-owned HIP device memory (e.g. torch tensor
 *     storage) on the plan's device; they must stay valid until the work
 *     enqueued on `stream` has finished.  Device work is asynchronous on
 *     `stream` (a hipStream_t; NULL = the null stream); argument checks are
 *     synchronous and happen before anything is enqueued.
 *   - Every device buffer a call takes starts on a 256-byte boundary (torch
 *     allocations do; a view that starts inside an allocation may not):
 *     EPIC_ERR_ARG otherwise.
 *   - Complex numbers are interleaved (re, im) pairs of the stated real type.
 *   - Array layouts are C order (last index fastest); sizes are elements.
 *   - E-field streams are [T][F][Na] packed samples in the array's format.
 *   - Images are [F][ny][nx] in natural (unshifted) transform order: pixel
 *     (ky, kx) with signed index kappa = k (k < N/2) or k - N (k >= N/2) lies
 *     at direction cosine l = kappa c / (f N d) (Sec. 2.1).
 *   - Gains g are [F][Na] complex128.  E'_a = E_a / g_a (Sec. 2.1).
 *   - A plan is used by one host thread at a time; plans are independent.
 */
#ifndef EPIC_H
#define EPIC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct epic_plan_s* epic_plan_t;
typedef void* epic_stream_t; /* hipStream_t */

typedef enum {
  EPIC_OK = 0,
  EPIC_ERR_ARG = -1,         /* bad pointer, size, shape, format or parameter */
  EPIC_ERR_ALLOC = -2,       /* device or host allocation failed */
  EPIC_ERR_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  EPIC_ERR_UNSUPPORTED = -4, /* valid but not implemented (e.g. grid size) */
  EPIC_ERR_STATE = -5        /* call out of order (e.g. no model set) */
} epic_status;

/* Packed antenna E-field sample formats (the F-engine output, Sec. 2.1). */
typedef enum {
  EPIC_CF32 = 0, /* 8 bytes: float32 re, float32 im */
  EPIC_CI8 = 1,  /* 2 bytes: int8 re, int8 im */
  EPIC_CI4 = 2   /* 1 byte: re in bits 7..4, im in bits 3..0, two's complement */
} epic_efmt;

/* Per-antenna status bits (OR-ed over all updates of a run). */
#define EPIC_ANT_FLAGGED 1u    /* flagged on input: not gridded/correlated/updated */
#define EPIC_ANT_D_ZERO 2u     /* |D_a| <= 1e-12 max|D|: gain held */
#define EPIC_ANT_NONFINITE 4u  /* update not finite: gain held */
#define EPIC_ANT_BAND_HELD 8u  /* band model without enough usable channels: gain held */
#define EPIC_ANT_BARRIER 16u   /* band solve: a grid barrier did not complete (gains NaN) */

/* One antenna array and its aperture grid (Sec. 2.1, eq. gridding).
 * Positions and grid are in metres.  Grid cell (jx, jy) sits at
 * (x0 + jx dx, y0 + jy dy); cell indices wrap modulo the grid size.
 * kernel 1 = nearest cell, jx = floor((x - x0)/dx + 0.5);
 * kernel 2 = 2x2 bilinear (area overlap of a one-cell tophat):
 *   i0 = floor(p), phi = p - i0, weights (1-phi, phi) per axis.
 * The imaging calls take nx == ny, a power of two in {16, 32, 64, 128, 256}:
 * Na <= 8 nx for nx <= 64 (and a gridding schedule that fits the LDS slot
 * table: at 64 x 64, 512 antennas fit with kernel 1 but not kernel 2),
 * Na <= 2048 for 128 and 256.  The stage-wise calls and the adjoint take
 * grids up to 64 x 64.  Other shapes give EPIC_ERR_UNSUPPORTED. */
typedef struct {
  int32_t n_ant;           /* Na >= 1 */
  int32_t n_chan;          /* F >= 1 */
  int32_t nx, ny;          /* grid size */
  int32_t kernel;          /* 1 or 2 */
  int32_t efmt;            /* epic_efmt */
  double dx, dy, x0, y0;   /* cell size and origin, metres */
  const double* ant_xy;    /* host [Na][2] antenna (x, y), metres */
  const double* freq_hz;   /* host [F] channel frequencies, Hz (> 0) */
  const uint8_t* ant_flag; /* host [Na], nonzero = flagged; or NULL */
} epic_array_desc;

/* Calibration model (Sec. 2.2): point-source sky for the model visibilities
 * V^M_ab = sum_s S_s exp(-2 pi i f (r_a - r_b) . s_s / c), the calibrator
 * direction whose nearest pixel k0 is tapped (eq. Kna_def), the damping
 * factor (eq. damping, 0 <= gamma < 1) and the calibration interval length in
 * samples (Fig. times). */
typedef struct {
  const double* src_lmS; /* host [n_src][3]: l, m, flux (data units) */
  int32_t n_src;         /* >= 1 */
  double cal_l, cal_m;   /* calibrator direction cosines */
  double gamma;          /* damping, [0, 1) */
  int32_t t_cal;         /* samples per calibration interval, >= 1 */
} epic_model_desc;

/* ---------------------------------------------------------------------- */
/* Library information and host-only helpers (no device needed)           */
/* ---------------------------------------------------------------------- */

/* ABI version, currently 2 (2: tuning records of four values). */
int32_t epic_abi_version(void);

/* Message describing the last error on this thread ("" if none).  Valid until
 * the next call on this thread. */
const char* epic_last_error(void);

/* Grid cells and kernel weights of each antenna (eq. gridding), exactly as the
 * device tables use them.  ixy: host [Na][K][2] int32 (jx, jy) after the
 * modulo wrap; w: host [Na][K] float64; K = 1 (kernel 1) or 4 (kernel 2),
 * cells in the order (i0,j0), (i0+1,j0), (i0,j0+1), (i0+1,j0+1).  Flagged
 * antennas are reported like the others. */
int epic_host_grid_cells(const epic_array_desc* desc, int32_t* ixy, double* w);

/* Calibrator pixel and model-side quantities per channel, computed on the
 * host in float64 exactly as the plan uses them.
 *   k0: host [F][2] int32 (kx, ky), the pixel nearest (cal_l, cal_m):
 *       kappa = floor(l f N d / c + 0.5) mod N.
 *   A:  host [F][Na] complex128, A_a(k0) = sum_j w_aj exp(+2 pi i j . k0 / N),
 *       the gridded antenna's response at the tapped pixel.  It stands for
 *       the factor W_b(s0) exp(+2 pi i f s0 . r_b / c) of eq. (Cna).
 *   D:  host [F][Na] complex128, D_a = sum_{b != a, b unflagged}
 *       conj(A_b) V^M_ab, the denominator of eq. (cal_solution), evaluated in
 *       O(Na * n_src) per channel by factoring V^M over sources.
 * Any of k0, A, D may be NULL. */
int epic_host_calibrator(const epic_array_desc* desc, const epic_model_desc* model,
                         int32_t* k0, double* A, double* D);

/* The same tables for several tapped pixels (see epical_set_model_pixels):
 * k0 host [n_pix][F][2], A and D host [n_pix][F][Na] complex128; any may be
 * NULL. */
int epic_host_calibrator_pixels(const epic_array_desc* desc, const epic_model_desc* model, const double* pix_lm,
                                int32_t n_pix, int32_t* k0, double* A, double* D);

/* The band coordinate of epical_set_band: host x[F], the frequencies of
 * channels b0..b1-1 mapped linearly onto [-1, 1] in channel order
 * (x = (f - mid) / half, mid and half from the first and last channel of the
 * band; all 0 for a band of one channel), 0 outside the band. */
int epic_host_band_coordinate(const epic_array_desc* desc, int32_t b0, int32_t b1, double* x);

/* ---------------------------------------------------------------------- */
/* Plans                                                                   */
/* ---------------------------------------------------------------------- */

/* Create a plan for n_arrays arrays on the current HIP device.  The plan
 * copies the descriptors, builds the gridding tables and owns all device
 * tables and scratch memory.  *out receives the plan. */
int epic_plan_create(const epic_array_desc* arrays, int32_t n_arrays, epic_plan_t* out);

/* Release the plan and its device memory (synchronises the device first). */
int epic_plan_destroy(epic_plan_t plan);

/* Set the calibration model of one array (required before epical_update and
 * epic_run): computes k0, A and D on the host and uploads them. */
int epical_set_model(epic_plan_t plan, int32_t array, const epic_model_desc* model);

/* EPICal from several tapped pixels (the multiple-pixel correlations named
 * in Sec. 6; the paper gives no formula, the reading used is stated here).
 * Like epical_set_model, with the tapped directions given explicitly (the
 * model's cal_l, cal_m are not used).
 *   pix_lm: host [n_pix][2] direction cosines (l, m), 1 <= n_pix <=
 *           EPIC_MAX_PIX; copied.  Pixel 0 is the one epic_image_accumulate
 *           reports as the tap.
 * Each pixel p has its own k_p, A_ap and D_ap (as epic_host_calibrator
 * computes them for one direction); epic_run taps every pixel,
 * P_p(t) = script-E'(s_p, t), correlates it with the uncalibrated E-fields,
 * C_ap = <E_a P_p*> - conj(A_ap) <|E_a|^2> / (Na conj g_a) (eq. Cna per
 * pixel), and updates each gain with the least-squares solution over the
 * pixels of Na C_ap = g_a D_ap (eq. cal_solution per pixel), damped as in
 * eq. (damping):
 *   g_a <- (1 - gamma) Na sum_p conj(D_ap) C_ap / sum_p |D_ap|^2 + gamma g_a.
 * With one pixel this is epical_set_model's update.  An antenna whose
 * sum_p |D_ap|^2 is below 1e-24 of the largest is held.  Needs Na <= 1024
 * when n_pix > 1 (EPIC_ERR_UNSUPPORTED otherwise); epical_update (one tap
 * per sample) then returns EPIC_ERR_UNSUPPORTED. */
#define EPIC_MAX_PIX 4
int epical_set_model_pixels(epic_plan_t plan, int32_t array, const epic_model_desc* model, const double* pix_lm,
                            int32_t n_pix);

/* Gains shared over a band of channels (Sec. 5: solutions averaged across
 * the central channels of the LWA band; Sec. 6: fitting a gain model, a
 * low-order polynomial in amplitude and phase over frequency).  The paper
 * gives no formulas; the reading used is stated here.
 *   mode EPIC_BAND_NONE   every channel updates from its own solution (default);
 *   mode EPIC_BAND_MEAN   the channels b0..b1-1 share the mean of their solutions;
 *   mode EPIC_BAND_POLY   the channels b0..b1-1 take amp(x) exp(i phase(x)), with
 *                         |s| fitted by a polynomial of degree deg_amp and the
 *                         phase, unwrapped along the usable channels in channel
 *                         order, by one of degree deg_phase (0..EPIC_BAND_MAX_DEG),
 *                         least squares with equal weights; a solution of
 *                         exactly zero has no phase and is left out.
 * Here s_fa = Na C_fa / D_fa is channel f's undamped solution (eq. Cna,
 * eq. cal_solution) at the end of an interval, and x the band coordinate:
 * the band's frequencies mapped linearly onto [-1, 1] in channel order
 * (epic_host_band_coordinate).  Every channel of the band is then damped
 * towards the model as in eq. (damping): g_fa <- (1 - gamma) m_fa + gamma g_fa;
 * channels outside the band keep their own update.  A channel's solution is
 * left out where the antenna is held (flagged, |D| below 1e-12 of the
 * largest, not finite); an antenna with no usable channel (mean) or fewer
 * than max(deg_amp, deg_phase) + 1 of them (poly) keeps its gains in the band
 * (EPIC_ANT_BAND_HELD).  The polynomial model needs strictly monotonic frequencies
 * over the band.  epic_run then solves all channels of the array in one
 * cooperative launch (every workgroup resident, grid-wide barriers between
 * the per-channel solutions, the band model and the update; a barrier that
 * does not complete leaves NaN gains and EPIC_ANT_BARRIER).  Needs Na <= 1024,
 * one tapped pixel and the per-array form (EPIC_OPT_BATCH 0 or 2, no
 * EPIC_OPT_GRAPH), else EPIC_ERR_UNSUPPORTED; epical_update then returns
 * EPIC_ERR_UNSUPPORTED.  b0, b1 are ignored for EPIC_BAND_NONE. */
#define EPIC_BAND_NONE 0
#define EPIC_BAND_MEAN 1
#define EPIC_BAND_POLY 2
#define EPIC_BAND_MAX_DEG 3
int epical_set_band(epic_plan_t plan, int32_t array, int32_t b0, int32_t b1, int32_t mode, int32_t deg_amp,
                    int32_t deg_phase);

/* Caller-supplied model denominator (eq. cal_solution: D_a = sum_{b != a}
 * conj(W_b(s0)) V^M_ab, which Sec. 2.2 notes is computed before observing,
 * from whatever model of the sky the caller holds), in place of the one
 * epical_set_model derives from its point-source list.  Needs a prior
 * epical_set_model / epical_set_model_pixels call, which fixes the tapped
 * pixels, A, gamma and t_cal (EPIC_ERR_STATE otherwise).
 *   D: host [n_pix][F][Na] complex128 (n_pix of that call, 1 for
 *      epical_set_model), finite (EPIC_ERR_ARG otherwise); copied.
 * The hold rule is re-derived from D: an antenna whose sum_p |D_ap|^2 is at
 * most 1e-24 of the channel's largest (|D_a| <= 1e-12 max|D| for one pixel)
 * is held; flagged antennas stay held.  Waits for the device. */
int epical_set_denominator(epic_plan_t plan, int32_t array, const double* D);

/* Options (key, value).  Keys:
 *   EPIC_OPT_SPLITS      time splits per channel of the imaging launch (0 = auto)
 *   EPIC_OPT_TRANSFORM   0 = FFT, 1 = FFT (FP32), or the 2D DFT as two complex
 *                        GEMMs on the matrix cores with split 16-bit operands
 *                        and FP32 accumulation: 2 = fp16 hi + lo (three part
 *                        products, ~22 bits), 3 = bf16 hi + lo (three, ~16 bits),
 *                        4 = bf16 hi + mid + lo (six, ~24 bits).  Grids
 *                        32 and 64 (up to 512 antennas), and 128 and 256 as
 *                        residue classes of 64 x 64 DFT-GEMMs (up to 512
 *                        antennas); imaged with one launch per array even when
 *                        batched.  Arrays the DFT-GEMM does not cover use the FFT.
 *   EPIC_OPT_TIMING      1 = record HIP events around each kernel (see below)
 *   EPIC_OPT_BATCH       0 = batched when the plan has several arrays, 1 = always
 *                        batched, 2 = never.  Batched, epic_run makes one launch per
 *                        stage for all arrays: one calibration solve, one
 *                        persistent imaging kernel pulling (array, channel, class,
 *                        time split) items from a work queue, one reduction.
 *   EPIC_OPT_GRAPH       1 = epic_run captures its batched launches in a hipGraph
 *                        on a plan-owned stream (ordered after and before the
 *                        caller's stream by events) and replays it while the
 *                        buffers and n_samples stay the same.
 *   EPIC_OPT_OVERLAP     1 (default) = where every array of the plan allows it
 *                        (no band; one tapped pixel with more than 64 antennas
 *                        or intervals longer than 8 samples, or several tapped
 *                        pixels with at most 512 antennas; an imaging engine of
 *                        the persistent kernel, the FFT transform) and the
 *                        plan's channels number fewer than the GPU's CUs (the
 *                        solve, one workgroup per channel, leaves CUs idle),
 *                        epic_run makes one launch for the calibration solve
 *                        and the imaging: the solve of each channel publishes
 *                        each interval's calibration as soon as it is known and
 *                        the imaging of a time split starts once its intervals
 *                        are published, so that the imaging runs on the CUs the
 *                        solve leaves free; results equal the separate launches'
 *                        (with one pixel gains bit for bit, with several the
 *                        same sums in another order; images within rounding).
 *                        Timing then counts the one launch as imaging.
 *                        0 = separate launches.  epic_run_noalloc never fuses. */
#define EPIC_OPT_SPLITS 1
#define EPIC_OPT_TRANSFORM 2
#define EPIC_OPT_TIMING 3
#define EPIC_OPT_BATCH 4
#define EPIC_OPT_GRAPH 5
#define EPIC_OPT_OVERLAP 6
/* EPIC_OPT_WAIT_POLLS  the bound of one wait of the fused run's imaging for
 *                      the calibration it needs, in polls of about 0.2 us
 *                      (0 = the default, 2^23, about 2 s; the waits always end
 *                      well before it).  A wait that reaches the bound gives
 *                      up, and the run writes NaN images (the gains are not
 *                      affected); a small bound makes that path testable.
 *                      Values above the default give EPIC_ERR_ARG. */
#define EPIC_OPT_WAIT_POLLS 7
int epic_plan_set_option(epic_plan_t plan, int32_t key, int64_t value);

/* Kernel timing, when EPIC_OPT_TIMING is on.  Events are recorded on the
 * stream each kernel is launched on.  Fills ms[k] with the total elapsed
 * milliseconds and launches[k] with the launch count of kernel kind k since
 * the last call, for k < n (kinds: 0 calibration solve, 1 imaging,
 * 2 image reduction, 3 adjoint, 4 a whole graph replay); waits for the
 * recorded events. */
#define EPIC_TIMER_SOLVE 0
#define EPIC_TIMER_IMAGE 1
#define EPIC_TIMER_REDUCE 2
#define EPIC_TIMER_ADJOINT 3
#define EPIC_TIMER_GRAPH 4
#define EPIC_TIMER_COUNT 5

/* Autotuner: for every array, time the imaging launch of the given E-field
 * stream (n_samples samples) with each candidate transform (FFT; for the grids
 * and arrays the DFT-GEMM covers, its three precisions), time-split count
 * (frames per workgroup) and, at 128 x 128 and 256 x 256 with integer
 * samples, residue-class engine (the default, and the dense engine with
 * gridding batches of 2 and 4 schedule entries), and keep the fastest for
 * later runs.
 * Synchronous (waits for the device); efield: one device pointer per array. */
int epic_plan_autotune(epic_plan_t plan, const void* const* efield, int64_t n_samples,
                       epic_stream_t stream);

/* epic_plan_autotune with a tuning cache: cache_path (host string) names a
 * JSON file of entries keyed by the GPU architecture, grid size, antenna
 * count, kernel, sample format, channel count and n_samples.  Arrays with an
 * entry take it without timing; the others are timed and their entries
 * added (the file is rewritten then).  A missing file starts an empty
 * cache; lines that are not entries of this format are ignored.  NULL
 * cache_path is epic_plan_autotune. */
int epic_plan_autotune_cached(epic_plan_t plan, const void* const* efield, int64_t n_samples,
                              const char* cache_path, epic_stream_t stream);

/* Tuning state per array: tuning[4 i + 0] = transform (EPIC_OPT_TRANSFORM
 * values 1..4, 0 = plan default), [4 i + 1] = time splits (0 = auto),
 * [4 i + 2] = residue-class engine (grids 128 and 256, integer samples):
 * 0 = default (the class-pair engine up to 512 antennas where its tables
 * fit, else the dense engine gridding 2 schedule entries per batch), 2 or 4 =
 * the dense engine with batches of 2 or 4 entries (ignored where it does not
 * apply: cf32 samples, other grids, more antennas than it stages),
 * [4 i + 3] = measured imaging time in microseconds (get only).  Host arrays
 * of 4 * n_arrays. */
int epic_plan_get_tuning(epic_plan_t plan, int32_t* tuning);
int epic_plan_set_tuning(epic_plan_t plan, const int32_t* tuning);
int epic_plan_get_timing(epic_plan_t plan, double* ms, int64_t* launches, int32_t n);

/* Read back the plan's device gridding tables of one array (eq. gridding):
 * ixy host [Na][K][2] int32 (jx, jy) after the modulo wrap, w host [Na][K]
 * float32 kernel weights as the device holds them, K = 1 (kernel 1) or 4
 * (kernel 2) in the cell order of epic_host_grid_cells.  Flagged antennas
 * carry weight 0 (they are not gridded).  Synchronous. */
int epic_plan_get_cells(epic_plan_t plan, int32_t array, int32_t* ixy, float* w);

/* Decode n packed integer samples (the F-engine output, Sec. 2.1) with the
 * imaging engines' own unpacking, for checking it:
 *   out[i] = (re, im) of sample i of `efield`, as int16.
 * efield: device, n samples in the array's format (EPIC_CI4 or EPIC_CI8;
 * EPIC_CF32 gives EPIC_ERR_UNSUPPORTED); out: device [n][2] int16. */
int epic_debug_unpack(epic_plan_t plan, int32_t array, const void* efield, int64_t n, int16_t* out,
                      epic_stream_t stream);

/* ---------------------------------------------------------------------- */
/* Stage-wise calls (each stage of the loop on its own, through HBM)       */
/* ---------------------------------------------------------------------- */

/* Calibrate and grid (Sec. 2.1: E'_a = E_a u_a, eq. gridding):
 *   grid[t][f][jy][jx] = sum_a sum_k w_ak [cell_ak == (jx,jy)] E_a(t0+t, f) u[f][a]
 * efield: device [T][F][Na] packed, samples t0 .. t0+nt-1 are read.
 * u:      device [F][Na] complex64, the applied calibration 1/g (any values).
 * grid:   device [nt][F][ny][nx] complex64, overwritten.
 * Flagged antennas are not gridded. */
int epic_grid(epic_plan_t plan, int32_t array, const void* efield, int64_t t0, int32_t nt,
              const float* u, float* grid, epic_stream_t stream);

/* Transform, square and accumulate (Sec. 2.1 MOFF summary equation; squaring
 * and time averaging):
 *   X_t(k) = (1/Na) sum_j grid[t][f][j] exp(+2 pi i (jx kx/nx + jy ky/ny))
 *   image[f][ky][kx] += sum_t |X_t(k)|^2     (not divided by nt)
 *   tap[t][f] = X_t(k0_f)                    (if tap != NULL; needs a model)
 * grid: device [nt][F][ny][nx] complex64; image: device [F][ny][nx] float32,
 * accumulated; tap: device [nt][F] complex64 or NULL.  Na = unflagged count. */
int epic_image_accumulate(epic_plan_t plan, int32_t array, const float* grid, int32_t nt,
                          float* image, float* tap, epic_stream_t stream);

/* EPICal correlation and update (eq. Kna_def, Cna, damping):
 *   kq[f][a] += (sum_t E_a(t) conj(tap[t][f]), sum_t |E_a(t)|^2, nt)
 * with the uncalibrated E-fields of samples t0 .. t0+nt-1.  If finalize != 0,
 * then with Kbar = K/n, Qbar = Q/n:
 *   C_a = Kbar_a - conj(A_a) Qbar_a / (Na conj(g_a))
 *   g_a <- (1 - gamma) Na C_a / D_a + gamma g_a
 * (gains held for flagged antennas, |D_a| <= 1e-12 max|D|, or a non-finite
 * update), and kq is reset to zero.
 * efield: device packed; tap: device [nt][F] complex64; kq: device [F][Na][4]
 * float64 (K re, K im, Q, n), zero it before the first call of an interval;
 * gains: device [F][Na] complex128 in/out; status: device [F][Na] uint32 OR-ed
 * with EPIC_ANT_* bits, or NULL.  nt may be 0 (finalize only). */
int epical_update(epic_plan_t plan, int32_t array, const void* efield, int64_t t0, int32_t nt,
                  const float* tap, double* kq, double* gains, int32_t finalize,
                  uint32_t* status, epic_stream_t stream);

/* ---------------------------------------------------------------------- */
/* The fused loop                                                          */
/* ---------------------------------------------------------------------- */

/* Run the calibrated EPIC loop over n_samples samples of every array
 * (Fig. schematic): interval n (t_cal samples, the last may be short) is
 * calibrated with g^(n); its tapped pixel and uncalibrated E-fields give
 * g^(n+1) by eq. (damping).  The tapped pixel is evaluated as the equal
 * beamformed sum (1/Na) sum_a A_a(k0) E_a / g_a of the gridded transform.
 * Per array i:
 *   efield[i]:    device [n_samples][F][Na] packed
 *   gains[i]:     device [F][Na] complex128; in: g^(0), out: g^(n_int)
 *   image[i]:     device [F][ny][nx] float32, out: (1/n_samples) sum_t |X_t|^2
 *   gain_hist[i]: device [n_int+1][F][Na] complex128 (g^(0) .. g^(n_int)) or NULL
 *   ant_status[i]:device [F][Na] uint32 (EPIC_ANT_* bits) or NULL
 * gain_hist and ant_status may themselves be NULL. */
int epic_run(epic_plan_t plan, const void* const* efield, int64_t n_samples, double* const* gains,
             float* const* image, double* const* gain_hist, uint32_t* const* ant_status,
             epic_stream_t stream);

/* epic_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, hosts that forbid hipMalloc): the same
 * loop, arguments, layouts and results as epic_run, with every intermediate
 * buffer (FP32 calibration per interval, partial images, the gain history
 * when gain_hist is NULL, the band solve's exchange area) in one static
 * device array of EPIC_STATIC_SCRATCH_BYTES per GPU, allocated when the
 * library's code is loaded on the device and held until the process ends.
 * The call makes no device or host allocation: it launches the per-array
 * kernels of epic_run (no batched work list, no graph, no timing events,
 * whatever the plan's options say).  If the run does not fit, the time splits
 * of the imaging launches are reduced (results agree with epic_run within
 * rounding); if it still does not fit, EPIC_ERR_ARG (pass gain_hist, or fewer
 * samples or channels per call).  Every call on a GPU shares that GPU's
 * array: calls that overlap in time on one GPU (several streams, threads or
 * plans) race and give wrong results; calls in one stream order are safe.
 * The array's device address is looked up once per device when a plan is
 * created on it; if that failed, this call returns EPIC_ERR_HIP. */
#define EPIC_STATIC_SCRATCH_BYTES (64ll << 20)
int epic_run_noalloc(epic_plan_t plan, const void* const* efield, int64_t n_samples, double* const* gains,
                     float* const* image, double* const* gain_hist, uint32_t* const* ant_status,
                     epic_stream_t stream);

/* Snapshot images of one array: the calibrated loop of epic_run (the same
 * calibration solve and gains) with one image per window of t_acc
 * consecutive samples instead of one image over the run -- the short
 * timescale images for transient science that motivate direct imaging
 * (Sec. 1: output rate and millisecond events).
 *   efield:    device [n_samples][F][Na] packed
 *   gains:     device [F][Na] complex128; in: g^(0), out: g^(n_int)
 *   images:    device [n_win][F][ny][nx] float32, n_win = ceil(n_samples / t_acc);
 *              window w = mean of |X_t|^2 over t = w t_acc .. min((w+1) t_acc, n_samples) - 1
 *              (the last window may be short), X_t as in epic_run
 *   gain_hist, ant_status: as in epic_run (may be NULL)
 * t_acc >= 1 (1: one image per sample).  Grids up to 64 x 64, FFT transform
 * (EPIC_ERR_UNSUPPORTED otherwise); several tapped pixels and gains shared
 * over a band apply as in epic_run. */
int epic_run_snapshots(epic_plan_t plan, int32_t array, const void* efield, int64_t n_samples, int64_t t_acc,
                       double* gains, float* images, double* gain_hist, uint32_t* ant_status,
                       epic_stream_t stream);

/* Fixed-gain imaging of one array (the loop with calibration frozen):
 *   image[f] = (1/n_samples) sum_t |X_t|^2 with E'_a = E_a / g[f][a].
 * gains: device [F][Na] complex128.  image: device [F][ny][nx] float32. */
int epic_image(epic_plan_t plan, int32_t array, const void* efield, int64_t n_samples,
               const double* gains, float* image, epic_stream_t stream);

/* Adjoint of epic_image with respect to the gains, for a real loss L(image):
 * given dL_dI = dL/dimage (device [F][ny][nx] float32) and the gains g
 * (device [F][Na] complex128), writes
 *   dL_dg[f][a] = dL/dRe g + i dL/dIm g  (= 2 dL/dg*)
 * as device [F][Na] complex128 (zero for flagged antennas).  Per-sample
 * transforms are recomputed, not stored:
 *   dL/dg*_a = conj(-1/g_a^2) (1/(T Na^2)) sum_t conj(E_a(t))
 *              sum_k w_ak [DFT-(R . DFT+(G_t))](cell_ak),   R = dL_dI. */
int epic_image_adjoint(epic_plan_t plan, int32_t array, const void* efield, int64_t n_samples,
                       const double* gains, const float* dL_dI, double* dL_dg,
                       epic_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* EPIC_H */
