#!/usr/bin/env python3
"""Benchmark of the calibrated EPIC loop on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lwa|lwa_band|hera|uneven|diff|tiny]

A step is one pass of the whole hot path over one batch of synthetic input:
EPICal calibration solve (tap, correlation, damped FP64 update every t_cal
samples) followed by calibrate + grid + 2D FFT + |X|^2 accumulation of every
(channel, sample) frame, as epic_run does it.  The default workload is the
LWA-station shape: 256 antennas, 4+4-bit E-fields, 128 channels, 64x64 grid
with the 2x2 kernel, 10,000 samples, gains updated every 100 samples.  The
E-field stream is resident in HBM before timing starts; each step restarts
from the same initial gains.

Other workloads: "hera" (350 antennas on a hexagonal lattice, 8+8-bit, 512
channels, 128x128, 2000 samples), "uneven" (eight arrays of 64..2048 antennas
on 32^2..256^2 grids, 256 channels, 500 samples: one step images all of
them), "diff" (fixed-gain image plus its hand-written adjoint, 64 channels,
1000 samples: one step is forward + backward).

Prints one JSON line (value = frames/s, frame = one channel x one sample of
one array), with the roofline of the dominant kernel measured by HIP events on
the stream it runs on, the FP64 oracle timed on the host cores on a bounded
sample of the same workload, and the alternative forms (split-precision
DFT-GEMM on the matrix cores; batched launches in a hipGraph after autotuning)
timed on the same inputs, with their error against the oracle.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1603_02126_amd import synth  # noqa: E402

PEAK_FP32_VECTOR_TFLOPS = 157.3   # MI355X published dense FP32 vector peak
PEAK_FP16_MFMA_TFLOPS = 2500.0    # MI355X published dense FP16 / BF16 matrix peak
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the imaging kernel on the LWA-shaped workload (averaged
# and snapshot forms), from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE in KiB
# per dispatch), each scaled by what the same counter reads for a plain 256 MiB
# device copy (FETCH x2.000, WRITE x1.000).  Valid only for the sources that
# determine the imaging kernels' code and their launch configuration (the time
# splits, chosen in epic_api.hip), as they were when the counters were taken:
# any change to one of them makes the figure stale and it is reported as null.
TRAFFIC_SOURCES = ("k_image.hip", "image_fft.h", "image_cls.h", "engine.h", "fft_reg.h", "xpose.h", "epic_internal.h",
                   "epic_api.hip")
TRAFFIC_MEASURED = {
    "lwa": {"sources_sha256": "cf146e0725967256acff341d28546c9dbb3940fe1e8653b838f13ed1e69d1254",
            "fetch_kib": 173447.7, "fetch_scale": 2.000, "write_kib": 8192.0, "write_scale": 1.000},
    "lwa_snapshot1": {"sources_sha256": "cf146e0725967256acff341d28546c9dbb3940fe1e8653b838f13ed1e69d1254",
                      "fetch_kib": 174325.0, "fetch_scale": 2.000, "write_kib": 20480115.3, "write_scale": 1.000},
}


# Issue-slot and LDS use of the LWA imaging kernel from rocprofv3 --pmc SQ
# counters (same validity rule as the traffic figures): the fraction of its
# SIMDs' FP32 issue rate the VALU instructions use (SQ_ACTIVE_INST_VALU per
# wave, two waves per SIMD, four cycles per instruction and wave) and the
# fraction of the launch the LDS is busy (SQ_LDS_IDX_ACTIVE per CU).
SQ_MEASURED = {
    "lwa": {"sources_sha256": "cf146e0725967256acff341d28546c9dbb3940fe1e8653b838f13ed1e69d1254", "valu_issue_frac": 0.58, "lds_busy_frac": 0.56},
}


def measured_sq(workload_name):
    m = SQ_MEASURED.get(workload_name)
    if m is None or m["sources_sha256"] != imaging_sources_digest():
        return None
    return {k: v for k, v in m.items() if k != "sources_sha256"}


def imaging_sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1603_02126_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload_name):
    m = TRAFFIC_MEASURED.get(workload_name)
    if m is None or m["sources_sha256"] != imaging_sources_digest():
        return None
    return (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024.0


def dft_mfma_flops_per_frame(n, products=3):
    """Executed matrix-core flops of the split-precision DFT-GEMM per frame:
    two complex M x M x M products, four real GEMMs each, `products` part
    products per real GEMM (3 for hi + lo, 6 for hi + mid + lo), for each of
    the (n / M)^2 residue classes of 64 x 64 (M = min(n, 64))."""
    m = min(n, 64)
    return (n // m) ** 2 * 2 * 4 * products * 2 * m ** 3


TRANSFORM_NAMES = ["default", "fft", "dft_gemm_fp16_split", "dft_gemm_bf16_split", "dft_gemm_bf16x3_split"]

# the DFT-GEMM forms: (name, EPIC_OPT_TRANSFORM value, part products per real product)
DFT_FORMS = (("dft_gemm_fp16_split", 2, 3), ("dft_gemm_bf16_split", 3, 3), ("dft_gemm_bf16x3_split", 4, 6))


def imaging_flops_per_frame(n, na, k2):
    """Algorithmic flops of one frame in the imaging kernel: radix-2 FFT count
    5 Ng log2 Ng, calibration 6 per antenna, gridding 4 per kernel cell per
    antenna, |X|^2 accumulation 4 per pixel."""
    ng = n * n
    return 5 * ng * math.log2(ng) + na * (6 + 4 * k2) + 4 * ng


def adjoint_flops_per_frame(n, na, k2):
    """Algorithmic flops of one frame of the adjoint: the forward frame again
    (calibrate, grid, FFT), R * X (2 per pixel), the conjugate FFT, degridding
    (4 per kernel cell per antenna) and the conj(E) product-accumulate (8 per
    antenna)."""
    ng = n * n
    return 2 * 5 * ng * math.log2(ng) + na * (6 + 4 * k2) + 2 * ng + na * (4 * k2 + 8)


def imaging_bytes_per_frame(na, bpe, n, n_samples, t_cal):
    """Algorithmic HBM bytes of one frame: the packed E-fields once, u once per
    interval per antenna, the image written once per run."""
    return na * bpe + 8.0 * na / t_cal + 4.0 * n * n / n_samples


def workload(name):
    if name == "lwa":
        return synth.config_lwa()
    if name == "lwa_band":
        return synth.config_lwa_band()
    if name == "hera":
        return synth.config_hera()
    if name == "tiny":
        return synth.config_tiny()
    if name == "diff":
        return synth.config_diff()
    if name == "uneven":
        return synth.config_uneven()
    raise SystemExit(f"unknown workload {name}")


def describe(wl):
    a = wl.array
    fmt = synth.FMT_NAMES[a.efmt]
    return (f"{wl.name}: {a.n_ant} antennas {fmt}, {a.n_chan} channels "
            f"{a.freq_hz[0] / 1e6:.1f}-{a.freq_hz[-1] / 1e6:.1f} MHz, {a.nx}x{a.ny} grid "
            f"{'2x2' if a.kernel == 2 else 'nearest-cell'} kernel, {wl.n_samples} samples, "
            f"gains every {wl.t_cal} samples (gamma {wl.gamma})")


def oracle_threads():
    """BLAS threads of this process (the in-process oracle legs)."""
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        return int(max([d.get("num_threads", 1) for d in info] or [1]))
    except Exception:
        return os.cpu_count() or 1


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# ---------------------------------------------------------------------------
# The oracle on the host cores: one worker process per core, one BLAS thread
# each, whole channels as tasks (channels are independent).  The pool is
# started before anything touches the GPU; its workers import numpy and the
# oracle only.
# ---------------------------------------------------------------------------

_POOL = None
_POOL_WORKERS = 0


def _pool_init():
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    try:
        import threadpoolctl
        threadpoolctl.threadpool_limits(1)
    except Exception:
        pass


def _pool_ready():
    from oracle import epic_oracle  # noqa: F401  (imported once per worker, outside the timed tasks)
    time.sleep(1.0)   # keeps every worker busy while the others start, so that all of them start now
    return os.getpid()


def start_oracle_pool(n_workers):
    """Start n_workers spawn-context worker processes and wait until each has
    imported the oracle."""
    global _POOL, _POOL_WORKERS
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    os.environ.update({k: "1" for k in keys})       # inherited by the workers before they load BLAS
    try:
        _POOL = ProcessPoolExecutor(n_workers, mp_context=mp.get_context("spawn"), initializer=_pool_init)
        pids = set(f.result() for f in [_POOL.submit(_pool_ready) for _ in range(n_workers)])
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    _POOL_WORKERS = n_workers
    print(f"# oracle pool: {n_workers} worker processes ({len(pids)} started), 1 BLAS thread each",
          file=sys.stderr, flush=True)


def _oracle_channel(wl, packed_ch, ch, pix):
    """Task: the FP64 loop on one channel; returns the image and last gains."""
    from oracle import epic_oracle as O
    pb = O.Problem.from_workload(wl)
    E = O.unpack(packed_ch, wl.array.efmt)
    if pix is None:
        r = O.run_channel(E, pb, ch, wl.g0[ch])
    else:
        pb.pix_lm = pix
        r = O.run_channel_multi(E, pb, ch, wl.g0[ch])
    return r["image"], r["gains"][-1]


def _oracle_gradient(wl, packed_ch, ch, M_ch):
    """Task: fixed-gain image and its gain gradient on one channel."""
    from oracle import epic_oracle as O
    a = wl.array
    cells = O.grid_cells(a.ant_xy, a.dx, a.dy, a.x0, a.y0, a.nx, a.ny, a.kernel)
    E = O.unpack(packed_ch, a.efmt)
    I = O.image_fixed_gains(E, wl.g0[ch], cells, a.nx, a.ny, float(a.n_ant))
    return O.image_gain_gradient(E, wl.g0[ch], cells, a.nx, a.ny, float(a.n_ant), 2 * (I - M_ch))


def pooled_oracle(tasks, budget_s):
    """Run (fn, args) tasks in waves of one task per worker until the budget
    is spent (at least one wave).  Returns (results, tasks done, wall s)."""
    out = []
    t0 = time.perf_counter()
    k = 0
    while k < len(tasks) and (k == 0 or time.perf_counter() - t0 < budget_s):
        wave = tasks[k:k + _POOL_WORKERS]
        futs = [_POOL.submit(fn, *args) for fn, args in wave]
        out.extend(f.result() for f in futs)
        k += len(wave)
    return out, k, time.perf_counter() - t0


def pool_record(value, sample):
    return {"value": value, "unit": "frames/s", "cores": _POOL_WORKERS, "kind": "oracle",
            "sample": sample, "parallelism": f"{_POOL_WORKERS} processes x 1 BLAS thread, whole channels per task",
            "cpu_model": cpu_model()}


def rel_err(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def gain_rel_err(got, ref):
    """Element-wise: the largest |g_gpu - g_oracle| / |g_oracle|."""
    return float(np.max(np.abs(got - ref) / np.abs(ref)))


def spread_channels(n_chan, n):
    """n channels spread over the band, then the rest in order."""
    first = sorted(set(int(round(i * (n_chan - 1) / max(1, n - 1))) for i in range(min(n, n_chan))))
    return first + [c for c in range(n_chan) if c not in first]


def cpu_baseline(wl, packed, budget_s, gpu_image=None, gpu_gains=None, extra_images=None, pix=None):
    """The FP64 oracle on whole channels of the same workload, one channel per
    worker process, in waves until the time budget is spent."""
    chans = spread_channels(wl.array.n_chan, _POOL_WORKERS)
    tasks = [(_oracle_channel, (wl, np.ascontiguousarray(packed[:, ch]), ch, pix)) for ch in chans]
    res, n_done, t_used = pooled_oracle(tasks, budget_s)
    done = chans[:n_done]
    results = [(c, {"image": im, "gains": g}) for c, (im, g) in zip(done, res)]
    frames = len(done) * wl.n_samples
    out = pool_record(frames / t_used, f"channels {sorted(done)} x all {wl.n_samples} samples ({frames} frames, "
                                       f"{t_used:.1f} s wall)")
    par = None
    if gpu_image is not None:
        par = {"channels": sorted(done),
               "image_rel_err": max(rel_err(gpu_image[c], r["image"]) for c, r in results),
               "gain_rel_err": max(gain_rel_err(gpu_gains[c], r["gains"]) for c, r in results)}
        for name, im in (extra_images or {}).items():
            par[f"{name}_image_rel_err"] = max(rel_err(im[c], r["image"]) for c, r in results)
    return out, par


def cpu_baseline_band(wl, packed, budget_s, band, gpu_prefix):
    """The FP64 oracle with gains shared over a band: the channels are
    coupled, so the sample is every channel over the first intervals (one
    interval timed first, then as many as the budget allows).  Parity: the
    GPU run over the same prefix of samples."""
    from oracle import epic_oracle as O
    pb = O.Problem.from_workload(wl)
    mode = {1: "mean", 2: "poly"}[band[2]]
    n_int = -(-wl.n_samples // wl.t_cal)

    def run(k):
        E = O.unpack(packed[:k * wl.t_cal], wl.array.efmt)
        t0 = time.perf_counter()
        r = O.run_band(E, pb, wl.g0, band[:2], mode)
        return r, time.perf_counter() - t0
    k = 1
    r, dt = run(1)
    if dt < budget_s / 2 and n_int > 1:
        k = int(min(n_int, max(2, budget_s // dt)))
        r, dt = run(k)
    frames = k * wl.t_cal * wl.array.n_chan
    out = {"value": frames / dt, "unit": "frames/s", "cores": oracle_threads(), "kind": "oracle",
           "sample": f"all {wl.array.n_chan} channels x the first {k} intervals ({frames} frames, {dt:.1f} s)"}
    im, gh = gpu_prefix(k * wl.t_cal)
    par = {"samples": k * wl.t_cal, "image_rel_err": max(rel_err(im[c], r["image"][c]) for c in range(im.shape[0])),
           "gain_rel_err": max(gain_rel_err(gh[n], r["gains"][n]) for n in range(gh.shape[0]))}
    return out, par


class Timer:
    """Times K steps of `step` after W warm-up steps, with the library's HIP
    event timers (recorded on the stream each kernel runs on) switched on for
    the timed steps only."""

    def __init__(self, plans):
        self.plans = plans

    def __call__(self, step, steps, warmup):
        import torch
        from paper_1603_02126_amd import lib
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        for p in self.plans:
            p.set_option(lib.OPT_TIMING, 1)
            p.timing()   # reset
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kt = {}
        for p in self.plans:
            for k, (ms, n) in p.timing().items():
                a, b = kt.get(k, (0.0, 0))
                kt[k] = (a + ms, b + n)
            p.set_option(lib.OPT_TIMING, 0)
        return elapsed, kt


def per_step(kt, kind, steps):
    ms, n = kt.get(kind, (0.0, 0))
    return {"ms_per_step": ms / steps, "launches_per_step": n / steps}


def base_record(args, metric_value, ms_step, dtype, config):
    return {
        "metric": "EPIC frames/s (grid+FFT+|E|^2+EPICal) vs plain FP32 path; % HBM roofline",
        "value": metric_value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic (seeded generator: random layout, power-law sky, complex-Gaussian sources and noise, "
                "quantised)",
        "config": config,
    }


def copy_reference(dev):
    import torch
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("# copy reference: 268435456 bytes read, 268435456 bytes written", file=sys.stderr, flush=True)


def new_plan(specs_wls, opts=None, pix=None, band=None):
    """A plan over the arrays of `specs_wls`; with `pix` the first array's
    EPICal taps those pixels instead of its calibrator alone; with
    band = (b0, b1, mode) its channels b0..b1-1 share gains."""
    from paper_1603_02126_amd import lib
    plan = lib.Plan([w.array for w in specs_wls])
    for i, w in enumerate(specs_wls):
        if i == 0 and pix is not None:
            plan.set_model_pixels(i, w.model_lmS, pix, w.gamma, w.t_cal)
        else:
            plan.set_model(i, w.model_lmS, w.cal_lm, w.gamma, w.t_cal)
    if band is not None:
        plan.set_band(0, *band)
    for k, v in (opts or {}).items():
        plan.set_option(k, v)
    return plan


def bench_single(args, dev):
    """One array through epic_run (lwa, hera, tiny)."""
    import torch
    from paper_1603_02126_amd import lib
    wl = workload(args.workload)
    a = wl.array
    print(f"# generating {describe(wl)}", file=sys.stderr, flush=True)
    tg = time.perf_counter()
    packed = synth.make_efield(wl, threads=min(16, os.cpu_count() or 1))
    print(f"# generated {packed.nbytes / 1e6:.1f} MB in {time.perf_counter() - tg:.1f} s", file=sys.stderr,
          flush=True)

    pix = None
    if args.pixels > 1:
        # several tapped pixels: the brightest model sources (the calibrator first)
        order = np.argsort(-wl.model_lmS[:, 2], kind="stable")[:args.pixels]
        pix = wl.model_lmS[order, :2]
    # lwa_band: every channel shares the band's mean solution (Sec. 5)
    band = (0, a.n_chan, lib.BAND_MEAN) if wl.name == "lwa_band" else None
    plan = new_plan([wl], {lib.OPT_SPLITS: args.splits} if args.splits else None, pix, band)
    e = torch.from_numpy(packed).to(dev)
    g0 = torch.from_numpy(wl.g0).to(dev)
    g = torch.empty_like(g0)
    img = torch.zeros((a.n_chan, a.ny, a.nx), dtype=torch.float32, device=dev)

    def stepper(pl, out_img):
        def step():
            g.copy_(g0)
            pl.run([e], wl.n_samples, [g], [out_img])
        return step

    dt, tim = Timer([plan])(stepper(plan, img), args.steps, args.warmup)
    gains_plain = g.cpu().numpy()
    print(f"# timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    frames = a.n_chan * wl.n_samples
    forms = {}
    # the fused run (one launch for solve and imaging, the default where the
    # plan allows it) times as imaging only; the separate launches give each
    # kernel's own duration, which the roofline and the kernel table use
    fused = tim[lib.TIMER_SOLVE][1] == 0 and tim[lib.TIMER_IMAGE][1] > 0
    tim_k, dt_sep = tim, None
    if fused:
        plan_s = new_plan([wl], {lib.OPT_OVERLAP: 0, **({lib.OPT_SPLITS: args.splits} if args.splits else {})},
                          pix, band)
        img_s = torch.zeros_like(img)
        dt_sep, tim_k = Timer([plan_s])(stepper(plan_s, img_s), args.steps, args.warmup)
        forms["separate_launches"] = {
            "ms_per_step": dt_sep / args.steps * 1e3, "frames_per_s": frames / (dt_sep / args.steps),
            "speedup_of_fused_run": dt_sep / dt,
            "gains_equal_fused": bool(np.array_equal(g.cpu().numpy(), gains_plain)),
            "max_rel_diff_vs_fused": rel_err(img_s.cpu().numpy(), img.cpu().numpy())}
        plan_s.close()
    if not args.no_forms:
        for name, tr, prods in DFT_FORMS:
            if not (a.nx in (32, 64) or (a.nx in (128, 256) and a.n_ant <= 512)):
                forms[name] = {"supported": False, "reason": "the DFT-GEMM form covers arrays of at most 512 antennas"}
                continue
            # form 1: split-precision DFT-GEMM on the matrix cores, same workload
            plan_d = new_plan([wl], {lib.OPT_TRANSFORM: tr}, pix, band)
            img_d = torch.zeros_like(img)
            dt_d, tim_d = Timer([plan_d])(stepper(plan_d, img_d), args.steps, args.warmup)
            ms_img_d = tim_d[lib.TIMER_IMAGE][0] / max(1, tim_d[lib.TIMER_IMAGE][1])
            mf = dft_mfma_flops_per_frame(a.nx, prods) * frames / (ms_img_d * 1e-3) / 1e12
            forms[name] = {
                "ms_per_step": dt_d / args.steps * 1e3, "frames_per_s": frames / (dt_d / args.steps),
                "speedup_vs_plain": dt / dt_d, "imaging_kernel_ms": ms_img_d,
                "mfma": {"achieved": mf, "peak": PEAK_FP16_MFMA_TFLOPS,
                         "unit": "TFLOP/s (executed, " + ("fp16" if tr == 2 else "bf16") + ")",
                         "frac": mf / PEAK_FP16_MFMA_TFLOPS},
                "max_rel_diff_vs_plain": rel_err(img_d.cpu().numpy(), img.cpu().numpy()),
                "gains": "identical to the plain path (the FP64 solve does not depend on the transform)",
                "_image": img_d}
            plan_d.close()
    # form 2: batched launches captured in a hipGraph, after autotuning
    if not args.no_forms and band is not None:
        forms["batched_graph_autotuned"] = {"supported": False,
                                            "reason": "gains shared over a band run in the per-array form"}
    elif not args.no_forms:
        plan_g = new_plan([wl], None, pix)
        tuning = plan_g.autotune([e], wl.n_samples)
        plan_g.set_option(lib.OPT_BATCH, 1)
        plan_g.set_option(lib.OPT_GRAPH, 1)
        img_g = torch.zeros_like(img)
        dt_g, tim_g = Timer([plan_g])(stepper(plan_g, img_g), args.steps, args.warmup)
        forms["batched_graph_autotuned"] = {
            "ms_per_step": dt_g / args.steps * 1e3, "frames_per_s": frames / (dt_g / args.steps),
            "speedup_vs_plain": dt / dt_g,
            "tuning": {"transform": TRANSFORM_NAMES[tuning[0][0]], "splits": tuning[0][1],
                       "grid_batch": tuning[0][2]},
            "graph_replay_ms": tim_g[lib.TIMER_GRAPH][0] / max(1, tim_g[lib.TIMER_GRAPH][1]),
            "max_rel_diff_vs_plain": rel_err(img_g.cpu().numpy(), img.cpu().numpy()),
            "_image": img_g}
        plan_g.close()
    if args.copy_calib:
        copy_reference(dev)

    ms_step = dt / args.steps * 1e3
    value = frames / (dt / args.steps)
    k2 = 1 if a.kernel == 1 else 4
    img_ms, img_n = tim_k[lib.TIMER_IMAGE]
    avg_img_ms = img_ms / max(1, img_n)
    flops_launch = imaging_flops_per_frame(a.nx, a.n_ant, k2) * frames
    achieved = flops_launch / (avg_img_ms * 1e-3) / 1e12
    bpe = synth.FMT_BYTES[a.efmt]
    bytes_launch = imaging_bytes_per_frame(a.n_ant, bpe, a.nx, wl.n_samples, wl.t_cal) * frames
    traffic = measured_traffic(args.workload) if not args.splits else None
    kernels = {"imaging": per_step(tim_k, lib.TIMER_IMAGE, args.steps),
               "calibration_solve": per_step(tim_k, lib.TIMER_SOLVE, args.steps),
               "image_reduce": per_step(tim_k, lib.TIMER_REDUCE, args.steps)}
    if fused:
        kernels = {"fused_solve_and_imaging": per_step(tim, lib.TIMER_IMAGE, args.steps),
                   "image_reduce": per_step(tim, lib.TIMER_REDUCE, args.steps),
                   "separate_launches": kernels}

    cpu, parity = None, None
    if args.cpu_budget > 0 and band is not None:
        print("# timing the FP64 oracle on the host (all channels, first intervals)", file=sys.stderr, flush=True)

        def gpu_prefix(n_s):
            gh = torch.zeros((-(-n_s // wl.t_cal) + 1, a.n_chan, a.n_ant), dtype=torch.complex128, device=dev)
            im = torch.zeros_like(img)
            g.copy_(g0)
            plan.run([e], n_s, [g], [im], gain_hist=[gh])
            torch.cuda.synchronize()
            return im.cpu().numpy(), gh.cpu().numpy()
        cpu, parity = cpu_baseline_band(wl, packed, args.cpu_budget, band, gpu_prefix)
    elif args.cpu_budget > 0:
        print("# timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        extra = {k: v["_image"].cpu().numpy() for k, v in forms.items() if "_image" in v}
        cpu, parity = cpu_baseline(wl, packed, args.cpu_budget, img.cpu().numpy(), gains_plain, extra, pix)
    for v in forms.values():
        v.pop("_image", None)

    engine = "k_image (calibrate+grid+FFT+|X|^2)" if a.nx <= 64 else \
        f"k_image_cls<{a.nx // 64}> (calibrate+grid by residue class+64-point FFTs+|X|^2)"
    if fused:
        engine += "; timed in the separate-launch form of the same plan"
    path = ("FP32 FFT, fused solve + imaging launch (k_run_fused)" if fused
            else "FP32 FFT, separate solve and imaging launches")
    out = base_record(args, value, ms_step, "f32", {
        "workload": describe(wl), "frames_per_step": frames, "n_ant": a.n_ant, "n_chan": a.n_chan,
        "grid": [a.ny, a.nx], "n_samples": wl.n_samples, "t_cal": wl.t_cal, "efmt": synth.FMT_NAMES[a.efmt],
        "path": path, "parallelism": "1 GPU", "tapped_pixels": args.pixels,
        "band": None if band is None else {"channels": [band[0], band[1]], "mode": "mean"}})
    out.update({
        "msamples_per_s": value * a.n_ant / 1e6,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "kernel": engine, "avg_launch_ms": avg_img_ms,
                     "flops_per_frame": imaging_flops_per_frame(a.nx, a.n_ant, k2),
                     "hbm_bytes_per_frame": bytes_launch / frames,
                     "hbm_frac": bytes_launch / (avg_img_ms * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "sq_counters": measured_sq(args.workload) if not args.splits else None,
                     "fused_launch_ms": (tim[lib.TIMER_IMAGE][0] / max(1, tim[lib.TIMER_IMAGE][1])
                                         if fused else None)},
        "kernels": kernels,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "forms": forms,
    })
    plan.close()
    return out


def bench_snapshot(args, dev):
    """Snapshot images (epic_run_snapshots): one image per window of t_acc
    samples instead of one per run.  At t_acc = 1 every frame writes its own
    16 KiB image, so HBM writes join the FP32 work as a bound."""
    import torch
    from paper_1603_02126_amd import lib
    from oracle import epic_oracle as O
    wl = workload(args.workload)
    a = wl.array
    t_acc = args.snapshot
    T = wl.n_samples
    n_win = -(-T // t_acc)
    print(f"# generating {describe(wl)}; snapshots every {t_acc} samples", file=sys.stderr, flush=True)
    packed = synth.make_efield(wl, threads=min(16, os.cpu_count() or 1))
    plan = new_plan([wl])
    e = torch.from_numpy(packed).to(dev)
    g0 = torch.from_numpy(wl.g0).to(dev)
    g = torch.empty_like(g0)
    imgs = torch.empty((n_win, a.n_chan, a.ny, a.nx), dtype=torch.float32, device=dev)

    def step():
        g.copy_(g0)
        plan.run_snapshots(0, e, T, t_acc, g, imgs)
    dt, tim = Timer([plan])(step, args.steps, args.warmup)
    print(f"# timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    frames = a.n_chan * T
    ms_step = dt / args.steps * 1e3
    img_ms, img_n = tim[lib.TIMER_IMAGE]
    avg_img_ms = img_ms / max(1, img_n)
    k2 = 1 if a.kernel == 1 else 4
    bpe = synth.FMT_BYTES[a.efmt]
    flops_launch = imaging_flops_per_frame(a.nx, a.n_ant, k2) * frames
    bytes_frame = a.n_ant * bpe + 8.0 * a.n_ant / wl.t_cal + 4.0 * a.nx * a.ny / t_acc
    bytes_launch = bytes_frame * frames
    tflops = flops_launch / (avg_img_ms * 1e-3) / 1e12
    gbs = bytes_launch / (avg_img_ms * 1e-3) / 1e9
    hbm_bound = bytes_launch / (PEAK_HBM_GBS * 1e9) > flops_launch / (PEAK_FP32_VECTOR_TFLOPS * 1e12)
    roof = ({"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS}
            if hbm_bound else
            {"bound": "alu", "achieved": tflops, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
             "frac": tflops / PEAK_FP32_VECTOR_TFLOPS})
    roof.update({"traffic": measured_traffic(f"{args.workload}_snapshot{t_acc}"),
                 "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                 "algorithmic_bytes_per_launch": bytes_launch, "hbm_bytes_per_frame": bytes_frame,
                 "flops_per_frame": imaging_flops_per_frame(a.nx, a.n_ant, k2),
                 "hbm_frac": gbs / PEAK_HBM_GBS, "alu_frac": tflops / PEAK_FP32_VECTOR_TFLOPS,
                 "kernel": "k_image_snap / k_image_pair_snap (calibrate+grid+FFT+|X|^2, one image per window)",
                 "avg_launch_ms": avg_img_ms})
    if args.copy_calib:
        copy_reference(dev)
    cpu, parity = None, None
    if args.cpu_budget > 0:
        print("# timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        pb = O.Problem.from_workload(wl)
        done, errs, gerrs, t_used = [], [], [], 0.0
        ch = 0
        gains = g.cpu().numpy()
        while ch < a.n_chan and (not done or t_used < args.cpu_budget):
            E = O.unpack(packed[:, ch], a.efmt)
            t0 = time.perf_counter()
            r = O.run_channel_snapshots(E, pb, ch, wl.g0[ch], t_acc)
            t_used += time.perf_counter() - t0
            got = imgs[:, ch].cpu().numpy()
            errs.append(float((np.abs(got - r["images"]).reshape(n_win, -1).max(1) /
                               np.abs(r["images"]).reshape(n_win, -1).max(1)).max()))
            gerrs.append(gain_rel_err(gains[ch], r["gains"][-1]))
            done.append(ch)
            del r
            ch += max(1, a.n_chan // 7)
        fr = len(done) * T
        cpu = {"value": fr / t_used, "unit": "frames/s", "cores": oracle_threads(), "kind": "oracle",
               "sample": f"channels {done} x all {T} samples ({fr} frames, {t_used:.1f} s)"}
        parity = {"channels": done, "max_window_image_rel_err": max(errs), "gain_rel_err": max(gerrs)}
    out = base_record(args, frames / (dt / args.steps), ms_step, "f32", {
        "workload": describe(wl) + f"; snapshot images every {t_acc} samples ({n_win} per channel)",
        "frames_per_step": frames, "n_ant": a.n_ant, "n_chan": a.n_chan, "grid": [a.ny, a.nx], "n_samples": T,
        "t_cal": wl.t_cal, "t_acc": t_acc, "efmt": synth.FMT_NAMES[a.efmt], "path": "snapshot images",
        "parallelism": "1 GPU"})
    out.update({"roofline": roof,
                "kernels": {"imaging": per_step(tim, lib.TIMER_IMAGE, args.steps),
                            "calibration_solve": per_step(tim, lib.TIMER_SOLVE, args.steps)},
                "image_bytes_per_step": 4.0 * a.nx * a.ny * n_win * a.n_chan,
                "cpu_baseline": cpu, "parity_vs_oracle": parity})
    plan.close()
    return out


def bench_uneven(args, dev):
    """Eight arrays of uneven size: per-array launches (plain) against the
    batched persistent form in a hipGraph after autotuning."""
    import torch
    from paper_1603_02126_amd import lib
    wls = workload("uneven")
    print(f"# generating {len(wls)} arrays", file=sys.stderr, flush=True)
    tg = time.perf_counter()
    packs = [synth.make_efield(w, threads=min(16, os.cpu_count() or 1)) for w in wls]
    print(f"# generated {sum(p.nbytes for p in packs) / 1e6:.1f} MB in {time.perf_counter() - tg:.1f} s",
          file=sys.stderr, flush=True)
    T = wls[0].n_samples
    es = [torch.from_numpy(p).to(dev) for p in packs]
    g0s = [torch.from_numpy(w.g0).to(dev) for w in wls]
    gs = [torch.empty_like(g) for g in g0s]

    def images():
        return [torch.zeros((w.array.n_chan, w.array.ny, w.array.nx), dtype=torch.float32, device=dev) for w in wls]

    def stepper(pl, imgs):
        def step():
            for g, g0 in zip(gs, g0s):
                g.copy_(g0)
            pl.run(es, T, gs, imgs)
        return step

    plan = new_plan(wls, {lib.OPT_BATCH: 2, lib.OPT_OVERLAP: 0} if args.per_array else None)
    imgs = images()
    dt, tim = Timer([plan])(stepper(plan, imgs), args.steps, args.warmup)
    gains_plain = [g.cpu().numpy() for g in gs]
    print(f"# timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    frames = sum(w.array.n_chan for w in wls) * T
    flops_step = sum(imaging_flops_per_frame(w.array.nx, w.array.n_ant, 4) * w.array.n_chan * T for w in wls)
    forms = {}
    # per-array separate launches (solve, imaging, reduction of each array):
    # the imaging kernels' own durations for the roofline
    fused = tim[lib.TIMER_SOLVE][1] == 0
    tim_k, dt_k = tim, dt
    if fused:
        plan_s = new_plan(wls, {lib.OPT_BATCH: 2, lib.OPT_OVERLAP: 0})
        imgs_s = images()
        dt_k, tim_k = Timer([plan_s])(stepper(plan_s, imgs_s), args.steps, args.warmup)
        forms["separate_per_array_launches"] = {
            "ms_per_step": dt_k / args.steps * 1e3, "frames_per_s": frames / (dt_k / args.steps),
            "speedup_of_fused_run": dt_k / dt,
            "gains_equal_fused": all(np.array_equal(g.cpu().numpy(), gp) for g, gp in zip(gs, gains_plain)),
            "max_rel_diff_vs_fused": max(rel_err(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(imgs_s, imgs))}
        plan_s.close()
    if not args.no_forms:
        plan_g = new_plan(wls)
        tuning = plan_g.autotune(es, T)
        plan_g.set_option(lib.OPT_BATCH, 1)
        plan_g.set_option(lib.OPT_GRAPH, 1)
        imgs_g = images()
        dt_g, tim_g = Timer([plan_g])(stepper(plan_g, imgs_g), args.steps, args.warmup)
        forms["batched_graph_autotuned"] = {
            "ms_per_step": dt_g / args.steps * 1e3, "frames_per_s": frames / (dt_g / args.steps),
            "speedup_vs_plain": dt / dt_g,
            "tuning": [{"grid": w.array.nx, "n_ant": w.array.n_ant,
                        "transform": TRANSFORM_NAMES[t[0]], "splits": t[1], "grid_batch": t[2]}
                       for w, t in zip(wls, tuning)],
            "graph_replay_ms": tim_g[lib.TIMER_GRAPH][0] / max(1, tim_g[lib.TIMER_GRAPH][1]),
            "max_rel_diff_vs_plain": max(rel_err(x.cpu().numpy(), y.cpu().numpy()) for x, y in zip(imgs_g, imgs)),
            "_images": imgs_g}
        plan_g.close()
    if args.copy_calib:
        copy_reference(dev)
    img_ms = tim_k[lib.TIMER_IMAGE][0] / args.steps
    achieved = flops_step / (img_ms * 1e-3) / 1e12
    bytes_step = sum(imaging_bytes_per_frame(w.array.n_ant, synth.FMT_BYTES[w.array.efmt], w.array.nx, T, w.t_cal)
                     * w.array.n_chan * T for w in wls)

    cpu, parity = None, None
    if args.cpu_budget > 0:
        # the oracle on whole (array, channel) tasks, every array in each round of
        # channels (the workload's own mix), more channels while the budget lasts
        print("# timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        chans = spread_channels(wls[0].array.n_chan, 64)
        tasks, keys = [], []
        for ch in chans:
            for i, (w, p) in enumerate(zip(wls, packs)):
                tasks.append((_oracle_channel, (w, np.ascontiguousarray(p[:, ch]), ch, None)))
                keys.append((i, ch))
        res, n_done, t_used = pooled_oracle(tasks, args.cpu_budget)
        ie, ge, ieg = [], [], []
        for (i, ch), (im, gl) in zip(keys[:n_done], res):
            ie.append(rel_err(imgs[i][ch].cpu().numpy(), im))
            ge.append(gain_rel_err(gains_plain[i][ch], gl))
            if "batched_graph_autotuned" in forms:
                ieg.append(rel_err(forms["batched_graph_autotuned"]["_images"][i][ch].cpu().numpy(), im))
        fr = n_done * T
        done = sorted(set(k for _, k in keys[:n_done]))
        cpu = pool_record(fr / t_used, f"{n_done} (array, channel) tasks: channels {done} of the {len(wls)} "
                                       f"arrays x all {T} samples ({fr} array-frames, {t_used:.1f} s wall)")
        parity = {"tasks": [list(k) for k in keys[:n_done]], "image_rel_err": max(ie), "gain_rel_err": max(ge)}
        if ieg:
            parity["batched_graph_autotuned_image_rel_err"] = max(ieg)
    for v in forms.values():
        v.pop("_images", None)

    ms_step = dt / args.steps * 1e3
    value = frames / (dt / args.steps)
    out = base_record(args, value, ms_step, "f32", {
        "workload": "uneven: 8 arrays, antennas " + ",".join(str(w.array.n_ant) for w in wls) + ", grids " +
                    ",".join(f"{w.array.nx}^2" for w in wls) + f", ci8, {wls[0].array.n_chan} channels each, "
                    f"{T} samples, gains every {wls[0].t_cal}",
        "frames_per_step": frames,
        "path": ("FP32 FFT, one fused solve + imaging launch for all arrays (k_run_fused)" if fused
                 else "FP32 FFT, one launch per array per stage" if tim[lib.TIMER_IMAGE][1] >= len(wls) * args.steps
                 else "FP32 FFT, batched: one persistent imaging launch for all arrays (k_image_batch)"),
        "parallelism": "1 GPU"})
    out.update({
        "msamples_per_s": sum(w.array.n_ant * w.array.n_chan for w in wls) * T / (dt / args.steps) / 1e6,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                     "kernel": "imaging kernels of all arrays (FFT, residue-class engines)" +
                               (", timed as separate per-array launches" if fused else ""),
                     "imaging_ms_per_step": img_ms,
                     "algorithmic_bytes_per_step": bytes_step,
                     "hbm_frac": bytes_step / (img_ms * 1e-3) / 1e9 / PEAK_HBM_GBS},
        "kernels": ({"fused_solve_and_imaging": per_step(tim, lib.TIMER_IMAGE, args.steps),
                     "image_reduce": per_step(tim, lib.TIMER_REDUCE, args.steps),
                     "separate_per_array_launches": {
                         "imaging": per_step(tim_k, lib.TIMER_IMAGE, args.steps),
                         "calibration_solve": per_step(tim_k, lib.TIMER_SOLVE, args.steps),
                         "image_reduce": per_step(tim_k, lib.TIMER_REDUCE, args.steps)}} if fused else
                    {"imaging": per_step(tim, lib.TIMER_IMAGE, args.steps),
                     "calibration_solve": per_step(tim, lib.TIMER_SOLVE, args.steps),
                     "image_reduce": per_step(tim, lib.TIMER_REDUCE, args.steps)}),
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "forms": forms,
    })
    plan.close()
    return out


def bench_diff(args, dev):
    """Differentiable form: fixed-gain image (forward) and its hand-written
    adjoint (backward) for L = sum (I - M)^2."""
    import torch
    from paper_1603_02126_amd import lib
    wl = workload("diff")
    a = wl.array
    print(f"# generating {describe(wl)}", file=sys.stderr, flush=True)
    packed = synth.make_efield(wl, threads=min(16, os.cpu_count() or 1))
    plan = new_plan([wl], {lib.OPT_SPLITS: args.splits} if args.splits else None)
    e = torch.from_numpy(packed).to(dev)
    g = torch.from_numpy(wl.g0).to(dev)
    # loss target: the expected image of the 50 brightest model sources plus the
    # noise floor, made by the library's fixed-gain imaging of a tone sky whose
    # time average is that expectation (built before timing)
    src50, sigma_d = synth.loss_target_sky(wl)
    tones = synth.tone_efield(a.ant_xy, a.freq_hz, src50, sigma_d)
    with lib.Plan([synth.dataclasses.replace(a, efmt=synth.FMT_CF32)]) as tone_plan:
        ones = torch.ones((a.n_chan, a.n_ant), dtype=torch.complex128, device=dev)
        M = tone_plan.image(0, torch.from_numpy(tones).to(dev), tones.shape[0], ones).double()
    torch.cuda.synchronize()
    M_np = M.cpu().numpy()
    img = torch.empty((a.n_chan, a.ny, a.nx), dtype=torch.float32, device=dev)
    grad = torch.empty((a.n_chan, a.n_ant), dtype=torch.complex128, device=dev)
    R = torch.empty_like(img)

    def step():
        plan.image(0, e, wl.n_samples, g, out=img)
        R.copy_(2.0 * (img.double() - M))   # dL/dI of the loss, then the adjoint
        plan.image_adjoint(0, e, wl.n_samples, g, R, out=grad)

    dt, tim = Timer([plan])(step, args.steps, args.warmup)
    frames = a.n_chan * wl.n_samples
    k2 = 4
    adj_ms = tim[lib.TIMER_ADJOINT][0] / max(1, tim[lib.TIMER_ADJOINT][1])
    fwd_ms = tim[lib.TIMER_IMAGE][0] / max(1, tim[lib.TIMER_IMAGE][1])
    achieved = adjoint_flops_per_frame(a.nx, a.n_ant, k2) * frames / (adj_ms * 1e-3) / 1e12
    cpu, parity = None, None
    if args.cpu_budget > 0:
        print("# timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        got = grad.cpu().numpy()
        chans = spread_channels(a.n_chan, _POOL_WORKERS)
        tasks = [(_oracle_gradient, (wl, np.ascontiguousarray(packed[:, ch]), ch, M_np[ch])) for ch in chans]
        res, n_done, t_used = pooled_oracle(tasks, args.cpu_budget)
        done = chans[:n_done]
        errs = [float(np.abs(got[ch] - ref).max() / np.abs(ref).max()) for ch, ref in zip(done, res)]
        fr = len(done) * wl.n_samples
        cpu = pool_record(fr / t_used, f"forward + gradient, channels {sorted(done)} x all {wl.n_samples} samples "
                                       f"({fr} frames, {t_used:.1f} s wall)")
        parity = {"channels": sorted(done), "gradient_rel_err": max(errs)}
    out = base_record(args, frames / (dt / args.steps), dt / args.steps * 1e3, "f32", {
        "workload": describe(wl) + "; loss sum (I - M)^2, M the model image of the 50 brightest sources "
                    "plus the noise floor",
        "frames_per_step": frames, "path": "epic_image + epic_image_adjoint (forward + backward)",
        "parallelism": "1 GPU"})
    out.update({
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                     "kernel": "k_adjoint (recompute X, R*X, conjugate FFT, degrid, conj(E) product)",
                     "avg_launch_ms": adj_ms,
                     "flops_per_frame": adjoint_flops_per_frame(a.nx, a.n_ant, k2)},
        "kernels": {"forward_imaging": {"ms_per_launch": fwd_ms}, "adjoint": {"ms_per_launch": adj_ms}},
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
    })
    plan.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lwa", choices=["lwa", "lwa_band", "hera", "tiny", "uneven", "diff"])
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--splits", type=int, default=0)
    ap.add_argument("--no-forms", action="store_true", help="time only the plain FP32 path")
    ap.add_argument("--pixels", type=int, default=1,
                    help="tapped pixels of EPICal (lwa/hera/tiny; > 1: calibrator plus brightest sources)")
    ap.add_argument("--snapshot", type=int, default=0,
                    help="t_acc > 0: time epic_run_snapshots (one image per t_acc samples) on lwa/tiny")
    ap.add_argument("--per-array", action="store_true",
                    help="uneven: time one launch per array and stage (no batching, no fused run)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="after timing, run one plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards by channel "
              "with no exchange, so N GPUs would each run this workload's channel share.", file=sys.stderr)
        sys.exit(2)

    if args.cpu_budget > 0 and args.snapshot == 0 and args.workload != "lwa_band":
        # before anything touches the GPU: the machine's CPU share is 16 cores
        start_oracle_pool(max(1, min(16, len(os.sched_getaffinity(0)))))

    import torch
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.snapshot > 0:
        out = bench_snapshot(args, dev)
    elif args.workload == "uneven":
        out = bench_uneven(args, dev)
    elif args.workload == "diff":
        out = bench_diff(args, dev)
    else:
        out = bench_single(args, dev)
    if _POOL is not None:
        _POOL.shutdown()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
