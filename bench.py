#!/usr/bin/env python3
"""Benchmark of the calibrated EPIC loop on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lwa]

A step is one pass of the whole hot path over one batch of synthetic input:
EPICal calibration solve (tap, correlation, damped FP64 update every t_cal
samples) followed by calibrate + grid + 2D FFT + |X|^2 accumulation of every
(channel, sample) frame, as epic_run does it.  The default workload is the
LWA-station shape: 256 antennas, 4+4-bit E-fields, 128 channels, 64x64 grid
with the 2x2 kernel, 10,000 samples, gains updated every 100 samples.  The
E-field stream is resident in HBM before timing starts; each step restarts
from the same initial gains.

Prints one JSON line (value = frames/s, frame = one channel x one sample),
with the roofline of the dominant kernel measured by HIP events on the
stream it runs on, and the FP64 oracle timed on the host cores on a bounded
sample of the same workload.
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
PEAK_FP16_MFMA_TFLOPS = 2500.0    # MI355X published dense FP16 matrix peak
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the imaging kernel on the LWA-shaped workload, from two
# rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE in KiB per dispatch), each scaled by
# what the same counter reads for a plain 256 MiB device copy (FETCH x2.000,
# WRITE x1.000).  Valid only for the kernel sources they were taken on: any change
# to those files makes the figure stale and it is reported as null.
TRAFFIC_SOURCES = ("k_image.hip", "image_fft.h", "engine.h", "fft_reg.h", "epic_internal.h", "epic_api.hip")
TRAFFIC_MEASURED = {
    "lwa": {"sources_sha256": "fe6ad469aaafb7ebd33308c5423e77e706396bb934be2c334bef7b68d2e8308f",
            "fetch_kib": 174255.0, "fetch_scale": 2.000, "write_kib": 32768.0, "write_scale": 1.000},
}


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


def dft_mfma_flops_per_frame(n):
    """Executed matrix-core flops of the split-precision DFT-GEMM per frame:
    two complex N x N x N products, four real GEMMs each, three split terms."""
    return 2 * 4 * 3 * 2 * n ** 3


def imaging_flops_per_frame(n, na, k2):
    """Algorithmic flops of one frame in the imaging kernel: radix-2 FFT count
    5 Ng log2 Ng, calibration 6 per antenna, gridding 4 per kernel cell per
    antenna, |X|^2 accumulation 4 per pixel."""
    ng = n * n
    return 5 * ng * math.log2(ng) + na * (6 + 4 * k2) + 4 * ng


def imaging_bytes_per_frame(na, bpe, n, n_samples, t_cal):
    """Algorithmic HBM bytes of one frame: the packed E-fields once, u once per
    interval per antenna, the image written once per run."""
    return na * bpe + 8.0 * na / t_cal + 4.0 * n * n / n_samples


def workload(name):
    if name == "lwa":
        return synth.config_lwa()
    if name == "tiny":
        return synth.config_tiny()
    if name == "diff":
        return synth.config_diff()
    raise SystemExit(f"unknown workload {name}")


def describe(wl):
    a = wl.array
    fmt = synth.FMT_NAMES[a.efmt]
    return (f"{wl.name}: {a.n_ant} antennas {fmt}, {a.n_chan} channels "
            f"{a.freq_hz[0] / 1e6:.1f}-{a.freq_hz[-1] / 1e6:.1f} MHz, {a.nx}x{a.ny} grid "
            f"{'2x2' if a.kernel == 2 else 'nearest-cell'} kernel, {wl.n_samples} samples, "
            f"gains every {wl.t_cal} samples (gamma {wl.gamma})")


def cpu_baseline(wl, packed, budget_s, gpu_image=None, gpu_gains=None, extra_images=None):
    """The FP64 oracle on whole channels of the same workload until the time
    budget is spent (at least one channel)."""
    from oracle import epic_oracle as O
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([d.get("num_threads", 1) for d in info] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    pb = O.Problem.from_workload(wl)
    E_all = packed
    done, t_used = [], 0.0
    results = []
    ch = 0
    t0 = time.perf_counter()
    while ch < wl.array.n_chan and (not done or t_used < budget_s):
        E = O.unpack(E_all[:, ch], wl.array.efmt)
        r = O.run_channel(E, pb, ch, wl.g0[ch])
        results.append((ch, r))
        done.append(ch)
        t_used = time.perf_counter() - t0
        ch += max(1, wl.array.n_chan // 7)
    frames = len(done) * wl.n_samples
    out = {"value": frames / t_used, "unit": "frames/s", "cores": int(threads), "kind": "oracle",
           "sample": f"channels {done} x all {wl.n_samples} samples ({frames} frames, {t_used:.1f} s)"}
    if gpu_image is not None:
        ie, ge = [], []
        for c, r in results:
            ref = r["image"]
            ie.append(float(np.abs(gpu_image[c] - ref).max() / np.abs(ref).max()))
            gr = r["gains"][-1]
            ge.append(float(np.max(np.abs(gpu_gains[c] - gr)) / np.sqrt(np.mean(np.abs(gr) ** 2))))
        out_par = {"channels": done, "image_rel_err": max(ie), "gain_rel_err": max(ge)}
        for name, im in (extra_images or {}).items():
            out_par[f"{name}_image_rel_err"] = max(float(np.abs(im[c] - r["image"]).max() / np.abs(r["image"]).max())
                                                   for c, r in results)
    else:
        out_par = None
    return out, out_par


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lwa")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle time (0 = skip)")
    ap.add_argument("--splits", type=int, default=0)
    ap.add_argument("--no-forms", action="store_true", help="time only the plain FP32 path")
    ap.add_argument("--copy-calib", action="store_true",
                    help="after timing, run one plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards by channel "
              "with no exchange, so N GPUs would each run this workload's channel share.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1603_02126_amd import lib

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    wl = workload(args.workload)
    a = wl.array
    print(f"# generating {describe(wl)}", file=sys.stderr, flush=True)
    tg = time.perf_counter()
    packed = synth.make_efield(wl, threads=min(16, os.cpu_count() or 1))
    print(f"# generated {packed.nbytes / 1e6:.1f} MB in {time.perf_counter() - tg:.1f} s", file=sys.stderr,
          flush=True)

    plan = lib.Plan([a])
    plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
    if args.splits:
        plan.set_option(lib.OPT_SPLITS, args.splits)
    e = torch.from_numpy(packed).to(dev)
    g0 = torch.from_numpy(wl.g0).to(dev)
    g = torch.empty_like(g0)
    img = torch.zeros((a.n_chan, a.ny, a.nx), dtype=torch.float32, device=dev)

    def timed_steps(pl, out_img, steps, warmup):
        def step():
            g.copy_(g0)
            pl.run([e], wl.n_samples, [g], [out_img])
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        pl.set_option(lib.OPT_TIMING, 1)
        pl.timing()   # reset
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        kt = pl.timing()
        pl.set_option(lib.OPT_TIMING, 0)
        return elapsed, kt

    dt, tim = timed_steps(plan, img, args.steps, args.warmup)
    print(f"# timed {args.steps} steps in {dt:.3f} s", file=sys.stderr, flush=True)
    forms = {}
    if not args.no_forms and a.nx in (32, 64):
        # form 1: split-precision DFT-GEMM on the matrix cores, same workload
        plan_d = lib.Plan([a])
        plan_d.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        plan_d.set_option(lib.OPT_TRANSFORM, 2)
        img_d = torch.zeros_like(img)
        dt_d, tim_d = timed_steps(plan_d, img_d, args.steps, args.warmup)
        ms_img_d = tim_d[lib.TIMER_IMAGE][0] / max(1, tim_d[lib.TIMER_IMAGE][1])
        mf = dft_mfma_flops_per_frame(a.nx) * a.n_chan * wl.n_samples / (ms_img_d * 1e-3) / 1e12
        forms["dft_gemm_fp16_split"] = {
            "ms_per_step": dt_d / args.steps * 1e3, "frames_per_s": a.n_chan * wl.n_samples / (dt_d / args.steps),
            "speedup_vs_plain": dt / dt_d, "imaging_kernel_ms": ms_img_d,
            "mfma": {"achieved": mf, "peak": PEAK_FP16_MFMA_TFLOPS, "unit": "TFLOP/s (executed, fp16)",
                     "frac": mf / PEAK_FP16_MFMA_TFLOPS},
            "_image": img_d}
        plan_d.close()
    if not args.no_forms:
        # form 2: batched launches captured in a hipGraph, after autotuning
        plan_g = lib.Plan([a])
        plan_g.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
        tuning = plan_g.autotune([e], wl.n_samples)
        plan_g.set_option(lib.OPT_BATCH, 1)
        plan_g.set_option(lib.OPT_GRAPH, 1)
        img_g = torch.zeros_like(img)
        dt_g, tim_g = timed_steps(plan_g, img_g, args.steps, args.warmup)
        forms["batched_graph_autotuned"] = {
            "ms_per_step": dt_g / args.steps * 1e3, "frames_per_s": a.n_chan * wl.n_samples / (dt_g / args.steps),
            "speedup_vs_plain": dt / dt_g, "tuning": {"transform": ["", "fft", "dft_gemm"][tuning[0][0]],
                                                      "splits": tuning[0][1]},
            "graph_replay_ms": tim_g[lib.TIMER_GRAPH][0] / max(1, tim_g[lib.TIMER_GRAPH][1]),
            "_image": img_g}
        plan_g.close()
    if args.copy_calib:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("# copy reference: 268435456 bytes read, 268435456 bytes written", file=sys.stderr, flush=True)
        del src, dst

    frames = a.n_chan * wl.n_samples
    ms_step = dt / args.steps * 1e3
    value = frames / (dt / args.steps)
    k2 = 1 if a.kernel == 1 else 4
    img_ms, img_n = tim[lib.TIMER_IMAGE]
    avg_img_ms = img_ms / max(1, img_n)
    flops_launch = imaging_flops_per_frame(a.nx, a.n_ant, k2) * frames
    achieved = flops_launch / (avg_img_ms * 1e-3) / 1e12
    bpe = synth.FMT_BYTES[a.efmt]
    bytes_launch = imaging_bytes_per_frame(a.n_ant, bpe, a.nx, wl.n_samples, wl.t_cal) * frames
    traffic = measured_traffic(args.workload) if not args.splits else None
    kernels = {
        "imaging": {"avg_ms": avg_img_ms, "launches": img_n},
        "calibration_solve": {"avg_ms": tim[lib.TIMER_SOLVE][0] / max(1, tim[lib.TIMER_SOLVE][1]),
                              "launches": tim[lib.TIMER_SOLVE][1]},
        "image_reduce": {"avg_ms": tim[lib.TIMER_REDUCE][0] / max(1, tim[lib.TIMER_REDUCE][1]),
                         "launches": tim[lib.TIMER_REDUCE][1]},
    }

    cpu, parity = None, None
    if args.cpu_budget > 0:
        print("# timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        extra = {k: v["_image"].cpu().numpy() for k, v in forms.items()}
        cpu, parity = cpu_baseline(wl, packed, args.cpu_budget, img.cpu().numpy(), g.cpu().numpy(), extra)
    for v in forms.values():
        v.pop("_image", None)

    out = {
        "metric": "EPIC frames/s (grid+FFT+|E|^2+EPICal) vs plain FP32 path; % HBM roofline",
        "value": value,
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded generator: random layout, power-law sky, complex-Gaussian sources and noise, "
                "quantised)",
        "config": {"workload": describe(wl), "frames_per_step": frames, "n_ant": a.n_ant, "n_chan": a.n_chan,
                   "grid": [a.ny, a.nx], "n_samples": wl.n_samples, "t_cal": wl.t_cal,
                   "efmt": synth.FMT_NAMES[a.efmt], "path": "plain FP32 FFT", "parallelism": "1 GPU"},
        "msamples_per_s": value * a.n_ant / 1e6,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "kernel": "k_image (calibrate+grid+FFT+|X|^2)",
                     "flops_per_frame": imaging_flops_per_frame(a.nx, a.n_ant, k2),
                     "hbm_bytes_per_frame": bytes_launch / frames,
                     "hbm_frac": bytes_launch / (avg_img_ms * 1e-3) / 1e9 / PEAK_HBM_GBS},
        "kernels": kernels,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
        "forms": forms,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
