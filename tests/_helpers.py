"""Shared helpers for the tests: run a workload through the HIP library and
through the oracle on identical inputs, and the parity metrics."""
import numpy as np

from oracle import epic_oracle as O
from paper_1603_02126_amd import synth

IMAGE_RTOL = 1e-5   # max |I_gpu - I_oracle| / max |I_oracle| per channel
GAIN_RTOL = 1e-4    # max over antennas, channels (and intervals) of |g_gpu - g_oracle| / |g_oracle|


def image_err(gpu, ref):
    """Per-channel normwise relative image error."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    num = np.abs(gpu - ref).reshape(ref.shape[0], -1).max(1)
    den = np.abs(ref).reshape(ref.shape[0], -1).max(1)
    return num / den


def gain_err(gpu, ref):
    """Element-wise relative gain error: the largest |g_gpu - g_oracle| /
    |g_oracle| over every antenna, channel (and interval).  A zero oracle gain
    counts as an error unless the GPU gain is zero too."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    diff = np.abs(gpu - ref)
    mag = np.abs(ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(mag > 0, diff / np.where(mag > 0, mag, 1.0), np.where(diff > 0, np.inf, 0.0))
    return float(np.max(rel))


def oracle_run(wl, packed, channels=None):
    """Oracle on the packed stream (same bytes the GPU sees)."""
    E = O.unpack(packed, wl.array.efmt)
    pb = O.Problem.from_workload(wl)
    chans = list(range(wl.array.n_chan)) if channels is None else list(channels)
    return O.run(E, pb, wl.g0, channels=chans)


def gpu_run(wl, packed, device, plan=None, splits=0, hist=True, transform=0, cls_engine=0):
    import torch
    from paper_1603_02126_amd import lib
    own = plan is None
    if own:
        plan = lib.Plan([wl.array])
        plan.set_model(0, wl.model_lmS, wl.cal_lm, wl.gamma, wl.t_cal)
    if splits:
        plan.set_option(lib.OPT_SPLITS, splits)
    if transform:
        plan.set_option(lib.OPT_TRANSFORM, transform)
    if cls_engine:
        plan.set_tuning([(0, 0, cls_engine)])
    a = wl.array
    e = torch.from_numpy(np.ascontiguousarray(packed)).to(device)
    g = torch.from_numpy(np.ascontiguousarray(wl.g0)).to(device)
    img = torch.zeros((a.n_chan, a.ny, a.nx), dtype=torch.float32, device=device)
    n_int = -(-wl.n_samples // wl.t_cal)
    gh = torch.zeros((n_int + 1, a.n_chan, a.n_ant), dtype=torch.complex128, device=device) if hist else None
    st = torch.zeros((a.n_chan, a.n_ant), dtype=torch.int32, device=device)
    plan.run([e], wl.n_samples, [g], [img], gain_hist=[gh] if hist else None, status=[st])
    torch.cuda.synchronize()
    out = dict(image=img.cpu().numpy(), gains=g.cpu().numpy(), status=st.cpu().numpy())
    if hist:
        out["hist"] = gh.cpu().numpy()
    if own:
        plan.close()
    return out
