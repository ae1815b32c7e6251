"""ctypes binding of libepic.so (include/epic.h).

Argument marshalling only: tensors are checked for device, dtype, shape and
contiguity and their storage pointers are handed to the C ABI together with
torch's current HIP stream.  Every step of the loop runs in the library's HIP
kernels; there is no fallback, and loading fails loudly when the library has
not been built.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libepic.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "epic.h")

EPIC_OK, EPIC_ERR_ARG, EPIC_ERR_ALLOC, EPIC_ERR_HIP, EPIC_ERR_UNSUPPORTED, EPIC_ERR_STATE = 0, -1, -2, -3, -4, -5
_NAMES = {EPIC_ERR_ARG: "EPIC_ERR_ARG", EPIC_ERR_ALLOC: "EPIC_ERR_ALLOC", EPIC_ERR_HIP: "EPIC_ERR_HIP",
          EPIC_ERR_UNSUPPORTED: "EPIC_ERR_UNSUPPORTED", EPIC_ERR_STATE: "EPIC_ERR_STATE"}
CF32, CI8, CI4 = 0, 1, 2
OPT_SPLITS, OPT_TRANSFORM, OPT_TIMING, OPT_BATCH, OPT_GRAPH, OPT_OVERLAP, OPT_WAIT_POLLS = 1, 2, 3, 4, 5, 6, 7
TIMER_SOLVE, TIMER_IMAGE, TIMER_REDUCE, TIMER_ADJOINT, TIMER_GRAPH, TIMER_COUNT = 0, 1, 2, 3, 4, 5
ANT_FLAGGED, ANT_D_ZERO, ANT_NONFINITE, ANT_BAND_HELD, ANT_BARRIER = 1, 2, 4, 8, 16
BAND_NONE, BAND_MEAN, BAND_POLY, BAND_MAX_DEG = 0, 1, 2, 3


class EpicError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class ArrayDesc(ctypes.Structure):
    _fields_ = [("n_ant", ctypes.c_int32), ("n_chan", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32), ("kernel", ctypes.c_int32), ("efmt", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("x0", ctypes.c_double),
                ("y0", ctypes.c_double), ("ant_xy", ctypes.POINTER(ctypes.c_double)),
                ("freq_hz", ctypes.POINTER(ctypes.c_double)), ("ant_flag", ctypes.POINTER(ctypes.c_uint8))]


class ModelDesc(ctypes.Structure):
    _fields_ = [("src_lmS", ctypes.POINTER(ctypes.c_double)), ("n_src", ctypes.c_int32),
                ("cal_l", ctypes.c_double), ("cal_m", ctypes.c_double), ("gamma", ctypes.c_double),
                ("t_cal", ctypes.c_int32)]


_lib = None

_SIGS = {
    "epic_abi_version": (ctypes.c_int32, []),
    "epic_last_error": (ctypes.c_char_p, []),
    "epic_host_grid_cells": (ctypes.c_int, [ctypes.POINTER(ArrayDesc), ctypes.c_void_p, ctypes.c_void_p]),
    "epic_host_calibrator": (ctypes.c_int, [ctypes.POINTER(ArrayDesc), ctypes.POINTER(ModelDesc),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "epic_plan_create": (ctypes.c_int, [ctypes.POINTER(ArrayDesc), ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]),
    "epic_plan_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "epical_set_model": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ModelDesc)]),
    "epical_set_model_pixels": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ModelDesc),
                                               ctypes.c_void_p, ctypes.c_int32]),
    "epic_host_calibrator_pixels": (ctypes.c_int, [ctypes.POINTER(ArrayDesc), ctypes.POINTER(ModelDesc),
                                                   ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                                   ctypes.c_void_p]),
    "epical_set_band": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "epic_host_band_coordinate": (ctypes.c_int, [ctypes.POINTER(ArrayDesc), ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.c_void_p]),
    "epical_set_denominator": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "epic_plan_get_cells": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "epic_debug_unpack": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_void_p, ctypes.c_void_p]),
    "epic_plan_set_option": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64]),
    "epic_plan_get_timing": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "epic_grid": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "epic_image_accumulate": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "epical_update": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "epic_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "epic_run_noalloc": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "epic_run_snapshots": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "epic_image": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "epic_image_adjoint": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "epic_plan_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]),
    "epic_plan_autotune_cached": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_char_p,
                                                 ctypes.c_void_p]),
    "epic_plan_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "epic_plan_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
}


def header_functions(path: str = HEADER) -> list:
    """Names of the functions include/epic.h declares."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|int32_t|const char\*)\s+(epic\w*)\s*\(", txt, flags=re.M)))


def load() -> ctypes.CDLL:
    """Load libepic.so (built by paper_1603_02126_amd.build); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1603_02126_amd.build` "
                           "(there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().epic_last_error().decode()


def _check(rc: int):
    if rc != EPIC_OK:
        raise EpicError(rc, last_error())


def _dptr(a: np.ndarray, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class _DescHolder:
    """An ArrayDesc plus the numpy buffers it points into."""

    def __init__(self, spec):
        self.xy = np.ascontiguousarray(spec.ant_xy, np.float64)
        self.freq = np.ascontiguousarray(spec.freq_hz, np.float64)
        flag = getattr(spec, "ant_flag", None)
        self.flag = None if flag is None else np.ascontiguousarray(flag, np.uint8)
        self.desc = ArrayDesc(
            n_ant=self.xy.shape[0], n_chan=self.freq.shape[0], nx=int(spec.nx), ny=int(spec.ny),
            kernel=int(spec.kernel), efmt=int(spec.efmt), dx=float(spec.dx), dy=float(spec.dy),
            x0=float(spec.x0), y0=float(spec.y0), ant_xy=_dptr(self.xy), freq_hz=_dptr(self.freq),
            ant_flag=None if self.flag is None else _dptr(self.flag, ctypes.c_uint8))


class _ModelHolder:
    def __init__(self, model_lmS, cal_lm, gamma, t_cal):
        self.src = np.ascontiguousarray(model_lmS, np.float64).reshape(-1, 3)
        self.desc = ModelDesc(src_lmS=_dptr(self.src), n_src=self.src.shape[0], cal_l=float(cal_lm[0]),
                              cal_m=float(cal_lm[1]), gamma=float(gamma), t_cal=int(t_cal))


# --------------------------------------------------------------------------
# host-only helpers
# --------------------------------------------------------------------------

def host_grid_cells(spec):
    """(ixy [Na, K, 2] int32, w [Na, K] float64) as the library's tables use them."""
    d = _DescHolder(spec)
    K = 1 if int(spec.kernel) == 1 else 4
    na = d.xy.shape[0]
    ixy = np.zeros((na, K, 2), np.int32)
    w = np.zeros((na, K), np.float64)
    _check(load().epic_host_grid_cells(ctypes.byref(d.desc), ixy.ctypes.data, w.ctypes.data))
    return ixy, w


def host_calibrator(spec, model_lmS, cal_lm, gamma=0.5, t_cal=1):
    """(k0 [F, 2], A [F, Na], D [F, Na]) computed by the library on the host."""
    d = _DescHolder(spec)
    m = _ModelHolder(model_lmS, cal_lm, gamma, t_cal)
    F, na = d.freq.shape[0], d.xy.shape[0]
    k0 = np.zeros((F, 2), np.int32)
    A = np.zeros((F, na), np.complex128)
    D = np.zeros((F, na), np.complex128)
    _check(load().epic_host_calibrator(ctypes.byref(d.desc), ctypes.byref(m.desc), k0.ctypes.data,
                                       A.ctypes.data, D.ctypes.data))
    return k0, A, D


def host_calibrator_pixels(spec, model_lmS, pix_lm, gamma=0.5, t_cal=1):
    """(k [P, F, 2], A [P, F, Na], D [P, F, Na]) of several tapped pixels."""
    d = _DescHolder(spec)
    pix = np.ascontiguousarray(np.atleast_2d(pix_lm), np.float64)
    m = _ModelHolder(model_lmS, pix[0], gamma, t_cal)
    P, F, na = pix.shape[0], d.freq.shape[0], d.xy.shape[0]
    k0 = np.zeros((P, F, 2), np.int32)
    A = np.zeros((P, F, na), np.complex128)
    D = np.zeros((P, F, na), np.complex128)
    _check(load().epic_host_calibrator_pixels(ctypes.byref(d.desc), ctypes.byref(m.desc), pix.ctypes.data, P,
                                              k0.ctypes.data, A.ctypes.data, D.ctypes.data))
    return k0, A, D


def host_band_coordinate(spec, b0, b1):
    """x [F]: the band coordinate of epical_set_band."""
    d = _DescHolder(spec)
    x = np.zeros(d.freq.shape[0], np.float64)
    _check(load().epic_host_band_coordinate(ctypes.byref(d.desc), int(b0), int(b1), x.ctypes.data))
    return x


# --------------------------------------------------------------------------
# device plan
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _req(t, dtype, shape, name, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device} (is on {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (is {t.dtype})")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (has {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def efield_layout(spec, n_samples):
    """(shape, torch dtype) of the packed E-field stream of an array."""
    torch = _torch()
    T, F, Na = int(n_samples), len(spec.freq_hz), len(spec.ant_xy)
    if int(spec.efmt) == CI4:
        return (T, F, Na), torch.uint8
    if int(spec.efmt) == CI8:
        return (T, F, Na, 2), torch.int8
    return (T, F, Na, 2), torch.float32


class Plan:
    """A device plan over one or more arrays (epic_plan_create)."""

    def __init__(self, specs: Sequence, device=None):
        torch = _torch()
        lib = load()
        self.specs = list(specs)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self._holders = [_DescHolder(s) for s in self.specs]
        arr = (ArrayDesc * len(self._holders))(*[h.desc for h in self._holders])
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.epic_plan_create(arr, len(self._holders), ctypes.byref(h)))
        self._h = h
        self._models = [None] * len(self.specs)

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().epic_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- configuration
    def set_model(self, array: int, model_lmS, cal_lm, gamma: float, t_cal: int):
        m = _ModelHolder(model_lmS, cal_lm, gamma, t_cal)
        _check(load().epical_set_model(self._h, int(array), ctypes.byref(m.desc)))
        self._models[array] = m

    def set_model_pixels(self, array: int, model_lmS, pix_lm, gamma: float, t_cal: int):
        """epical_set_model_pixels: EPICal from several tapped directions pix_lm [P, 2]."""
        pix = np.ascontiguousarray(np.atleast_2d(pix_lm), np.float64)
        m = _ModelHolder(model_lmS, pix[0], gamma, t_cal)
        _check(load().epical_set_model_pixels(self._h, int(array), ctypes.byref(m.desc), pix.ctypes.data,
                                              int(pix.shape[0])))
        m.pix = pix
        self._models[array] = m

    def set_band(self, array: int, b0: int, b1: int, mode: int, deg_amp: int = 0, deg_phase: int = 0):
        """epical_set_band: gains shared over channels b0..b1-1 (BAND_MEAN / BAND_POLY; BAND_NONE clears)."""
        _check(load().epical_set_band(self._h, int(array), int(b0), int(b1), int(mode), int(deg_amp),
                                      int(deg_phase)))

    def set_denominator(self, array: int, D):
        """epical_set_denominator: caller-supplied D [n_pix, F, Na] (or [F, Na]) complex128."""
        d = np.ascontiguousarray(D, np.complex128)
        _check(load().epical_set_denominator(self._h, int(array), d.ctypes.data))

    def get_cells(self, array: int):
        """epic_plan_get_cells: (ixy [Na, K, 2] int32, w [Na, K] float32) read back from the device."""
        s = self.specs[array]
        K = 1 if int(s.kernel) == 1 else 4
        na = len(s.ant_xy)
        ixy = np.zeros((na, K, 2), np.int32)
        w = np.zeros((na, K), np.float32)
        _check(load().epic_plan_get_cells(self._h, int(array), ixy.ctypes.data, w.ctypes.data))
        return ixy, w

    def debug_unpack(self, array: int, packed, n=None, out=None, stream=None):
        """epic_debug_unpack: the first n samples of a packed integer stream as int16 [n, 2]."""
        torch = _torch()
        if not isinstance(packed, torch.Tensor) or packed.device != self.device or not packed.is_contiguous():
            raise ValueError("packed must be a contiguous tensor on the plan's device")
        bpe = {CI4: 1, CI8: 2, CF32: 8}[int(self.specs[array].efmt)]
        avail = packed.numel() * packed.element_size() // bpe
        n = avail if n is None else int(n)
        if n < 0 or n > avail:
            raise ValueError("n exceeds the samples held by packed")
        if out is None:
            out = torch.empty((n, 2), dtype=torch.int16, device=self.device)
        po = _req(out, torch.int16, (n, 2), "out", self.device)
        _check(load().epic_debug_unpack(self._h, int(array), ctypes.c_void_p(packed.data_ptr()), n, po,
                                        _stream(stream)))
        return out

    def set_option(self, key: int, value: int):
        _check(load().epic_plan_set_option(self._h, int(key), int(value)))

    def timing(self):
        """{kind: (total ms, launches)} since the last call (needs OPT_TIMING)."""
        ms = np.zeros(TIMER_COUNT, np.float64)
        n = np.zeros(TIMER_COUNT, np.int64)
        _check(load().epic_plan_get_timing(self._h, ms.ctypes.data, n.ctypes.data, TIMER_COUNT))
        return {k: (float(ms[k]), int(n[k])) for k in range(TIMER_COUNT)}

    def autotune(self, efields, n_samples, cache=None, stream=None):
        """Time the candidate transforms / splits / class engines per array on
        these inputs and keep the fastest; with `cache` (a JSON file path) arrays
        already in the cache take its entry (epic_plan_autotune_cached)."""
        ptrs = [self._efield(i, efields[i], f"efield[{i}]")[0] for i in range(len(self.specs))]
        arr = (ctypes.c_void_p * len(ptrs))(*ptrs)
        if cache is None:
            _check(load().epic_plan_autotune(self._h, arr, int(n_samples), _stream(stream)))
        else:
            _check(load().epic_plan_autotune_cached(self._h, arr, int(n_samples), os.fsencode(cache),
                                                     _stream(stream)))
        return self.get_tuning()

    def get_tuning(self):
        """[(transform, splits, class engine, imaging microseconds)] per array;
        class engine 0 = default, 2 or 4 = the dense residue-class engine with
        gridding batches of that many schedule entries."""
        t = np.zeros(4 * len(self.specs), np.int32)
        _check(load().epic_plan_get_tuning(self._h, t.ctypes.data))
        return [tuple(int(v) for v in t[4 * i:4 * i + 4]) for i in range(len(self.specs))]

    def set_tuning(self, tuning):
        t = np.zeros(4 * len(self.specs), np.int32)
        for i, (tr, sp, *rest) in enumerate(tuning):
            t[4 * i], t[4 * i + 1] = tr, sp
            t[4 * i + 2] = rest[0] if rest else 0
        _check(load().epic_plan_set_tuning(self._h, t.ctypes.data))

    def _dims(self, i):
        s = self.specs[i]
        return len(s.freq_hz), len(s.ant_xy), int(s.ny), int(s.nx)

    def _efield(self, i, t, name="efield"):
        torch = _torch()
        s = self.specs[i]
        F, Na = len(s.freq_hz), len(s.ant_xy)
        shape, dt = efield_layout(s, t.shape[0] if isinstance(t, torch.Tensor) else 0)
        p = _req(t, dt, None, name, self.device)
        if tuple(t.shape[1:]) != tuple(shape[1:]):
            raise ValueError(f"{name} must have shape [T]{list(shape[1:])} (has {tuple(t.shape)})")
        return p, t.shape[0]

    # -- stage-wise calls
    def grid(self, i, efield, t0, nt, u, out=None, stream=None):
        torch = _torch()
        F, Na, ny, nx = self._dims(i)
        pe, T = self._efield(i, efield)
        if t0 < 0 or nt < 0 or t0 + nt > T:
            raise ValueError("sample range outside the E-field stream")
        pu = _req(u, torch.complex64, (F, Na), "u", self.device)
        if out is None:
            out = torch.empty((nt, F, ny, nx), dtype=torch.complex64, device=self.device)
        po = _req(out, torch.complex64, (nt, F, ny, nx), "grid", self.device)
        _check(load().epic_grid(self._h, i, pe, int(t0), int(nt), pu, po, _stream(stream)))
        return out

    def image_accumulate(self, i, grid, image, tap=None, stream=None):
        torch = _torch()
        F, Na, ny, nx = self._dims(i)
        nt = grid.shape[0]
        pg = _req(grid, torch.complex64, (nt, F, ny, nx), "grid", self.device)
        pi = _req(image, torch.float32, (F, ny, nx), "image", self.device)
        pt = None if tap is None else _req(tap, torch.complex64, (nt, F), "tap", self.device)
        _check(load().epic_image_accumulate(self._h, i, pg, int(nt), pi, pt, _stream(stream)))
        return image

    def epical_update(self, i, efield, t0, nt, tap, kq, gains, finalize, status=None, stream=None):
        torch = _torch()
        F, Na, ny, nx = self._dims(i)
        pe, T = self._efield(i, efield)
        if t0 < 0 or nt < 0 or t0 + nt > T:
            raise ValueError("sample range outside the E-field stream")
        pt = _req(tap, torch.complex64, (nt, F), "tap", self.device) if nt > 0 else None
        pk = _req(kq, torch.float64, (F, Na, 4), "kq", self.device)
        pg = _req(gains, torch.complex128, (F, Na), "gains", self.device)
        ps = None if status is None else _req(status, torch.int32, (F, Na), "status", self.device)
        _check(load().epical_update(self._h, i, pe, int(t0), int(nt), pt, pk, pg, int(bool(finalize)), ps,
                                    _stream(stream)))

    # -- fused loop
    def run_noalloc(self, efields, n_samples, gains, images, gain_hist=None, status=None, stream=None):
        """epic_run_noalloc: epic_run with every intermediate in the library's static device scratch."""
        self.run(efields, n_samples, gains, images, gain_hist, status, stream, _entry="epic_run_noalloc")

    def run(self, efields, n_samples, gains, images, gain_hist=None, status=None, stream=None, _entry="epic_run"):
        """epic_run over all arrays; lists of tensors, one per array."""
        torch = _torch()
        n = len(self.specs)
        if not (len(efields) == len(gains) == len(images) == n):
            raise ValueError("one efield / gains / image tensor per array")
        keep = []
        pe, pg, pi, ph, ps = [], [], [], [], []
        for i in range(n):
            F, Na, ny, nx = self._dims(i)
            p, T = self._efield(i, efields[i], f"efield[{i}]")
            if T < n_samples:
                raise ValueError(f"efield[{i}] holds {T} samples < n_samples={n_samples}")
            pe.append(p)
            pg.append(_req(gains[i], torch.complex128, (F, Na), f"gains[{i}]", self.device))
            pi.append(_req(images[i], torch.float32, (F, ny, nx), f"image[{i}]", self.device))
            if gain_hist is not None:
                m = self._models[i]
                if m is None:
                    raise RuntimeError("set_model first")
                n_int = -(-int(n_samples) // int(m.desc.t_cal))
                ph.append(_req(gain_hist[i], torch.complex128, (n_int + 1, F, Na), f"gain_hist[{i}]", self.device))
            if status is not None:
                ps.append(_req(status[i], torch.int32, (F, Na), f"status[{i}]", self.device))
        VP = ctypes.c_void_p * n
        a_e, a_g, a_i = VP(*pe), VP(*pg), VP(*pi)
        a_h = VP(*ph) if gain_hist is not None else None
        a_s = VP(*ps) if status is not None else None
        keep += [a_e, a_g, a_i, a_h, a_s]
        _check(getattr(load(), _entry)(self._h, a_e, int(n_samples), a_g, a_i, a_h, a_s, _stream(stream)))

    def run_snapshots(self, i, efield, n_samples, t_acc, gains, images, gain_hist=None, status=None, stream=None):
        """epic_run_snapshots: images [ceil(n_samples / t_acc), F, ny, nx] float32, one per window."""
        torch = _torch()
        F, Na, ny, nx = self._dims(i)
        pe, T = self._efield(i, efield)
        if T < n_samples:
            raise ValueError("n_samples exceeds the E-field stream")
        n_win = -(-int(n_samples) // int(t_acc)) if t_acc > 0 else 0
        pg = _req(gains, torch.complex128, (F, Na), "gains", self.device)
        pi = _req(images, torch.float32, (n_win, F, ny, nx), "images", self.device)
        ph = ps = None
        if gain_hist is not None:
            m = self._models[i]
            if m is None:
                raise RuntimeError("set_model first")
            n_int = -(-int(n_samples) // int(m.desc.t_cal))
            ph = _req(gain_hist, torch.complex128, (n_int + 1, F, Na), "gain_hist", self.device)
        if status is not None:
            ps = _req(status, torch.int32, (F, Na), "status", self.device)
        _check(load().epic_run_snapshots(self._h, int(i), pe, int(n_samples), int(t_acc), pg, pi, ph, ps,
                                         _stream(stream)))

    def image(self, i, efield, n_samples, gains, out=None, stream=None):
        """epic_image: time-averaged image with fixed gains [F, Na] complex128."""
        torch = _torch()
        F, Na, ny, nx = self._dims(i)
        pe, T = self._efield(i, efield)
        if T < n_samples:
            raise ValueError("n_samples exceeds the E-field stream")
        pg = _req(gains, torch.complex128, (F, Na), "gains", self.device)
        if out is None:
            out = torch.empty((F, ny, nx), dtype=torch.float32, device=self.device)
        po = _req(out, torch.float32, (F, ny, nx), "image", self.device)
        _check(load().epic_image(self._h, i, pe, int(n_samples), pg, po, _stream(stream)))
        return out

    def image_adjoint(self, i, efield, n_samples, gains, dL_dI, out=None, stream=None):
        """epic_image_adjoint: dL/dRe g + i dL/dIm g for a real loss of the image."""
        torch = _torch()
        F, Na, ny, nx = self._dims(i)
        pe, T = self._efield(i, efield)
        if T < n_samples:
            raise ValueError("n_samples exceeds the E-field stream")
        pg = _req(gains, torch.complex128, (F, Na), "gains", self.device)
        pr = _req(dL_dI, torch.float32, (F, ny, nx), "dL_dI", self.device)
        if out is None:
            out = torch.empty((F, Na), dtype=torch.complex128, device=self.device)
        po = _req(out, torch.complex128, (F, Na), "dL_dg", self.device)
        _check(load().epic_image_adjoint(self._h, i, pe, int(n_samples), pg, pr, po, _stream(stream)))
        return out
