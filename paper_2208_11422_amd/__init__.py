"""Light-field Richardson-Lucy deconvolution on MI355X: Python binding.

A thin ctypes layer over ``liblfrl.so`` (C ABI declared in include/lfrl.h).
It only marshals arguments: every step of the computation runs in the
library's HIP kernels.  PyTorch provides device memory and streams; importing
torch first also loads the HIP runtime the library shares with it.

The functions named ``lfrl_*`` mirror the C entry points one to one; the
:class:`Plan` class is a small convenience wrapper over them.  There is no CPU
fallback: if the library is missing every call raises :class:`LfrlError`.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import torch

__all__ = [
    "LfrlError", "PlanDesc", "PlanInfo", "RlOpts", "RlReport",
    "lfrl_plan_footprint", "lfrl_plan", "lfrl_plan_destroy", "lfrl_plan_get_info",
    "lfrl_forward", "lfrl_backward", "lfrl_deconvolve", "lfrl_metric", "lfrl_metric_ex",
    "lfrl_metric_noalloc", "lfrl_psf_compute", "Optics", "psf_from_optics",
    "lfrl_metric_cutoff", "lfrl_profile_enable", "lfrl_profile_read", "lfrl_last_error",
    "Plan", "library_path", "STOP_NONE", "STOP_METRIC", "STOP_TRACK", "FP32", "SPLIT_FP16",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblfrl.so")

FP32, SPLIT_FP16, SPLIT_BF16 = 0, 1, 2
STOP_NONE, STOP_METRIC, STOP_TRACK = 0, 1, 2
UPDATE_RL, UPDATE_ISRA = 0, 1
INIT_ONES, INIT_GIVEN, INIT_BACKPROJECT = 0, 1, 2
REGION_TRIANGLE, REGION_RECTANGLE, REGION_WHOLE = 0, 1, 2
NORM_MATRIX, NORM_REGION, NORM_SPECTRAL = 0, 1, 2

_STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_NOMEM", -3: "ERR_DEVICE",
           -4: "ERR_UNSUPPORTED", -5: "ERR_NUMERIC"}


class LfrlError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lfrl {_STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


class PlanDesc(ctypes.Structure):
    _fields_ = [("nnum", ctypes.c_int32), ("nz", ctypes.c_int32), ("ksize", ctypes.c_int32),
                ("max_h", ctypes.c_int32), ("max_w", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("tile_q", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("max_batch", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("tile_q", ctypes.c_int32), ("tile_out", ctypes.c_int32),
                ("taps", ctypes.c_int32), ("nfreq", ctypes.c_int32),
                ("max_tiles", ctypes.c_int32), ("split_k", ctypes.c_int32),
                ("resident_bytes", ctypes.c_size_t), ("workspace_bytes", ctypes.c_size_t),
                ("tune_candidates", ctypes.c_int32), ("tune_ms", ctypes.c_double),
                ("nfreq_unique", ctypes.c_int32)]


class RlOpts(ctypes.Structure):
    _fields_ = [("max_iters", ctypes.c_int32), ("stop", ctypes.c_int32),
                ("patience", ctypes.c_int32), ("init", ctypes.c_int32),
                ("xs", ctypes.c_double), ("ys", ctypes.c_double),
                ("update", ctypes.c_int32), ("region", ctypes.c_int32),
                ("norm", ctypes.c_int32), ("window", ctypes.c_int32),
                ("background", ctypes.c_double)]


class Optics(ctypes.Structure):
    """Optical parameters of lfrl_psf_compute (lengths in one unit)."""
    _fields_ = [("wavelength", ctypes.c_double), ("na", ctypes.c_double),
                ("n_medium", ctypes.c_double), ("mag", ctypes.c_double),
                ("d_ml", ctypes.c_double), ("f_ml", ctypes.c_double),
                ("nnum", ctypes.c_int32), ("nz", ctypes.c_int32), ("ksize", ctypes.c_int32),
                ("osr", ctypes.c_int32), ("nquad", ctypes.c_int32), ("flags", ctypes.c_uint32)]


PSF_UNIT_SUM = 1


class RlReport(ctypes.Structure):
    _fields_ = [("iters_run", ctypes.c_int32), ("best_iter", ctypes.c_int32),
                ("stopped", ctypes.c_int32), ("weak_voxels", ctypes.c_int32),
                ("metric_trace", ctypes.POINTER(ctypes.c_double)),
                ("flux_trace", ctypes.POINTER(ctypes.c_double))]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise LfrlError(-4, f"{_LIB_PATH} is not built (run __graft_entry__.build() or "
                            "python paper_2208_11422_amd/build.py)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    sz = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "lfrl_plan_footprint": [ctypes.POINTER(PlanDesc), sz, sz],
        "lfrl_plan": [ctypes.POINTER(vp), ctypes.POINTER(PlanDesc), vp, vp],
        "lfrl_plan_destroy": [vp],
        "lfrl_plan_get_info": [vp, ctypes.POINTER(PlanInfo)],
        "lfrl_forward": [vp, i32, i32, vp, vp, vp],
        "lfrl_backward": [vp, i32, i32, vp, vp, vp],
        "lfrl_deconvolve": [vp, i32, i32, vp, vp, ctypes.POINTER(RlOpts),
                            ctypes.POINTER(RlReport), vp],
        "lfrl_metric": [i32, i32, i32, vp, dbl, dbl, vp, vp],
        "lfrl_metric_ex": [i32, i32, i32, vp, dbl, dbl, i32, i32, vp, vp],
        "lfrl_metric_noalloc": [i32, i32, i32, vp, dbl, dbl, i32, i32, vp, vp],
        "lfrl_metric_cutoff": [dbl, dbl, i32, dbl, dbl, i32, i32,
                               ctypes.POINTER(dbl), ctypes.POINTER(dbl)],
        "lfrl_job_footprint": [vp, i32, i32, sz],
        "lfrl_job_create": [ctypes.POINTER(vp), vp, i32, i32, vp, vp, ctypes.POINTER(RlOpts),
                            ctypes.c_uint32, vp],
        "lfrl_job_step": [ctypes.POINTER(vp), i32, ctypes.POINTER(i32), vp],
        "lfrl_job_poll": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "lfrl_job_result": [vp, vp, ctypes.POINTER(RlReport), vp],
        "lfrl_job_destroy": [vp],
        "lfrl_deconvolve_batch": [ctypes.POINTER(vp), i32, ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.POINTER(RlOpts), ctypes.POINTER(RlReport), vp],
        "lfrl_psf_compute": [ctypes.POINTER(Optics), ctypes.POINTER(dbl), vp, vp],
        "lfrl_profile_enable": [vp, i32],
        "lfrl_profile_read": [vp, ctypes.c_char_p, ctypes.POINTER(dbl),
                              ctypes.POINTER(ctypes.c_int64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.lfrl_last_error.argtypes = []
    lib.lfrl_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def lfrl_last_error() -> str:
    return _load().lfrl_last_error().decode()


def _check(rc: int) -> None:
    if rc != 0:
        raise LfrlError(rc, lfrl_last_error())


def _stream(stream) -> Optional[int]:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _dev_f32(t: torch.Tensor, name: str, shape=None) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise LfrlError(-1, f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise LfrlError(-1, f"{name} must be contiguous float32")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise LfrlError(-1, f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


# ---------------------------------------------------------------------------
# one-to-one wrappers of the C entry points
# ---------------------------------------------------------------------------
def lfrl_plan_footprint(desc: PlanDesc):
    r, w = ctypes.c_size_t(), ctypes.c_size_t()
    _check(_load().lfrl_plan_footprint(ctypes.byref(desc), ctypes.byref(r), ctypes.byref(w)))
    return r.value, w.value


def lfrl_plan(desc: PlanDesc, psf: torch.Tensor, stream=None) -> int:
    shape = (desc.nz, desc.nnum, desc.nnum, desc.ksize, desc.ksize)
    ptr = _dev_f32(psf, "psf", shape)
    h = ctypes.c_void_p()
    _check(_load().lfrl_plan(ctypes.byref(h), ctypes.byref(desc), ptr, _stream(stream)))
    return h.value


def lfrl_plan_destroy(plan: int) -> None:
    _check(_load().lfrl_plan_destroy(plan))


def lfrl_plan_get_info(plan: int) -> dict:
    info = PlanInfo()
    _check(_load().lfrl_plan_get_info(plan, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in PlanInfo._fields_}


def lfrl_forward(plan: int, h: int, w: int, vol: torch.Tensor, img: torch.Tensor,
                 stream=None) -> None:
    _check(_load().lfrl_forward(plan, h, w, _dev_f32(vol, "vol"), _dev_f32(img, "img"),
                                _stream(stream)))


def lfrl_backward(plan: int, h: int, w: int, img: torch.Tensor, vol: torch.Tensor,
                  stream=None) -> None:
    _check(_load().lfrl_backward(plan, h, w, _dev_f32(img, "img"), _dev_f32(vol, "vol"),
                                 _stream(stream)))


def lfrl_deconvolve(plan: int, h: int, w: int, img: torch.Tensor, vol: torch.Tensor,
                    opts: RlOpts, want_metric: bool = True, want_flux: bool = False,
                    stream=None) -> dict:
    rep, mt, ft = _report_buffers(max(int(opts.max_iters), 1), want_metric, want_flux)
    _check(_load().lfrl_deconvolve(plan, h, w, _dev_f32(img, "img"), _dev_f32(vol, "vol"),
                                   ctypes.byref(opts), ctypes.byref(rep), _stream(stream)))
    return _report_dict(rep, mt, ft, opts.stop)


def lfrl_metric(nz: int, h: int, w: int, img: torch.Tensor, xs: float, ys: float,
                out: torch.Tensor, stream=None) -> None:
    if not out.is_cuda or out.dtype != torch.float64 or out.numel() < 1:
        raise LfrlError(-1, "out must be a CUDA float64 tensor")
    _check(_load().lfrl_metric(nz, h, w, _dev_f32(img, "img"), float(xs), float(ys),
                               out.data_ptr(), _stream(stream)))


def lfrl_metric_ex(nz: int, h: int, w: int, img: torch.Tensor, xs: float, ys: float,
                   region: int, norm: int, out: torch.Tensor, stream=None) -> None:
    if not out.is_cuda or out.dtype != torch.float64 or out.numel() < 1:
        raise LfrlError(-1, "out must be a CUDA float64 tensor")
    _check(_load().lfrl_metric_ex(nz, h, w, _dev_f32(img, "img"), float(xs), float(ys),
                                  int(region), int(norm), out.data_ptr(), _stream(stream)))


def lfrl_metric_noalloc(nz: int, h: int, w: int, img: torch.Tensor, xs: float, ys: float,
                        region: int, norm: int, out: torch.Tensor, stream=None) -> None:
    if not out.is_cuda or out.dtype != torch.float64 or out.numel() < 1:
        raise LfrlError(-1, "out must be a CUDA float64 tensor")
    _check(_load().lfrl_metric_noalloc(nz, h, w, _dev_f32(img, "img"), float(xs), float(ys),
                                       int(region), int(norm), out.data_ptr(), _stream(stream)))


def lfrl_psf_compute(optics: Optics, depths, psf: torch.Tensor, stream=None) -> None:
    """PSF set [nz][nnum][nnum][ksize][ksize] from optical parameters into psf
    (a CUDA float32 tensor); depths has optics.nz entries."""
    z = (ctypes.c_double * max(1, len(depths)))(*[float(d) for d in depths])
    if len(depths) != optics.nz:
        raise LfrlError(-1, f"{len(depths)} depths for nz = {optics.nz}")
    _check(_load().lfrl_psf_compute(ctypes.byref(optics), z, _dev_f32(psf, "psf"),
                                    _stream(stream)))


def psf_from_optics(*, wavelength: float, na: float, n_medium: float, mag: float,
                    d_ml: float, f_ml: float, nnum: int, ksize: int, depths, osr: int = 3,
                    nquad: int = 0, unit_sum: bool = False, device=None,
                    stream=None) -> torch.Tensor:
    """Allocate and compute a PSF set (see lfrl_psf_compute)."""
    dev = torch.device(device) if device is not None else torch.device("cuda", 0)
    o = Optics(wavelength=wavelength, na=na, n_medium=n_medium, mag=mag, d_ml=d_ml, f_ml=f_ml,
               nnum=nnum, nz=len(depths), ksize=ksize, osr=osr, nquad=nquad,
               flags=PSF_UNIT_SUM if unit_sum else 0)
    out = torch.empty((len(depths), nnum, nnum, ksize, ksize), dtype=torch.float32, device=dev)
    lfrl_psf_compute(o, depths, out, stream)
    return out


def lfrl_metric_cutoff(d_ml: float, mag: float, nnum: int, wavelength: float, na: float,
                       h: int, w: int):
    xs, ys = ctypes.c_double(), ctypes.c_double()
    _check(_load().lfrl_metric_cutoff(d_ml, mag, nnum, wavelength, na, h, w,
                                      ctypes.byref(xs), ctypes.byref(ys)))
    return xs.value, ys.value


JOB_FLUX = 1
PLAN_AUTOTUNE, NORMALIZE_PSF = 1, 2


def _report_buffers(n: int, want_metric: bool, want_flux: bool):
    mt = (ctypes.c_double * n)() if want_metric else None
    ft = (ctypes.c_double * n)() if want_flux else None
    rep = RlReport()
    rep.metric_trace = ctypes.cast(mt, ctypes.POINTER(ctypes.c_double)) if mt is not None else None
    rep.flux_trace = ctypes.cast(ft, ctypes.POINTER(ctypes.c_double)) if ft is not None else None
    return rep, mt, ft


def _report_dict(rep: RlReport, mt, ft, stop: int) -> dict:
    k = rep.iters_run
    out = {"iters_run": k, "best_iter": rep.best_iter, "stopped": bool(rep.stopped),
           "weak_voxels": rep.weak_voxels}
    if mt is not None and stop != STOP_NONE:
        out["metric_trace"] = list(mt[:k])
    if ft is not None:
        out["flux_trace"] = list(ft[:k])
    return out


def lfrl_job_footprint(plan: int, h: int, w: int) -> int:
    b = ctypes.c_size_t()
    _check(_load().lfrl_job_footprint(plan, h, w, ctypes.byref(b)))
    return b.value


def lfrl_job_create(plan: int, h: int, w: int, img: torch.Tensor, opts: RlOpts,
                    vol0: Optional[torch.Tensor] = None, flags: int = 0, stream=None) -> int:
    j = ctypes.c_void_p()
    v0 = _dev_f32(vol0, "vol0") if vol0 is not None else None
    _check(_load().lfrl_job_create(ctypes.byref(j), plan, h, w, _dev_f32(img, "img"), v0,
                                   ctypes.byref(opts), flags, _stream(stream)))
    return j.value


def lfrl_job_step(jobs, stream=None) -> int:
    arr = (ctypes.c_void_p * max(len(jobs), 1))(*jobs)
    active = ctypes.c_int32()
    _check(_load().lfrl_job_step(arr, len(jobs), ctypes.byref(active), _stream(stream)))
    return active.value


def lfrl_job_poll(job: int):
    d, k = ctypes.c_int32(), ctypes.c_int32()
    _check(_load().lfrl_job_poll(job, ctypes.byref(d), ctypes.byref(k)))
    return bool(d.value), k.value


def lfrl_job_result(job: int, vol: Optional[torch.Tensor], max_iters: int, stop: int,
                    want_metric: bool = True, want_flux: bool = False, stream=None) -> dict:
    rep, mt, ft = _report_buffers(max(max_iters, 1), want_metric, want_flux)
    _check(_load().lfrl_job_result(job, _dev_f32(vol, "vol") if vol is not None else None,
                                   ctypes.byref(rep), _stream(stream)))
    return _report_dict(rep, mt, ft, stop)


def lfrl_job_destroy(job: int) -> None:
    _check(_load().lfrl_job_destroy(job))


def lfrl_deconvolve_batch(plans, hs, ws, imgs, vols, opts, want_flux: bool = False,
                          stream=None) -> list:
    n = len(plans)
    P = (ctypes.c_void_p * n)(*plans)
    H = (ctypes.c_int32 * n)(*hs)
    W = (ctypes.c_int32 * n)(*ws)
    I = (ctypes.c_void_p * n)(*[_dev_f32(t, "img") for t in imgs])
    V = (ctypes.c_void_p * n)(*[_dev_f32(t, "vol") for t in vols])
    O = (RlOpts * n)(*opts)
    R = (RlReport * n)()
    keep = []
    for i in range(n):
        rep, mt, ft = _report_buffers(max(int(opts[i].max_iters), 1), True, want_flux)
        R[i] = rep
        keep.append((mt, ft))
    _check(_load().lfrl_deconvolve_batch(P, n, H, W, I, V, O, R, _stream(stream)))
    return [_report_dict(R[i], keep[i][0], keep[i][1], opts[i].stop) for i in range(n)]


def lfrl_profile_enable(plan: int, on: bool) -> None:
    _check(_load().lfrl_profile_enable(plan, 1 if on else 0))


def lfrl_profile_read(plan: int, kernel: str):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(_load().lfrl_profile_read(plan, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------
class Plan:
    """Resident PSF spectra for one PSF set, serving images up to max_h x max_w."""

    def __init__(self, psf: torch.Tensor, max_h: int, max_w: int, tile_q: int = 0,
                 precision: int = FP32, max_batch: int = 1, autotune: bool = False,
                 normalize_psf: bool = False, stream=None):
        nz, n, n2, k, k2 = psf.shape
        if n != n2 or k != k2:
            raise LfrlError(-1, "psf must be [nz][N][N][K][K]")
        self.desc = PlanDesc(nnum=n, nz=nz, ksize=k, max_h=max_h, max_w=max_w,
                             precision=precision, tile_q=tile_q,
                             flags=(PLAN_AUTOTUNE if autotune else 0)
                             | (NORMALIZE_PSF if normalize_psf else 0), max_batch=max_batch)
        self.nnum, self.nz, self.ksize = n, nz, k
        self.device = psf.device
        self.handle = lfrl_plan(self.desc, psf, stream)
        self.info = lfrl_plan_get_info(self.handle)

    def close(self) -> None:
        if getattr(self, "handle", None):
            lfrl_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, vol: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        _, h, w = vol.shape
        if out is None:
            out = torch.empty((h, w), dtype=torch.float32, device=vol.device)
        lfrl_forward(self.handle, h, w, vol, out, stream)
        return out

    def backward(self, img: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        h, w = img.shape
        if out is None:
            out = torch.empty((self.nz, h, w), dtype=torch.float32, device=img.device)
        lfrl_backward(self.handle, h, w, img, out, stream)
        return out

    def deconvolve(self, img: torch.Tensor, iters: int, *, stop: int = STOP_NONE,
                   patience: int = 1, xs: float = 1.0, ys: float = 1.0,
                   init: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                   want_flux: bool = False, stream=None, **variants):
        """``variants``: update, background, backproject_start, region, norm,
        window (see rl_opts)."""
        h, w = img.shape
        if out is None:
            out = torch.empty((self.nz, h, w), dtype=torch.float32, device=img.device)
        if init is not None:
            out.copy_(init)
        opts = rl_opts(iters, stop, patience, xs, ys, init is not None, **variants)
        rep = lfrl_deconvolve(self.handle, h, w, img, out, opts, want_metric=True,
                              want_flux=want_flux, stream=stream)
        return out, rep


def rl_opts(iters: int, stop: int = STOP_NONE, patience: int = 1, xs: float = 1.0,
            ys: float = 1.0, given_start: bool = False, *, update: int = UPDATE_RL,
            background: float = 0.0, backproject_start: bool = False,
            region: int = REGION_TRIANGLE, norm: int = NORM_MATRIX, window: int = 1) -> RlOpts:
    """lfrl_rl_opts from keyword arguments (the defaults are the method as the
    paper states it)."""
    if given_start and backproject_start:
        raise LfrlError(-1, "a given start volume and the back projection start exclude each other")
    init = INIT_GIVEN if given_start else INIT_BACKPROJECT if backproject_start else INIT_ONES
    return RlOpts(max_iters=iters, stop=stop, patience=patience, init=init, xs=xs, ys=ys,
                  update=update, region=region, norm=norm, window=window,
                  background=background)


class Job:
    """One frame's Richardson-Lucy run held on the device (see lfrl_job_create)."""

    def __init__(self, plan: Plan, img: torch.Tensor, iters: int, *, stop: int = STOP_NONE,
                 patience: int = 1, xs: float = 1.0, ys: float = 1.0,
                 init: Optional[torch.Tensor] = None, want_flux: bool = False, stream=None,
                 **variants):
        self.plan = plan
        self.h, self.w = img.shape
        self.opts = rl_opts(iters, stop, patience, xs, ys, init is not None, **variants)
        self.want_flux = want_flux
        self.handle = lfrl_job_create(plan.handle, self.h, self.w, img, self.opts, vol0=init,
                                      flags=JOB_FLUX if want_flux else 0, stream=stream)

    @staticmethod
    def step(jobs, stream=None) -> int:
        """One iteration for every job not done; returns how many are not done."""
        return lfrl_job_step([j.handle for j in jobs], stream)

    def poll(self):
        return lfrl_job_poll(self.handle)

    def result(self, out: Optional[torch.Tensor] = None, stream=None):
        if out is None:
            out = torch.empty((self.plan.nz, self.h, self.w), dtype=torch.float32,
                              device=self.plan.device)
        rep = lfrl_job_result(self.handle, out, int(self.opts.max_iters), int(self.opts.stop),
                              want_flux=self.want_flux, stream=stream)
        return out, rep

    def close(self) -> None:
        if getattr(self, "handle", None):
            lfrl_job_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def metric(img: torch.Tensor, xs: float, ys: float, stream=None, *,
           region: int = REGION_TRIANGLE, norm: int = NORM_MATRIX) -> float:
    """DCT entropy of a 2-D image, or of the z-MIP of a [nz][h][w] volume."""
    if img.dim() == 2:
        nz, (h, w) = 1, img.shape
    else:
        nz, h, w = img.shape
    out = torch.empty(1, dtype=torch.float64, device=img.device)
    lfrl_metric_ex(nz, h, w, img, xs, ys, region, norm, out, stream)
    return float(out.item())
