"""Python binding of libehi (include/ehi.h): argument marshalling only.

Every stage runs in the HIP library; this module checks tensor shapes, dtypes
and devices, passes raw device pointers and the current HIP stream, and turns
status codes into exceptions.  PyTorch provides device memory (the survey
workspace is one uint8 tensor) and streams.

If the shared library is missing the import of the library fails loudly; there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libehi.so")

EHI_OK, EHI_EINVAL, EHI_ENOMEM, EHI_EHIP, EHI_ENOTPD, EHI_ESTATE = range(6)
PREC_PLAIN_FP32 = 0
PREC_SPLIT_BF16 = 1
_PREC = {"plain_fp32": PREC_PLAIN_FP32, "split_bf16": PREC_SPLIT_BF16}
WEIGHT_LONG_RECORD, WEIGHT_FINITE_RECORD = 0, 1
_WEIGHT = {"long_record": WEIGHT_LONG_RECORD, "finite_record": WEIGHT_FINITE_RECORD}

# every symbol declared in include/ehi.h
SYMBOLS = (
    "ehi_workspace_bytes", "ehi_create", "ehi_build_green", "ehi_build_hessian", "ehi_factor",
    "ehi_apply_multipliers", "ehi_lambda_max", "ehi_copy_green_dft", "ehi_copy_compressed", "ehi_load_green_dft",
    "ehi_copy_hessian", "ehi_load_hessian", "ehi_copy_factor", "ehi_destroy", "ehi_last_error",
    "ehi_version", "ehi_profile_enable", "ehi_profile_read", "ehi_batch_workspace_bytes",
    "ehi_factor_batch", "ehi_factor_batch_static", "ehi_set_stream", "ehi_set_launch", "ehi_get_launch",
    "ehi_set_medium", "ehi_forward_subgrid", "ehi_backpropagate", "ehi_residual_spectra",
    "ehi_multipliers_to_time", "ehi_misfit", "ehi_cg_init", "ehi_cg_shift_dot", "ehi_cg_update",
    "ehi_cg_direction", "ehi_mdot", "ehi_combine", "ehi_hbm_probe", "ehi_set_refinement",
)
PROF_KINDS = ("setup", "step", "dft", "herk", "factor", "solve", "model")
_PROF_N = 8


class EhiError(RuntimeError):
    def __init__(self, status: int, msg: str, bad_freq: int = -1):
        super().__init__(f"ehi status {status}: {msg}")
        self.status = status
        self.bad_freq = bad_freq


class SurveyDesc(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int32), ("nx", ctypes.c_int32), ("nb", ctypes.c_int32),
        ("h", ctypes.c_double), ("dt", ctypes.c_double),
        ("nt", ctypes.c_int32), ("stride", ctypes.c_int32), ("nr", ctypes.c_int32),
        ("rec_iz", ctypes.POINTER(ctypes.c_int32)), ("rec_ix", ctypes.POINTER(ctypes.c_int32)),
        ("nf", ctypes.c_int32), ("freq_hz", ctypes.POINTER(ctypes.c_double)),
        ("precision", ctypes.c_int32), ("max_ns", ctypes.c_int32), ("nr_batch", ctypes.c_int32),
        ("weighting", ctypes.c_int32), ("chunk", ctypes.c_int32),
        ("keep_z", ctypes.c_int32), ("keep_x", ctypes.c_int32), ("windows", ctypes.c_int32),
        ("decim", ctypes.c_int32), ("herk_split", ctypes.c_int32), ("herk_form", ctypes.c_int32),
    ]


_lib_handle = None


def lib() -> ctypes.CDLL:
    """Load libehi.so (once).  Raises if it has not been built."""
    global _lib_handle
    if _lib_handle is not None:
        return _lib_handle
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, st = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int
    L.ehi_workspace_bytes.argtypes = [ctypes.POINTER(SurveyDesc)]
    L.ehi_workspace_bytes.restype = ctypes.c_size_t
    L.ehi_create.argtypes = [ctypes.POINTER(SurveyDesc), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.ehi_create.restype = st
    L.ehi_build_green.argtypes = [vp, vp]
    L.ehi_build_green.restype = st
    L.ehi_build_hessian.argtypes = [vp]
    L.ehi_build_hessian.restype = st
    L.ehi_factor.argtypes = [vp, ctypes.c_double, ctypes.POINTER(i32)]
    L.ehi_factor.restype = st
    L.ehi_apply_multipliers.argtypes = [vp, vp, vp, i32, vp]
    L.ehi_apply_multipliers.restype = st
    L.ehi_lambda_max.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    L.ehi_lambda_max.restype = st
    for name in ("ehi_copy_green_dft", "ehi_copy_compressed", "ehi_load_green_dft", "ehi_copy_hessian",
                 "ehi_load_hessian", "ehi_copy_factor"):
        getattr(L, name).argtypes = [vp, vp]
        getattr(L, name).restype = st
    L.ehi_profile_enable.argtypes = [vp, ctypes.c_int]
    L.ehi_profile_enable.restype = st
    L.ehi_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.ehi_profile_read.restype = st
    L.ehi_batch_workspace_bytes.argtypes = [ctypes.POINTER(vp), i32]
    L.ehi_batch_workspace_bytes.restype = ctypes.c_size_t
    L.ehi_factor_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_double), vp,
                                   ctypes.c_size_t, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.ehi_factor_batch.restype = st
    L.ehi_factor_batch_static.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_double), vp,
                                          ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.ehi_factor_batch_static.restype = st
    L.ehi_set_stream.argtypes = [vp, vp]
    L.ehi_set_stream.restype = st
    L.ehi_set_launch.argtypes = [vp, i32, i32, i32]
    L.ehi_set_launch.restype = st
    L.ehi_get_launch.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.ehi_get_launch.restype = st
    L.ehi_set_medium.argtypes = [vp, vp]
    L.ehi_set_medium.restype = st
    for name in ("ehi_forward_subgrid", "ehi_backpropagate"):
        getattr(L, name).argtypes = [vp, vp, i32, vp]
        getattr(L, name).restype = st
    for name in ("ehi_residual_spectra", "ehi_multipliers_to_time"):
        getattr(L, name).argtypes = [vp, vp, i32, vp, vp]
        getattr(L, name).restype = st
    L.ehi_misfit.argtypes = [vp, vp, vp, i32, ctypes.c_int64, vp, vp, vp]
    L.ehi_misfit.restype = st
    i64, dbl = ctypes.c_int64, ctypes.c_double
    L.ehi_cg_init.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp]
    L.ehi_cg_shift_dot.argtypes = [vp, vp, dbl, i32, i64, vp, vp]
    L.ehi_cg_update.argtypes = [vp, vp, vp, vp, vp, vp, dbl, i32, i64, vp, vp, vp]
    L.ehi_cg_direction.argtypes = [vp, vp, vp, vp, i32, i64, vp]
    L.ehi_mdot.argtypes = [vp, i64, i32, vp, i32, i64, vp, vp]
    L.ehi_combine.argtypes = [vp, i64, i32, vp, i32, i64, dbl, vp, vp]
    for name in ("ehi_cg_init", "ehi_cg_shift_dot", "ehi_cg_update", "ehi_cg_direction", "ehi_mdot",
                 "ehi_combine"):
        getattr(L, name).restype = st
    L.ehi_set_refinement.argtypes = [vp, i32]
    L.ehi_set_refinement.restype = st
    L.ehi_hbm_probe.argtypes = [i32, vp, vp, vp, vp, vp, ctypes.c_size_t, ctypes.c_double, i32, vp, vp]
    L.ehi_hbm_probe.restype = st
    L.ehi_destroy.argtypes = [vp]
    L.ehi_destroy.restype = st
    L.ehi_last_error.argtypes = []
    L.ehi_last_error.restype = ctypes.c_char_p
    L.ehi_version.argtypes = []
    L.ehi_version.restype = ctypes.c_char_p
    _lib_handle = L
    return L


def _check(status: int, bad_freq: int = -1):
    if status != EHI_OK:
        raise EhiError(status, lib().ehi_last_error().decode(), bad_freq)


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _require(t: torch.Tensor, dtype, shape, name: str, device: torch.device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def make_desc(nz, nx, nb, h, dt, nt, stride, rec_iz, rec_ix, freqs_hz, precision, max_ns,
              nr_batch, weighting="long_record", chunk=0, keep=(0, 0), windows=1, decim=1,
              herk_split=0, herk_form=0):
    riz = np.ascontiguousarray(rec_iz, dtype=np.int32)
    rix = np.ascontiguousarray(rec_ix, dtype=np.int32)
    fr = np.ascontiguousarray(freqs_hz, dtype=np.float64)
    if riz.shape != rix.shape or riz.ndim != 1:
        raise ValueError("rec_iz and rec_ix must be 1-D arrays of equal length")
    prec = _PREC[precision] if isinstance(precision, str) else int(precision)
    d = SurveyDesc(nz=nz, nx=nx, nb=nb, h=h, dt=dt, nt=nt, stride=stride, nr=len(riz),
                   rec_iz=riz.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   rec_ix=rix.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                   nf=len(fr), freq_hz=fr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                   precision=prec, max_ns=max_ns, nr_batch=nr_batch,
                   weighting=_WEIGHT[weighting] if isinstance(weighting, str) else int(weighting),
                   chunk=int(chunk), keep_z=int(keep[0]), keep_x=int(keep[1]), windows=int(windows),
                   decim=int(decim), herk_split=int(herk_split), herk_form=int(herk_form))
    return d, (riz, rix, fr)   # keep the arrays alive with the descriptor


def workspace_bytes(**kw) -> int:
    d, keep = make_desc(**kw)
    n = lib().ehi_workspace_bytes(ctypes.byref(d))
    if n == 0:
        raise EhiError(EHI_EINVAL, lib().ehi_last_error().decode())
    return int(n)


class Survey:
    """One survey handle over a torch-allocated workspace on one GPU."""

    def __init__(self, *, nz: int, nx: int, nb: int, h: float, dt: float, nt: int, stride: int,
                 rec_iz: Sequence[int], rec_ix: Sequence[int], freqs_hz: Sequence[float],
                 precision="split_bf16", max_ns: int = 256, nr_batch: int = 0,
                 weighting="long_record", chunk: int = 0, keep=(0, 0), windows: int = 1, decim: int = 1,
                 herk_split: int = 0, herk_form: int = 0, workspace: Optional[torch.Tensor] = None,
                 device=None,
                 stream: Optional[torch.cuda.Stream] = None):
        self._h = None
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.nz, self.nx, self.nb, self.nt, self.stride = nz, nx, nb, nt, stride
        self.nr, self.nf = len(rec_ix), len(freqs_hz)
        self.nzs = (nz + stride - 1) // stride
        self.nxs = (nx + stride - 1) // stride
        self.precision = precision
        self.max_ns = max_ns
        self.nr_batch = nr_batch
        self.keep = (int(keep[0]), int(keep[1]))
        d, _alive = make_desc(nz, nx, nb, h, dt, nt, stride, rec_iz, rec_ix, freqs_hz, precision,
                              max_ns, nr_batch, weighting, chunk, keep, windows, decim, herk_split, herk_form)
        self.weighting = weighting
        L = lib()
        nbytes = L.ehi_workspace_bytes(ctypes.byref(d))
        if nbytes == 0:
            raise EhiError(EHI_EINVAL, L.ehi_last_error().decode())
        self.workspace_bytes = int(nbytes)
        with torch.cuda.device(self.device):
            if workspace is not None:
                # a caller-owned uint8 buffer (e.g. shared by surveys built in turn)
                if workspace.dtype != torch.uint8 or workspace.device != self.device or not workspace.is_contiguous():
                    raise ValueError("workspace must be a contiguous uint8 tensor on the survey's device")
                if workspace.numel() < nbytes + 256:
                    raise ValueError(f"workspace has {workspace.numel()} bytes, needs {nbytes + 256}")
                raw = workspace
            else:
                raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-raw.data_ptr()) % 256
            self._ws = raw
            self._ws_ptr = raw.data_ptr() + off
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h_out = ctypes.c_void_p()
            _check(L.ehi_create(ctypes.byref(d), ctypes.c_void_p(self._ws_ptr), ctypes.c_size_t(nbytes),
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h_out)))
        self._h = h_out

    # -- stages ---------------------------------------------------------------
    def build_green(self, vel: torch.Tensor):
        _require(vel, torch.float32, (self.nz, self.nx), "vel", self.device)
        self._vel = vel  # keep alive while the stream may still read it
        _check(lib().ehi_build_green(self._h, ctypes.c_void_p(vel.data_ptr())))

    def build_hessian(self):
        _check(lib().ehi_build_hessian(self._h))

    def factor(self, mu: float):
        bad = ctypes.c_int32(-1)
        st = lib().ehi_factor(self._h, ctypes.c_double(mu), ctypes.byref(bad))
        _check(st, bad.value)

    def apply_multipliers(self, resid: torch.Tensor, out: Optional[torch.Tensor] = None,
                          stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        if resid.dim() != 3:
            raise ValueError("resid must be [nf][ns][nr]")
        ns = resid.shape[1]
        _require(resid, torch.complex64, (self.nf, ns, self.nr), "resid", self.device)
        if out is None:
            out = torch.empty_like(resid)
        _require(out, torch.complex64, (self.nf, ns, self.nr), "out", self.device)
        sp = 0 if stream is None else stream.cuda_stream
        _check(lib().ehi_apply_multipliers(self._h, ctypes.c_void_p(resid.data_ptr()),
                                           ctypes.c_void_p(out.data_ptr()), ns, ctypes.c_void_p(sp)))
        return out

    def lambda_max(self) -> float:
        v = ctypes.c_double(0.0)
        _check(lib().ehi_lambda_max(self._h, ctypes.byref(v)))
        return float(v.value)

    # -- steps either side of the deblur, forward/adjoint modelling --------------
    def set_medium(self, vel: torch.Tensor):
        """Load the medium for forward_subgrid / backpropagate only."""
        _require(vel, torch.float32, (self.nz, self.nx), "vel", self.device)
        self._vel = vel
        _check(lib().ehi_set_medium(self._h, ctypes.c_void_p(vel.data_ptr())))

    def forward_subgrid(self, src: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """S src: ``src`` float32 [ns][nt][nzs][nxs] -> traces [ns][nr][nt]."""
        ns = src.shape[0]
        _require(src, torch.float32, (ns, self.nt, self.nzs, self.nxs), "src", self.device)
        if out is None:
            out = torch.empty((ns, self.nr, self.nt), dtype=torch.float32, device=self.device)
        _require(out, torch.float32, (ns, self.nr, self.nt), "out", self.device)
        _check(lib().ehi_forward_subgrid(self._h, ctypes.c_void_p(src.data_ptr()), ns,
                                         ctypes.c_void_p(out.data_ptr())))
        return out

    def backpropagate(self, data: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """S^T data: traces float32 [ns][nr][nt] -> subgrid source [ns][nt][nzs][nxs]."""
        ns = data.shape[0]
        _require(data, torch.float32, (ns, self.nr, self.nt), "data", self.device)
        if out is None:
            out = torch.empty((ns, self.nt, self.nzs, self.nxs), dtype=torch.float32, device=self.device)
        _require(out, torch.float32, (ns, self.nt, self.nzs, self.nxs), "out", self.device)
        _check(lib().ehi_backpropagate(self._h, ctypes.c_void_p(data.data_ptr()), ns,
                                       ctypes.c_void_p(out.data_ptr())))
        return out

    def residual_spectra(self, dres: torch.Tensor, out: Optional[torch.Tensor] = None,
                         stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """Time-domain residuals float32 [ns][nr][nt] -> complex64 [nf][ns][nr]."""
        ns = dres.shape[0]
        _require(dres, torch.float32, (ns, self.nr, self.nt), "dres", self.device)
        if out is None:
            out = torch.empty((self.nf, ns, self.nr), dtype=torch.complex64, device=self.device)
        _require(out, torch.complex64, (self.nf, ns, self.nr), "out", self.device)
        sp = 0 if stream is None else stream.cuda_stream
        _check(lib().ehi_residual_spectra(self._h, ctypes.c_void_p(dres.data_ptr()), ns,
                                          ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(sp)))
        return out

    def multipliers_to_time(self, X: torch.Tensor, out: Optional[torch.Tensor] = None,
                            stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """Multipliers complex64 [nf][ns][nr] (frequencies = bins of the
        2nt-point transform) -> float32 [ns][nr][nt]."""
        if X.dim() != 3:
            raise ValueError("X must be [nf][ns][nr]")
        ns = X.shape[1]
        _require(X, torch.complex64, (self.nf, ns, self.nr), "X", self.device)
        if out is None:
            out = torch.empty((ns, self.nr, self.nt), dtype=torch.float32, device=self.device)
        _require(out, torch.float32, (ns, self.nr, self.nt), "out", self.device)
        sp = 0 if stream is None else stream.cuda_stream
        _check(lib().ehi_multipliers_to_time(self._h, ctypes.c_void_p(X.data_ptr()), ns,
                                             ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(sp)))
        return out

    # -- stage inputs/outputs ------------------------------------------------------
    def copy_green_dft(self) -> torch.Tensor:
        out = torch.empty((self.nf, self.nr, self.nzs, self.nxs), dtype=torch.complex64, device=self.device)
        _check(lib().ehi_copy_green_dft(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def copy_compressed(self) -> torch.Tensor:
        """Compressed spectra of a compressed survey: complex64 [nf][nr][keep_z][keep_x]."""
        kz, kx = self.keep
        out = torch.empty((self.nf, self.nr, kz, kx), dtype=torch.complex64, device=self.device)
        _check(lib().ehi_copy_compressed(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def load_green_dft(self, g: torch.Tensor):
        _require(g, torch.complex64, (self.nf, self.nr, self.nzs, self.nxs), "ghat", self.device)
        self._ghat_in = g
        _check(lib().ehi_load_green_dft(self._h, ctypes.c_void_p(g.data_ptr())))

    def copy_hessian(self) -> torch.Tensor:
        out = torch.empty((self.nf, self.nr, self.nr), dtype=torch.complex128, device=self.device)
        _check(lib().ehi_copy_hessian(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def load_hessian(self, H: torch.Tensor):
        _require(H, torch.complex128, (self.nf, self.nr, self.nr), "hessian", self.device)
        self._h_in = H
        _check(lib().ehi_load_hessian(self._h, ctypes.c_void_p(H.data_ptr())))

    def copy_factor(self) -> torch.Tensor:
        out = torch.empty((self.nf, self.nr, self.nr), dtype=torch.complex128, device=self.device)
        _check(lib().ehi_copy_factor(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def set_refinement(self, steps: int):
        """FP64-residual refinement steps of each deblur (split-BF16 form; default 1)."""
        _check(lib().ehi_set_refinement(self._h, int(steps)))

    def set_stream(self, stream: Optional[torch.cuda.Stream]):
        """Route this survey's later work to ``stream`` (None = the default stream)."""
        _check(lib().ehi_set_stream(self._h, ctypes.c_void_p(0 if stream is None else stream.cuda_stream)))
        self.stream = stream

    def set_launch(self, tblock: int = 0, seg_rows: int = 0, band: int = -1):
        """Marching launch shape; 0 keeps tblock / seg_rows, band 0 = automatic,
        band -1 keeps the current band request."""
        _check(lib().ehi_set_launch(self._h, int(tblock), int(seg_rows), int(band)))

    def get_launch(self) -> tuple:
        """(time levels per marching launch, rows per marching segment, band width)."""
        tb, sr, bw = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().ehi_get_launch(self._h, ctypes.byref(tb), ctypes.byref(sr), ctypes.byref(bw)))
        return int(tb.value), int(sr.value), int(bw.value)

    # -- kernel timing -------------------------------------------------------------
    def profile(self, enable: bool = True):
        _check(lib().ehi_profile_enable(self._h, 1 if enable else 0))

    def read_profile(self) -> dict:
        """{kind: (milliseconds, launches)} of the runs recorded since the last read."""
        ms = (ctypes.c_double * _PROF_N)()
        nl = (ctypes.c_int64 * _PROF_N)()
        _check(lib().ehi_profile_read(self._h, ms, nl))
        return {k: (float(ms[i]), int(nl[i])) for i, k in enumerate(PROF_KINDS)}

    def close(self, sync: bool = True):
        """Release the handle and the workspace.  With ``sync=False`` the caller
        guarantees that no enqueued work still reads or writes the survey."""
        if self._h is not None:
            if sync:
                torch.cuda.synchronize(self.device)
            lib().ehi_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            if self._h is not None:
                lib().ehi_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def misfit(dd: torch.Tensor, pred: torch.Tensor, obs: torch.Tensor, err: Optional[torch.Tensor] = None,
           stream: Optional[torch.cuda.Stream] = None):
    """(err = dd - pred, relerr[s] = sum err^2 / sum obs^2) for float32 records
    [ns][...] of equal shape on one device; relerr float64 [ns]."""
    if dd.shape != pred.shape or dd.shape != obs.shape:
        raise ValueError("dd, pred and obs must have the same shape")
    ns = dd.shape[0]
    dev = dd.device
    for t, n in ((dd, "dd"), (pred, "pred"), (obs, "obs")):
        _require(t, torch.float32, dd.shape, n, dev)
    if err is None:
        err = torch.empty_like(dd)
    _require(err, torch.float32, dd.shape, "err", dev)
    rel = torch.empty(ns, dtype=torch.float64, device=dev)
    n_per = dd.numel() // max(ns, 1)
    sp = 0 if stream is None else stream.cuda_stream
    _check(lib().ehi_misfit(ctypes.c_void_p(dd.data_ptr()), ctypes.c_void_p(pred.data_ptr()),
                            ctypes.c_void_p(obs.data_ptr()), ns, n_per, ctypes.c_void_p(err.data_ptr()),
                            ctypes.c_void_p(rel.data_ptr()), ctypes.c_void_p(sp)))
    return err, rel


def factor_batch(surveys: Sequence["Survey"], mu: Sequence[float],
                 stream: Optional[torch.cuda.Stream] = None):
    """Factor several surveys in one launch (uneven sizes).  The surveys'
    streams are synchronised first.  Raises EhiError (with .bad_survey and
    .bad_freq) on a non-positive pivot."""
    if len(surveys) != len(mu) or not surveys:
        raise ValueError("one mu per survey")
    L = lib()
    for sv in surveys:
        torch.cuda.synchronize(sv.device)
    handles = (ctypes.c_void_p * len(surveys))(*[sv._h.value for sv in surveys])
    nbytes = L.ehi_batch_workspace_bytes(handles, len(surveys))
    if nbytes == 0:
        raise EhiError(EHI_EINVAL, L.ehi_last_error().decode())
    dev = surveys[0].device
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    ptr = ws.data_ptr() + (-ws.data_ptr()) % 256
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    mus = (ctypes.c_double * len(mu))(*[float(m) for m in mu])
    bs, bf = ctypes.c_int32(-1), ctypes.c_int32(-1)
    rc = L.ehi_factor_batch(handles, len(surveys), mus, ctypes.c_void_p(ptr), ctypes.c_size_t(nbytes),
                            ctypes.c_void_p(st.cuda_stream), ctypes.byref(bs), ctypes.byref(bf))
    if rc != EHI_OK:
        err = EhiError(rc, L.ehi_last_error().decode(), bf.value)
        err.bad_survey = bs.value
        raise err


def factor_batch_static(surveys: Sequence["Survey"], mu: Sequence[float],
                        stream: Optional[torch.cuda.Stream] = None):
    """``factor_batch`` with the library's static job table (no device
    allocation: ehi_factor_batch_static); at most 4096 (survey, frequency)
    jobs, all surveys on the current device."""
    if len(surveys) != len(mu) or not surveys:
        raise ValueError("one mu per survey")
    L = lib()
    for sv in surveys:
        torch.cuda.synchronize(sv.device)
    handles = (ctypes.c_void_p * len(surveys))(*[sv._h.value for sv in surveys])
    st = stream if stream is not None else torch.cuda.current_stream(surveys[0].device)
    mus = (ctypes.c_double * len(mu))(*[float(m) for m in mu])
    bs, bf = ctypes.c_int32(-1), ctypes.c_int32(-1)
    rc = L.ehi_factor_batch_static(handles, len(surveys), mus, ctypes.c_void_p(st.cuda_stream),
                                   ctypes.byref(bs), ctypes.byref(bf))
    if rc != EHI_OK:
        err = EhiError(rc, L.ehi_last_error().decode(), bf.value)
        err.bad_survey = bs.value
        raise err


def survey_from(spec, precision="split_bf16", max_ns=None, nr_batch=0, **kw) -> Survey:
    """Build a handle from any object with the survey attributes (nz, nx, nb, h,
    dt, nt, stride, rec_iz, rec_ix, freqs_hz, ns)."""
    return Survey(nz=spec.nz, nx=spec.nx, nb=spec.nb, h=spec.h, dt=spec.dt, nt=spec.nt,
                  stride=spec.stride, rec_iz=spec.rec_iz, rec_ix=spec.rec_ix,
                  freqs_hz=spec.freqs_hz, precision=precision,
                  max_ns=max_ns if max_ns is not None else max(1, spec.ns),
                  nr_batch=nr_batch, **kw)


def hbm_probe(mode: int, a: torch.Tensor, b=None, c=None, d=None, e=None, e_frac: float = 0.0,
              grid: int = 8192, sink=None, stream: Optional[torch.cuda.Stream] = None):
    """Enqueue one streaming probe launch (ehi_hbm_probe) over equally sized
    uint8 device tensors a..e (unused ones may be None)."""
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)
    _check(lib().ehi_hbm_probe(int(mode), ptr(a), ptr(b), ptr(c), ptr(d), ptr(e), ctypes.c_size_t(a.numel()),
                               ctypes.c_double(e_frac), int(grid), ptr(sink), ctypes.c_void_p(_stream_ptr(stream))))
