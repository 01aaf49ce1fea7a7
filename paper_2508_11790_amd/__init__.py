"""Windowed beamspace MVDR beamforming on AMD MI355X (gfx950).

Python binding of the C ABI in ``include/wbmvdr.h``: argument marshalling only.  Every step
of the computation runs in the library's HIP kernels; PyTorch provides device memory
(tensors) and streams.  The method follows "Scaling Wideband Massive MIMO Radar via Beamspace
Dimension Reduction" (Sec. III): FFT channelizer, zero-padded spatial DFT, per-target W-bin
beamspace window, loaded sample covariance and MVDR correlator per (target, subband).
"""

from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import FORM_FUSED, FORM_GRAPH, FORM_PLAIN, WbmError  # noqa: F401

__all__ = ["Plan", "WbmError", "FORM_PLAIN", "FORM_FUSED", "FORM_GRAPH", "version"]

_FORMS = {"plain": FORM_PLAIN, "fused": FORM_FUSED, "graph": FORM_GRAPH}


def version() -> str:
    return _lib.load().wbm_version().decode()


def _torch():
    import torch
    return torch


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(stream) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_tensor(t, name, shape, dtype, device):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError(f"{name} must be on the plan's GPU")


class Plan:
    """One problem shape: N elements, M-point spatial DFT, K subbands, L train / Lt test
    snapshots, up to ``max_targets`` targets with windows up to ``w_max`` bins."""

    def __init__(self, N: int, M: int, K: int, L: int, Lt: int, max_targets: int, w_max: int,
                 beta: float = 0.2, d_over_lambda: float = 0.5, half_bin: bool = False):
        lib = _lib.load()
        torch = _torch()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.cfg = _lib.WbmConfig(N, M, K, L, Lt, max_targets, w_max,
                                  _lib.WBM_HALF_BIN if half_bin else 0, beta, d_over_lambda)
        self.N, self.M, self.K, self.L, self.Lt = N, M, K, L, Lt
        self.B = L + Lt
        self.S = self.B * K
        self.max_targets, self.w_max = max_targets, w_max
        h = C.c_void_p()
        _lib.check(lib.wbm_plan_create(C.byref(self.cfg), C.byref(h)))
        self._h = h

    @property
    def workspace_bytes(self) -> int:
        return int(_lib.load().wbm_plan_workspace_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().wbm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ helpers
    def _targets(self, az_rad, win):
        az = np.ascontiguousarray(np.asarray(az_rad, dtype=np.float64).ravel())
        T = int(az.size)
        w = None
        if win is not None:
            w = np.ascontiguousarray(np.asarray(win, dtype=np.int32).ravel())
            if w.size != T:
                raise ValueError("win must have one entry per target")
        return az, w, T

    def _x(self, x):
        torch = _torch()
        _check_tensor(x, "x", (self.N, self.S), torch.complex64, self.device)

    # ------------------------------------------------------------------ entry points
    def beamform(self, x, az_rad: Sequence[float], win: Optional[Sequence[int]], loading: float,
                 form: str = "fused", out=None, weights=None, starts=None, info=None,
                 want_weights: bool = True, want_starts: bool = True, stream=None):
        """Windowed beamspace MVDR of every (target, subband) pair; returns a dict of tensors
        ``out`` [T, K, Lt] complex64, ``weights`` [T, K, w_max], ``starts`` [T, K] int32,
        ``info`` [T, K] int32 (each optional output only if requested / passed)."""
        torch = _torch()
        self._x(x)
        az, w, T = self._targets(az_rad, win)
        dev = self.device
        if out is None:
            out = torch.empty((T, self.K, self.Lt), dtype=torch.complex64, device=dev)
        if weights is None and want_weights:
            weights = torch.empty((T, self.K, self.w_max), dtype=torch.complex64, device=dev)
        if starts is None and want_starts:
            starts = torch.empty((T, self.K), dtype=torch.int32, device=dev)
        if info is None:
            info = torch.empty((T, self.K), dtype=torch.int32, device=dev)
        _check_tensor(out, "out", (T, self.K, self.Lt), torch.complex64, dev)
        if weights is not None:
            _check_tensor(weights, "weights", (T, self.K, self.w_max), torch.complex64, dev)
        if starts is not None:
            _check_tensor(starts, "starts", (T, self.K), torch.int32, dev)
        _check_tensor(info, "info", (T, self.K), torch.int32, dev)
        _lib.check(_lib.load().wbm_beamform(
            self._h, _ptr(x), az.ctypes.data, None if w is None else w.ctypes.data, T,
            float(loading), _FORMS[form], _ptr(out), _ptr(weights), _ptr(starts), _ptr(info),
            _stream(stream)))
        return dict(out=out, weights=weights, starts=starts, info=info)

    def channelize(self, x, X=None, stream=None):
        """FFT channelizer: x [N, S] -> X [K, B, N] complex64."""
        torch = _torch()
        self._x(x)
        if X is None:
            X = torch.empty((self.K, self.B, self.N), dtype=torch.complex64, device=self.device)
        _check_tensor(X, "X", (self.K, self.B, self.N), torch.complex64, self.device)
        _lib.check(_lib.load().wbm_channelize(self._h, _ptr(x), _ptr(X), _stream(stream)))
        return X

    def beamspace(self, X, Y=None, stream=None):
        """Zero-padded spatial DFT: X [K, B, N] -> Y [K, M, B] complex64."""
        torch = _torch()
        _check_tensor(X, "X", (self.K, self.B, self.N), torch.complex64, self.device)
        if Y is None:
            Y = torch.empty((self.K, self.M, self.B), dtype=torch.complex64, device=self.device)
        _check_tensor(Y, "Y", (self.K, self.M, self.B), torch.complex64, self.device)
        _lib.check(_lib.load().wbm_beamspace(self._h, _ptr(X), _ptr(Y), _stream(stream)))
        return Y

    def steer(self, az_rad, win, stream=None):
        """Window starts [T, K] int32 and windowed steering vectors [T, K, w_max] complex128."""
        torch = _torch()
        az, w, T = self._targets(az_rad, win)
        starts = torch.empty((T, self.K), dtype=torch.int32, device=self.device)
        abar = torch.empty((T, self.K, self.w_max), dtype=torch.complex128, device=self.device)
        _lib.check(_lib.load().wbm_steer(self._h, az.ctypes.data,
                                         None if w is None else w.ctypes.data, T, _ptr(starts),
                                         _ptr(abar), _stream(stream)))
        return starts, abar

    STAGES = ("steer", "channelize", "beamspace", "mvdr")

    def stage_times(self, x, az_rad, win, loading: float, reps: int = 20, stream=None):
        """Average milliseconds per kernel of the fused sequence, timed with HIP events."""
        self._x(x)
        az, w, T = self._targets(az_rad, win)
        ms = np.zeros(4, dtype=np.float64)
        _lib.check(_lib.load().wbm_stage_times(self._h, _ptr(x), az.ctypes.data,
                                               None if w is None else w.ctypes.data, T,
                                               float(loading), int(reps), ms.ctypes.data,
                                               _stream(stream)))
        return dict(zip(self.STAGES, ms.tolist()))

    def full_mvdr(self, x, az_rad, loading: float, want_weights: bool = True, stream=None):
        """Full-dimensional element-space MVDR per subband: out [T, K, Lt], weights [T, K, N],
        info [K]."""
        torch = _torch()
        self._x(x)
        az, _, T = self._targets(az_rad, None)
        out = torch.empty((T, self.K, self.Lt), dtype=torch.complex64, device=self.device)
        weights = (torch.empty((T, self.K, self.N), dtype=torch.complex64, device=self.device)
                   if want_weights else None)
        info = torch.empty((self.K,), dtype=torch.int32, device=self.device)
        _lib.check(_lib.load().wbm_full_mvdr(self._h, _ptr(x), az.ctypes.data, T, float(loading),
                                             _ptr(out), _ptr(weights), _ptr(info),
                                             _stream(stream)))
        return dict(out=out, weights=weights, info=info)
