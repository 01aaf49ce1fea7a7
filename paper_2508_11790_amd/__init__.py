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

__all__ = ["Plan", "Mlp", "WbmError", "FORM_PLAIN", "FORM_FUSED", "FORM_GRAPH", "version",
           "MLP_PARAMS", "MLP_STATIC_MAX_BATCH", "mlp_grad_static"]

MLP_PARAMS = _lib.MLP_PARAMS

_FORMS = {"plain": FORM_PLAIN, "fused": FORM_FUSED, "graph": FORM_GRAPH,
          "mixed": _lib.FORM_MIXED, "mixed_bf16": _lib.FORM_MIXED_BF16,
          "fused_f32": _lib.FORM_FUSED_F32, "graph_f32": _lib.FORM_GRAPH_F32}
# precision of the fused sequence a launch configuration applies to: "ext" (fused / graph /
# learned forms) or "f32" (fused_f32 / graph_f32, the mixed forms' transforms, planar array)
_PRECS = {"ext": _lib.PREC_EXT, "f32": _lib.PREC_F32, "mixed": _lib.PREC_MIXED,
          "mixed_bf16": _lib.PREC_MIXED_BF16}
INFO_ROUTED = _lib.INFO_ROUTED
INFO_WIDTH = _lib.INFO_WIDTH


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

    _PAIR_KERNELS = {"mfma": _lib.PAIR_MFMA, "wave": _lib.PAIR_WAVE, "block": _lib.PAIR_BLOCK,
                     "resident": _lib.PAIR_RESIDENT}

    def set_tuning(self, chan_logtile: int, beam_logtile: int, pair_kernel: str = "block",
                   overlap: int = 1, precision: str = "ext"):
        """Pin the fused sequence's FFT tiles (log2 complex per workgroup: 11..13, or 10..13 in
        extended precision), pair kernel ("mfma", "wave", "block" or "resident"; extended
        precision: "wave" or "block") and subband chunks overlapping the spatial DFT with the
        pair kernel (1, 2, 4, 8) for one precision ("ext" or "f32"); skips that precision's
        first-call timing search."""
        if pair_kernel not in self._PAIR_KERNELS:
            raise ValueError(f"pair_kernel must be one of {sorted(self._PAIR_KERNELS)}")
        _lib.check(_lib.load().wbm_plan_set_tuning(self._h, _PRECS[precision], int(chan_logtile),
                                                   int(beam_logtile),
                                                   self._PAIR_KERNELS[pair_kernel], int(overlap)))

    def get_tuning(self, precision: str = "ext"):
        """(chan_logtile, beam_logtile, pair_kernel name, overlap chunks) of one precision."""
        c, b, p, o = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _lib.check(_lib.load().wbm_plan_get_tuning(self._h, _PRECS[precision], C.byref(c),
                                                   C.byref(b), C.byref(p), C.byref(o)))
        name = {v: k for k, v in self._PAIR_KERNELS.items()}[p.value]
        return int(c.value), int(b.value), name, int(o.value)

    @property
    def tuning(self):
        """Launch configuration of the extended-precision fused sequence (get_tuning("ext"))."""
        return self.get_tuning("ext")

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

    def lift(self, weights, starts, c_hat=None, stream=None):
        """Lifted correlators (Eq. 21) of every pair: weights [T, K, w_max] complex64 and
        starts [T, K] int32 (as beamform returns them) -> c_hat [T, K, N] complex64."""
        torch = _torch()
        T = int(weights.shape[0])
        _check_tensor(weights, "weights", (T, self.K, self.w_max), torch.complex64, self.device)
        _check_tensor(starts, "starts", (T, self.K), torch.int32, self.device)
        if c_hat is None:
            c_hat = torch.empty((T, self.K, self.N), dtype=torch.complex64, device=self.device)
        _check_tensor(c_hat, "c_hat", (T, self.K, self.N), torch.complex64, self.device)
        _lib.check(_lib.load().wbm_lift(self._h, _ptr(weights), _ptr(starts), T, _ptr(c_hat),
                                        _stream(stream)))
        return c_hat

    def apply_lifted(self, x, c_hat, out=None, stream=None):
        """Beam outputs of lifted correlators applied in element space to the test snapshots:
        x [N, S] and c_hat [T, K, N] -> out [T, K, Lt] complex64 (channelizes x itself)."""
        torch = _torch()
        self._x(x)
        T = int(c_hat.shape[0])
        _check_tensor(c_hat, "c_hat", (T, self.K, self.N), torch.complex64, self.device)
        if out is None:
            out = torch.empty((T, self.K, self.Lt), dtype=torch.complex64, device=self.device)
        _check_tensor(out, "out", (T, self.K, self.Lt), torch.complex64, self.device)
        _lib.check(_lib.load().wbm_apply_lifted(self._h, _ptr(x), _ptr(c_hat), T, _ptr(out),
                                                _stream(stream)))
        return out

    def synthesize(self, out, z=None, stream=None):
        """Subband synthesis (inverse channelizer per test block): out [T, K, Lt] -> z [T, Lt*K]
        complex64, the wideband beam output of every target."""
        torch = _torch()
        T = int(out.shape[0])
        _check_tensor(out, "out", (T, self.K, self.Lt), torch.complex64, self.device)
        if z is None:
            z = torch.empty((T, self.Lt * self.K), dtype=torch.complex64, device=self.device)
        _check_tensor(z, "z", (T, self.Lt * self.K), torch.complex64, self.device)
        _lib.check(_lib.load().wbm_synthesize(self._h, _ptr(out), T, _ptr(z), _stream(stream)))
        return z

    def beam_pattern(self, c, omega, pattern=None, stream=None):
        """Beam patterns (Eq. 22): c [..., N] complex64 correlators, omega [Q] float64 angles
        (device) -> pattern [..., Q] float32 cosine similarities with the element steering."""
        torch = _torch()
        if c.dtype != torch.complex64 or c.shape[-1] != self.N or not c.is_contiguous():
            raise ValueError(f"c must be contiguous complex64 [..., {self.N}]")
        _check_tensor(omega, "omega", (int(omega.numel()),), torch.float64, self.device)
        pairs, Q = int(c.numel() // self.N), int(omega.numel())
        if pattern is None:
            pattern = torch.empty((*c.shape[:-1], Q), dtype=torch.float32, device=self.device)
        _check_tensor(pattern, "pattern", (*c.shape[:-1], Q), torch.float32, self.device)
        _lib.check(_lib.load().wbm_beam_pattern(self._h, _ptr(c), pairs, _ptr(omega), Q,
                                                _ptr(pattern), _stream(stream)))
        return pattern

    def range_doppler(self, z, chirp, R: int, P: int, guard: int = 2, train: int = 8,
                      threshold_db: float = 10.0, stream=None):
        """Range-Doppler power maps and 1-D CFAR detections of pulse trains: z [T, >= P R]
        complex64 (P pulses of R samples), chirp [Lp] complex64 -> (power [T, R, P] float32,
        det [T, R, P] uint8)."""
        torch = _torch()
        if z.dtype != torch.complex64 or z.dim() != 2 or not z.is_contiguous():
            raise ValueError("z must be a contiguous complex64 [T, S] tensor")
        _check_tensor(chirp, "chirp", (int(chirp.numel()),), torch.complex64, self.device)
        T, Lp = int(z.shape[0]), int(chirp.numel())
        F = 1
        while F < R + Lp - 1:
            F *= 2
        work = torch.empty(T * P * R + 2 * F + P, dtype=torch.complex64, device=self.device)
        power = torch.empty((T, R, P), dtype=torch.float32, device=self.device)
        det = torch.empty((T, R, P), dtype=torch.uint8, device=self.device)
        _lib.check(_lib.load().wbm_range_doppler(
            self._h, _ptr(z), T, int(z.shape[1]), _ptr(chirp), Lp, int(R), int(P), int(guard),
            int(train), float(threshold_db), _ptr(work), _ptr(power), _ptr(det),
            _stream(stream)))
        return power, det

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

    # ------------------------------------------------------------------ planar array
    def _upa_targets(self, az_rad, el_rad, win_z, win_x):
        az = np.ascontiguousarray(np.asarray(az_rad, dtype=np.float64).ravel())
        el = np.ascontiguousarray(np.asarray(el_rad, dtype=np.float64).ravel())
        wz = np.ascontiguousarray(np.asarray(win_z, dtype=np.int32).ravel())
        wx = np.ascontiguousarray(np.asarray(win_x, dtype=np.int32).ravel())
        T = int(az.size)
        if not (el.size == wz.size == wx.size == T):
            raise ValueError("el_rad, win_z and win_x must have one entry per target")
        return az, el, wz, wx, T

    def beamform_upa(self, x, nz: int, mz: int, az_rad, el_rad, win_z, win_x, loading: float,
                     form: str = "fused", out=None, weights=None, starts=None, info=None,
                     want_weights: bool = True, want_starts: bool = True, stream=None):
        """Windowed beamspace MVDR on an nz x (N / nz) planar array with an mz x (M / mz) beam
        grid; returns ``out`` [T, K, Lt], ``weights`` [T, K, w_max] (window cells, z fastest),
        ``starts`` [T, K, 2] int32 (s_z, s_x) and ``info`` [T, K]."""
        torch = _torch()
        self._x(x)
        az, el, wz, wx, T = self._upa_targets(az_rad, el_rad, win_z, win_x)
        dev = self.device
        if out is None:
            out = torch.empty((T, self.K, self.Lt), dtype=torch.complex64, device=dev)
        if weights is None and want_weights:
            weights = torch.empty((T, self.K, self.w_max), dtype=torch.complex64, device=dev)
        if starts is None and want_starts:
            starts = torch.empty((T, self.K, 2), dtype=torch.int32, device=dev)
        if info is None:
            info = torch.empty((T, self.K), dtype=torch.int32, device=dev)
        _check_tensor(out, "out", (T, self.K, self.Lt), torch.complex64, dev)
        if weights is not None:
            _check_tensor(weights, "weights", (T, self.K, self.w_max), torch.complex64, dev)
        if starts is not None:
            _check_tensor(starts, "starts", (T, self.K, 2), torch.int32, dev)
        _check_tensor(info, "info", (T, self.K), torch.int32, dev)
        _lib.check(_lib.load().wbm_beamform_upa(
            self._h, _ptr(x), int(nz), int(mz), az.ctypes.data, el.ctypes.data, wz.ctypes.data,
            wx.ctypes.data, T, float(loading), _FORMS[form], _ptr(out), _ptr(weights),
            _ptr(starts), _ptr(info), _stream(stream)))
        return dict(out=out, weights=weights, starts=starts, info=info)

    def beamspace_upa(self, X, nz: int, mz: int, Y=None, stream=None):
        """Planar beamspace: X [K, B, N] -> Y [K, M, B] complex64, beam (mz, mx) at mx * Mz + mz."""
        torch = _torch()
        _check_tensor(X, "X", (self.K, self.B, self.N), torch.complex64, self.device)
        if Y is None:
            Y = torch.empty((self.K, self.M, self.B), dtype=torch.complex64, device=self.device)
        _check_tensor(Y, "Y", (self.K, self.M, self.B), torch.complex64, self.device)
        _lib.check(_lib.load().wbm_beamspace_upa(self._h, _ptr(X), int(nz), int(mz), _ptr(Y),
                                                 _stream(stream)))
        return Y

    def steer_upa(self, nz: int, mz: int, az_rad, el_rad, win_z, win_x, stream=None):
        """Planar window starts [T, K, 2] int32 (s_z, s_x) and windowed steering [T, K, w_max]
        complex128."""
        torch = _torch()
        az, el, wz, wx, T = self._upa_targets(az_rad, el_rad, win_z, win_x)
        starts = torch.empty((T, self.K, 2), dtype=torch.int32, device=self.device)
        abar = torch.empty((T, self.K, self.w_max), dtype=torch.complex128, device=self.device)
        _lib.check(_lib.load().wbm_steer_upa(self._h, int(nz), int(mz), az.ctypes.data,
                                             el.ctypes.data, wz.ctypes.data, wx.ctypes.data, T,
                                             _ptr(starts), _ptr(abar), _stream(stream)))
        return starts, abar

    def lift_upa(self, weights, starts, nz: int, mz: int, win_z, c_hat=None, stream=None):
        """Planar lifted correlators (Eq. 21): weights [T, K, w_max], starts [T, K, 2] int32 (as
        beamform_upa returns them), win_z [T] -> c_hat [T, K, N] complex64."""
        torch = _torch()
        T = int(weights.shape[0])
        _check_tensor(weights, "weights", (T, self.K, self.w_max), torch.complex64, self.device)
        _check_tensor(starts, "starts", (T, self.K, 2), torch.int32, self.device)
        wz = torch.as_tensor(np.asarray(win_z, dtype=np.int32).ravel()).to(self.device)
        if wz.numel() != T:
            raise ValueError("win_z must have one entry per target")
        if c_hat is None:
            c_hat = torch.empty((T, self.K, self.N), dtype=torch.complex64, device=self.device)
        _check_tensor(c_hat, "c_hat", (T, self.K, self.N), torch.complex64, self.device)
        _lib.check(_lib.load().wbm_lift_upa(self._h, _ptr(weights), _ptr(starts), int(nz),
                                            int(mz), _ptr(wz), T, _ptr(c_hat), _stream(stream)))
        return c_hat

    def beam_pattern_upa(self, c, nz: int, omega, pattern=None, stream=None):
        """Planar beam patterns (Eq. 22): c [..., N] complex64 correlators, omega [Q, 2] float64
        (Omega_z, Omega_x) on the device -> pattern [..., Q] float32."""
        torch = _torch()
        if c.dtype != torch.complex64 or c.shape[-1] != self.N or not c.is_contiguous():
            raise ValueError(f"c must be contiguous complex64 [..., {self.N}]")
        Q = int(omega.shape[0]) if omega.dim() == 2 else -1
        _check_tensor(omega, "omega", (Q, 2), torch.float64, self.device)
        pairs = int(c.numel() // self.N)
        if pattern is None:
            pattern = torch.empty((*c.shape[:-1], Q), dtype=torch.float32, device=self.device)
        _check_tensor(pattern, "pattern", (*c.shape[:-1], Q), torch.float32, self.device)
        _lib.check(_lib.load().wbm_beam_pattern_upa(self._h, _ptr(c), pairs, int(nz), _ptr(omega),
                                                    Q, _ptr(pattern), _stream(stream)))
        return pattern

    STAGES = ("steer", "channelize", "beamspace", "mvdr")

    def stage_times(self, x, az_rad, win, loading: float, reps: int = 20, stream=None,
                    precision: str = "ext"):
        """Average milliseconds per kernel of the fused sequence in one precision ("ext": the
        fused form, "f32": fused_f32, "mixed" / "mixed_bf16": the mixed forms, whose pair stage
        is the MFMA kernel plus the FP64 re-solve of routed windows), timed with HIP events."""
        self._x(x)
        az, w, T = self._targets(az_rad, win)
        ms = np.zeros(4, dtype=np.float64)
        _lib.check(_lib.load().wbm_stage_times(self._h, _ptr(x), az.ctypes.data,
                                               None if w is None else w.ctypes.data, T,
                                               float(loading), _PRECS[precision], int(reps),
                                               ms.ctypes.data, _stream(stream)))
        return dict(zip(self.STAGES, ms.tolist()))

    # ------------------------------------------------------------------ loading / window predictor
    def profiles(self, x, az_rad, noise_power: float = 1.0, stream=None):
        """Network input of every pair: [T, K, 64] float32 log10 training power profile."""
        torch = _torch()
        self._x(x)
        az, _, T = self._targets(az_rad, None)
        feat = torch.empty((T, self.K, 64), dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().wbm_profiles(self._h, _ptr(x), az.ctypes.data, T, float(noise_power),
                                            _ptr(feat), _stream(stream)))
        return feat

    def beamform_pairs(self, x, az_rad, win, pair_win, pair_loading, out=None, weights=None,
                       starts=None, info=None, stream=None):
        """Windowed MVDR with a window width (int32 [T, K]) and loading (float32 [T, K]) per
        pair; win [T] is the window gathered per target (sub-windows are centred in it)."""
        torch = _torch()
        self._x(x)
        az, w, T = self._targets(az_rad, win)
        dev = self.device
        _check_tensor(pair_win, "pair_win", (T, self.K), torch.int32, dev)
        _check_tensor(pair_loading, "pair_loading", (T, self.K), torch.float32, dev)
        out = torch.empty((T, self.K, self.Lt), dtype=torch.complex64, device=dev) if out is None else out
        weights = (torch.empty((T, self.K, self.w_max), dtype=torch.complex64, device=dev)
                   if weights is None else weights)
        starts = torch.empty((T, self.K), dtype=torch.int32, device=dev) if starts is None else starts
        info = torch.empty((T, self.K), dtype=torch.int32, device=dev) if info is None else info
        _lib.check(_lib.load().wbm_beamform_pairs(
            self._h, _ptr(x), az.ctypes.data, None if w is None else w.ctypes.data, T,
            _ptr(pair_win), _ptr(pair_loading), _ptr(out), _ptr(weights), _ptr(starts), _ptr(info),
            _stream(stream)))
        return dict(out=out, weights=weights, starts=starts, info=info)

    def beamform_learned(self, x, az_rad, params, noise_power: float = 1.0, fallback_win: int = 9,
                         fallback_loading: float = 10.0, stream=None):
        """Learned form: per-pair (loading, window) from the network, then windowed MVDR."""
        torch = _torch()
        self._x(x)
        az, _, T = self._targets(az_rad, None)
        dev = self.device
        _check_tensor(params, "params", (MLP_PARAMS,), torch.float32, dev)
        out = torch.empty((T, self.K, self.Lt), dtype=torch.complex64, device=dev)
        weights = torch.empty((T, self.K, self.w_max), dtype=torch.complex64, device=dev)
        pair_win = torch.empty((T, self.K), dtype=torch.int32, device=dev)
        pair_loading = torch.empty((T, self.K), dtype=torch.float32, device=dev)
        fallback = torch.empty((T, self.K), dtype=torch.int32, device=dev)
        starts = torch.empty((T, self.K), dtype=torch.int32, device=dev)
        info = torch.empty((T, self.K), dtype=torch.int32, device=dev)
        _lib.check(_lib.load().wbm_beamform_learned(
            self._h, _ptr(x), az.ctypes.data, T, _ptr(params), float(noise_power), int(fallback_win),
            float(fallback_loading), _ptr(out), _ptr(weights), _ptr(pair_win), _ptr(pair_loading),
            _ptr(fallback), _ptr(starts), _ptr(info), _stream(stream)))
        return dict(out=out, weights=weights, pair_win=pair_win, pair_loading=pair_loading,
                    fallback=fallback, starts=starts, info=info)

    def sinr(self, az_rad, win, weights, starts, jam_az, jam_inr, noise_power: float = 1.0,
             pair_win=None, stream=None):
        """Output SINR [T, K] of weights against the exact noise + jammer covariance."""
        torch = _torch()
        az, w, T = self._targets(az_rad, win)
        ja = np.ascontiguousarray(np.asarray(jam_az, dtype=np.float64).ravel())
        ji = np.ascontiguousarray(np.asarray(jam_inr, dtype=np.float64).ravel())
        if ja.size != ji.size:
            raise ValueError("jam_az and jam_inr must have the same length")
        out = torch.empty((T, self.K), dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().wbm_sinr(
            self._h, az.ctypes.data, None if w is None else w.ctypes.data, T, _ptr(weights),
            _ptr(pair_win), _ptr(starts), ja.ctypes.data if ja.size else None,
            ji.ctypes.data if ji.size else None, int(ja.size), float(noise_power), _ptr(out),
            _stream(stream)))
        return out

    def full_mvdr(self, x, az_rad, loading: float, want_weights: bool = True, stream=None,
                  subbands=None):
        """Full-dimensional element-space MVDR per subband: out [T, K, Lt], weights [T, K, N],
        info [K]; subbands = (k0, nk) restricts it to k0 .. k0 + nk - 1 (other entries are
        left unwritten)."""
        torch = _torch()
        self._x(x)
        az, _, T = self._targets(az_rad, None)
        k0, nk = (0, 0) if subbands is None else (int(subbands[0]), int(subbands[1]))
        out = torch.zeros((T, self.K, self.Lt), dtype=torch.complex64, device=self.device)
        weights = (torch.zeros((T, self.K, self.N), dtype=torch.complex64, device=self.device)
                   if want_weights else None)
        info = torch.zeros((self.K,), dtype=torch.int32, device=self.device)
        _lib.check(_lib.load().wbm_full_mvdr(self._h, _ptr(x), az.ctypes.data, T, float(loading),
                                             k0, nk, _ptr(out), _ptr(weights), _ptr(info),
                                             _stream(stream)))
        return dict(out=out, weights=weights, info=info)


class Mlp:
    """Workspace of the loading / window predictor network (64 -> 128 -> 128 -> 2, GELU)."""

    def __init__(self, max_batch: int):
        lib = _lib.load()
        h = C.c_void_p()
        _lib.check(lib.wbm_mlp_create(int(max_batch), C.byref(h)))
        self._h = h
        self.max_batch = int(max_batch)
        self.device = _torch().device("cuda", _torch().cuda.current_device())

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().wbm_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, params, inp, stream=None):
        torch = _torch()
        n = int(inp.shape[0])
        _check_tensor(params, "params", (MLP_PARAMS,), torch.float32, self.device)
        _check_tensor(inp, "in", (n, 64), torch.float32, self.device)
        out = torch.empty((n, 2), dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().wbm_mlp_forward(self._h, _ptr(params), _ptr(inp), n, _ptr(out),
                                               _stream(stream)))
        return out

    def grad(self, params, inp, target, grad=None, loss=None, stream=None):
        torch = _torch()
        n = int(inp.shape[0])
        _check_tensor(params, "params", (MLP_PARAMS,), torch.float32, self.device)
        _check_tensor(inp, "in", (n, 64), torch.float32, self.device)
        _check_tensor(target, "target", (n, 2), torch.float32, self.device)
        grad = torch.empty((MLP_PARAMS,), dtype=torch.float32, device=self.device) if grad is None else grad
        loss = torch.empty((1,), dtype=torch.float32, device=self.device) if loss is None else loss
        _lib.check(_lib.load().wbm_mlp_grad(self._h, _ptr(params), _ptr(inp), _ptr(target), n,
                                            _ptr(grad), _ptr(loss), _stream(stream)))
        return grad, loss

    def adam(self, params, m, v, grad, step: int, lr: float, stream=None):
        _lib.check(_lib.load().wbm_mlp_adam(self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(grad),
                                            int(step), float(lr), _stream(stream)))

    def sweep_labels(self, sinr, deltas, widths, noise_power: float = 1.0, stream=None):
        """sinr [len(deltas) * len(widths), npairs] -> label [npairs, 2]."""
        torch = _torch()
        d = np.ascontiguousarray(np.asarray(deltas, dtype=np.float64))
        w = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
        npairs = int(sinr.shape[1])
        _check_tensor(sinr, "sinr", (d.size * w.size, npairs), torch.float32, self.device)
        label = torch.empty((npairs, 2), dtype=torch.float32, device=self.device)
        _lib.check(_lib.load().wbm_sweep_labels(self._h, _ptr(sinr), npairs, d.ctypes.data, d.size,
                                                w.ctypes.data, w.size, float(noise_power),
                                                _ptr(label), _stream(stream)))
        return label


MLP_STATIC_MAX_BATCH = _lib.MLP_STATIC_MAX_BATCH


def mlp_grad_static(params, inp, target, grad, loss=None, stream=None):
    """Gradient and loss of the predictor network as Mlp.grad, through the library's static
    device scratch instead of an Mlp workspace: nothing is allocated, so the caller passes the
    outputs (grad [MLP_PARAMS] float32, loss [1] float32 or None).  n <= MLP_STATIC_MAX_BATCH;
    calls that overlap on one GPU share the scratch and must be serialised."""
    torch = _torch()
    n = int(inp.shape[0])
    dev = params.device
    _check_tensor(params, "params", (MLP_PARAMS,), torch.float32, dev)
    _check_tensor(inp, "in", (n, 64), torch.float32, dev)
    _check_tensor(target, "target", (n, 2), torch.float32, dev)
    _check_tensor(grad, "grad", (MLP_PARAMS,), torch.float32, dev)
    if loss is not None:
        _check_tensor(loss, "loss", (1,), torch.float32, dev)
    _lib.check(_lib.load().wbm_mlp_grad_static(_ptr(params), _ptr(inp), _ptr(target), n,
                                               _ptr(grad), _ptr(loss), _stream(stream)))
    return grad, loss
