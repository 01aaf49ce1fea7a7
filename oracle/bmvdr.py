"""FP64 definition of windowed beamspace MVDR (test infrastructure only).

Notation (1-D uniform linear array, the paper's N_z = M_z = W_z = 1 case):
N elements, M-point spatial DFT (M >= N, zero padding), K subbands from a
K-point time DFT, L training and Lt test snapshots (blocks) per subband,
T targets (the paper calls targets k and subbands l; here k is the subband).

Readings of points the paper leaves open (each also listed in the design
notes of the repository):
* channelizer: rectangular, non-overlapping K-sample blocks, unitary DFT;
  bin k stands for signed index ks = k or k - K; subband centre
  f_k/f_c = 1 + beta*ks/K (plain FFT bins), or 1 + beta*(ks + 1/2)/K when the
  half-bin centres of Eq. 1 are asked for (the channelizer then multiplies
  sample tau of each block by exp(-j pi tau / K) before the DFT);
* window: W consecutive bins starting at s = floor(u - (W-1)/2 + 1/2),
  u = M * (d/lambda_c) * sin(az) * f_k/f_c the (fractional) beam bin of the
  target, taken modulo M (the DFT is periodic); bins in ascending order;
* diagonal loading delta*I is added after the 1/L scaling of Eq. 11;
* the first L blocks train the covariance, the next Lt blocks are the test
  snapshots the weights are applied to.
"""

from __future__ import annotations

import math
from typing import Dict, Optional, Sequence

import numpy as np
import scipy.linalg

__all__ = [
    "subband_signed_index", "subband_freq_ratio", "channelize", "channelize_bins",
    "beamspace", "beamspace_rows", "spatial_frequency", "beam_position",
    "window_start", "window_bins", "steering", "beamspace_steering",
    "sample_covariance", "mvdr_weights", "beam_output", "lift_correlator",
    "beam_pattern", "synthesize", "lifted_outputs", "windowed_mvdr", "full_mvdr", "interference_covariance",
    "sinr", "sinr_loss_db", "rel_weight_error",
]


# --------------------------------------------------------------------------- subbands

def subband_signed_index(K: int) -> np.ndarray:
    """Signed frequency index of FFT bin k: k for k < K/2, else k - K."""
    k = np.arange(K)
    return np.where(k < K // 2, k, k - K)


def subband_freq_ratio(K: int, beta: float, half_bin: bool = False) -> np.ndarray:
    """f_k / f_c for every channelizer bin (Sec. II-A, Eq. 1; Eq. 4-5 use it).

    Eq. 1 places subband l (l = -K/2+1 .. K/2) at f_c + ((l - 1/2)/K) f_s.
    With ``half_bin`` bin k carries l = ks + 1, i.e. ratio 1 + beta (ks + 1/2)/K;
    otherwise a plain FFT bin is centred at 1 + beta ks / K.  beta = f_s / f_c.
    The expression is evaluated as ``1.0 + (beta * (ks + off)) / K`` in float64.
    """
    off = 0.5 if half_bin else 0.0
    ks = subband_signed_index(K).astype(np.float64)
    return np.array([1.0 + (beta * (float(v) + off)) / K for v in ks], dtype=np.float64)


def channelize(x: np.ndarray, K: int, half_bin: bool = False) -> np.ndarray:
    """FFT channelizer (Sec. III-A; Sec. IV-B uses an FFT-based channelizer).

    x[N, S] with S = B*K  ->  X[N, B, K],
    X[e, b, k] = K^-1/2 sum_tau x[e, b*K + tau] * h[tau] * exp(-j 2 pi tau k / K),
    h[tau] = 1, or exp(-j pi tau / K) for the half-bin centres of Eq. 1.
    """
    x = np.asarray(x, dtype=np.complex128)
    N, S = x.shape
    B = S // K
    blocks = x.reshape(N, B, K)
    if half_bin:
        blocks = blocks * np.exp(-1j * np.pi * np.arange(K) / K)[None, None, :]
    return np.fft.fft(blocks, axis=2, norm="ortho")


def channelize_bins(x: np.ndarray, K: int, bins: Sequence[int], half_bin: bool = False) -> np.ndarray:
    """Same as :func:`channelize` but only at the listed bins, by the direct DFT sum.

    Returns X[N, B, len(bins)].  Used where the full channelizer output would
    not fit host memory.
    """
    x = np.asarray(x)
    N, S = x.shape
    B = S // K
    tau = np.arange(K, dtype=np.float64)
    bins = np.asarray(bins, dtype=np.int64)
    F = np.exp(-2j * np.pi * np.outer(tau, bins) / K) / math.sqrt(K)   # [K, nb]
    if half_bin:
        F = F * np.exp(-1j * np.pi * tau / K)[:, None]
    out = np.empty((N, B, len(bins)), dtype=np.complex128)
    step = max(1, (64 << 20) // (B * K * 16))
    for e0 in range(0, N, step):
        blk = np.asarray(x[e0:e0 + step], dtype=np.complex128).reshape(-1, B, K)
        out[e0:e0 + step] = blk @ F
    return out


# --------------------------------------------------------------------------- beamspace

def beamspace(X: np.ndarray, M: int) -> np.ndarray:
    """Beamspace transform (Sec. III-B, Eq. 14-17, one dimension).

    X[N, B, K] -> Y[M, B, K] with Y[m] = M^-1/2 sum_{e<N} X[e] exp(-j 2 pi m e / M):
    the truncated M x N DFT matrix D applied to every element vector (zero
    padding N -> M).
    """
    N = X.shape[0]
    assert M >= N
    return np.fft.fft(X, n=M, axis=0) / math.sqrt(M)


def beamspace_rows(Xk: np.ndarray, M: int, bins: Sequence[int]) -> np.ndarray:
    """Rows ``bins`` of D X for one subband, by the direct sum of Eq. 14/17.

    Xk[N, B] -> [len(bins), B].
    """
    N = Xk.shape[0]
    bins = np.asarray(bins, dtype=np.float64)
    D = np.exp(-2j * np.pi * np.outer(bins, np.arange(N)) / M) / math.sqrt(M)
    return D @ Xk


# --------------------------------------------------------------------------- steering / window

def spatial_frequency(sin_az: float, ratio: float, dl: float = 0.5) -> float:
    """Omega = 2 pi (d/lambda_c) sin(az) f_k/f_c  (Eq. 2-5, azimuth only; pi sin(az) at d = lambda/2)."""
    return 2.0 * math.pi * dl * sin_az * ratio


def beam_position(sin_az: float, ratio: float, M: int, dl: float = 0.5) -> float:
    """Fractional beamspace bin u of the steering vector: Omega = 2 pi u / M.

    Evaluated as ``((M * dl) * sin_az) * ratio`` in float64 (exact operation order).
    """
    return ((float(M) * dl) * sin_az) * ratio


def window_start(u: float, W: int) -> int:
    """First bin of the W-bin window centred on the target's beam (Sec. III-B, Eq. 18).

    s = floor((u - (W-1)/2) + 1/2): the window centre is the nearest bin
    position to u (ties go to the higher start).  For odd W this is the
    FFT bin nearest the target, with (W-1)/2 bins on each side.
    """
    c = u - 0.5 * float(W - 1)
    return int(math.floor(c + 0.5))


def window_bins(start: int, W: int, M: int) -> np.ndarray:
    """Bins selected by S_k (Eq. 18-19): (start + i) mod M for i < W."""
    return (start + np.arange(W)) % M


def steering(N: int, omega: float) -> np.ndarray:
    """a(Omega) = [1, e^{j Omega}, ..., e^{j Omega (N-1)}]^T  (Eq. 8)."""
    return np.exp(1j * omega * np.arange(N, dtype=np.float64))


def beamspace_steering(N: int, M: int, omega: float, bins: Sequence[int]) -> np.ndarray:
    """Windowed beamspace steering a~ = S D a (Sec. III-C, below Eq. 20), direct sum."""
    a = steering(N, omega)
    return beamspace_rows(a[:, None], M, bins)[:, 0]


# --------------------------------------------------------------------------- MVDR

def sample_covariance(Ytrain: np.ndarray, delta: float) -> np.ndarray:
    """R = (1/L) sum_n y[n] y[n]^H + delta I   (Eq. 11; Eq. 20 uses it on windowed data).

    Ytrain[W, L] holds one snapshot per column.
    """
    W, L = Ytrain.shape
    R = (Ytrain @ Ytrain.conj().T) / L
    return R + delta * np.eye(W)


def mvdr_weights(R: np.ndarray, a: np.ndarray) -> np.ndarray:
    """MVDR correlator c = R^-1 a / (a^H R^-1 a)  (Eq. 12-13, Eq. 20).

    Computed through the Cholesky factor R = G G^H: v = G^-1 a, q = v^H v,
    c = G^-H v / q.
    """
    G = np.linalg.cholesky(R)
    v = scipy.linalg.solve_triangular(G, a, lower=True)
    q = float(np.vdot(v, v).real)
    return scipy.linalg.solve_triangular(G.conj().T, v, lower=False) / q


def beam_output(w: np.ndarray, Ytest: np.ndarray) -> np.ndarray:
    """Beamformer output c^H y[n] for every test snapshot (Sec. II-B, below Eq. 13)."""
    return w.conj() @ Ytest


def lift_correlator(w: np.ndarray, bins: Sequence[int], M: int, N: int) -> np.ndarray:
    """Antenna-space equivalent correlator c^ = D^H S^T c~  (Eq. 21)."""
    bins = np.asarray(bins, dtype=np.float64)
    DH = np.exp(2j * np.pi * np.outer(np.arange(N), bins) / M) / math.sqrt(M)   # rows of D^H at the bins
    return DH @ w


def beam_pattern(c: np.ndarray, omegas: Sequence[float]) -> np.ndarray:
    """Cosine similarity |<c, a(Omega)>| / (||c|| ||a(Omega)||)  (Eq. 22), one value per Omega."""
    N = c.shape[0]
    out = np.empty(len(omegas))
    for i, om in enumerate(omegas):
        a = steering(N, om)
        out[i] = abs(np.vdot(c, a)) / (np.linalg.norm(c) * np.linalg.norm(a))
    return out


def synthesize(Z: np.ndarray, K: int, half_bin: bool = False) -> np.ndarray:
    """Subband synthesis (Sec. II / Sec. IV-B: the per-subband beamformer outputs are combined by
    an inverse FFT into the wideband signal): the inverse of :func:`channelize` per block.

    Z[..., K, B] (subband axis, then block axis) -> z[..., B*K],
    z[b*K + tau] = K^-1/2 conj(h[tau]) sum_k Z[k, b] exp(+j 2 pi tau k / K), with h the
    channelizer's pre-twiddle (1, or exp(-j pi tau / K) for the half-bin centres).
    """
    Z = np.asarray(Z, dtype=np.complex128)
    assert Z.shape[-2] == K
    blocks = np.fft.ifft(np.moveaxis(Z, -2, -1), axis=-1, norm="ortho")     # [..., B, K]
    if half_bin:
        blocks = blocks * np.exp(1j * np.pi * np.arange(K) / K)
    return blocks.reshape(*blocks.shape[:-2], -1)


def lifted_outputs(x: np.ndarray, c_hat: np.ndarray, *, K: int, L: int, Lt: int,
                   half_bin: bool = False) -> np.ndarray:
    """Beam outputs from lifted correlators applied in element space (Eq. 21 and the remark
    after it): z[t, k, l] = c^_tk^H X_k[:, L + l] for the test snapshots, no beamspace step.

    x[N, S]; c_hat[T, K, N] -> z[T, K, Lt].
    """
    X = channelize(x, K, half_bin)                         # [N, B, K]
    T = c_hat.shape[0]
    z = np.empty((T, K, Lt), dtype=np.complex128)
    for t in range(T):
        for k in range(K):
            z[t, k] = beam_output(c_hat[t, k], X[:, L:L + Lt, k])
    return z


# --------------------------------------------------------------------------- pipelines

def windowed_mvdr(x: np.ndarray, *, M: int, K: int, L: int, Lt: int,
                  sin_az: Sequence[float], win: Sequence[int], delta: float,
                  beta: float = 0.2, dl: float = 0.5, half_bin: bool = False,
                  subbands: Optional[Sequence[int]] = None,
                  X: Optional[np.ndarray] = None,
                  return_windows: bool = False) -> Dict[str, np.ndarray]:
    """Windowed beamspace MVDR for every (target, subband) pair (Fig. 2, Sec. III).

    Steps per subband k: channelize (Sec. III-A) -> beamspace rows of the
    window (Eq. 17-19) -> covariance of the first L snapshots plus loading
    (Eq. 11) -> MVDR correlator (Eq. 20) -> output on the next Lt snapshots.

    Returns dict with ``start`` [T, nk] int64, ``u`` [T, nk], ``w`` [T, nk, Wmax]
    (zero padded), ``a`` [T, nk, Wmax] (windowed steering), ``z`` [T, nk, Lt],
    ``R`` list-of-lists of the loaded covariances, ``subbands``, and with
    ``return_windows`` ``Yw`` list-of-lists of the windowed snapshots [W, L + Lt].
    ``X`` may be given instead of ``x`` (channelized [N, B, K], or [N, B, len(subbands)] with
    the listed subbands' columns in that order).
    """
    N = x.shape[0] if x is not None else X.shape[0]
    T = len(sin_az)
    win = [int(v) for v in win]
    Wmax = max(win)
    ks = list(range(K)) if subbands is None else [int(k) for k in subbands]
    if X is None:
        X = channelize(x, K, half_bin) if subbands is None else channelize_bins(x, K, ks, half_bin)
        kcol = {k: (k if subbands is None else i) for i, k in enumerate(ks)}
    elif subbands is not None and X.shape[2] == len(ks) != K:
        kcol = {k: i for i, k in enumerate(ks)}      # X holds only the listed subbands
    else:
        kcol = {k: k for k in ks}
    ratio = subband_freq_ratio(K, beta, half_bin)
    nk = len(ks)
    start = np.zeros((T, nk), dtype=np.int64)
    upos = np.zeros((T, nk))
    w_out = np.zeros((T, nk, Wmax), dtype=np.complex128)
    a_out = np.zeros((T, nk, Wmax), dtype=np.complex128)
    z_out = np.zeros((T, nk, Lt), dtype=np.complex128)
    Rs = [[None] * nk for _ in range(T)]
    Yws = [[None] * nk for _ in range(T)] if return_windows else None
    for ik, k in enumerate(ks):
        Xk = X[:, :L + Lt, kcol[k]]
        Yk = beamspace(Xk, M)                                                 # [M, B]
        for t in range(T):
            W = win[t]
            u = beam_position(float(sin_az[t]), float(ratio[k]), M, dl)
            s = window_start(u, W)
            bins = window_bins(s, W, M)
            Yw = Yk[bins]                                                     # S_k D y, [W, B]
            a = beamspace_steering(N, M, spatial_frequency(float(sin_az[t]), float(ratio[k]), dl), bins)
            R = sample_covariance(Yw[:, :L], delta)
            w = mvdr_weights(R, a)
            start[t, ik], upos[t, ik] = s, u
            w_out[t, ik, :W] = w
            a_out[t, ik, :W] = a
            z_out[t, ik] = beam_output(w, Yw[:, L:L + Lt])
            Rs[t][ik] = R
            if return_windows:
                Yws[t][ik] = Yw
    out = dict(start=start, u=upos, w=w_out, a=a_out, z=z_out, R=Rs, subbands=np.asarray(ks))
    if return_windows:
        out["Yw"] = Yws
    return out


def full_mvdr(x: np.ndarray, *, K: int, L: int, Lt: int, sin_az: Sequence[float], delta: float,
              beta: float = 0.2, dl: float = 0.5, half_bin: bool = False,
              subbands: Optional[Sequence[int]] = None,
              X: Optional[np.ndarray] = None) -> Dict[str, np.ndarray]:
    """Full-dimensional element-space MVDR per subband (Sec. II-B, Eq. 11-13).

    R = (1/L) sum X X^H + delta I_N over the first L blocks, c = R^-1 a / (a^H R^-1 a)
    with a the element steering vector at the subband centre, output c^H X on
    the next Lt blocks.  Returns ``w`` [T, nk, N] and ``z`` [T, nk, Lt].
    """
    N = x.shape[0]
    T = len(sin_az)
    ks = list(range(K)) if subbands is None else [int(k) for k in subbands]
    if X is None:
        X = channelize(x, K, half_bin) if subbands is None else channelize_bins(x, K, ks, half_bin)
        kcol = {k: (k if subbands is None else i) for i, k in enumerate(ks)}
    else:
        kcol = {k: k for k in ks}
    ratio = subband_freq_ratio(K, beta, half_bin)
    nk = len(ks)
    w_out = np.zeros((T, nk, N), dtype=np.complex128)
    z_out = np.zeros((T, nk, Lt), dtype=np.complex128)
    for ik, k in enumerate(ks):
        Xk = X[:, :L + Lt, kcol[k]]
        R = sample_covariance(Xk[:, :L], delta)
        for t in range(T):
            a = steering(N, spatial_frequency(float(sin_az[t]), float(ratio[k]), dl))
            w = mvdr_weights(R, a)
            w_out[t, ik] = w
            z_out[t, ik] = beam_output(w, Xk[:, L:L + Lt])
    return dict(w=w_out, z=z_out, subbands=np.asarray(ks))


# --------------------------------------------------------------------------- scoring

def interference_covariance(N: int, jam_sin: Sequence[float], jam_inr: Sequence[float],
                            ratio: float, dl: float = 0.5, noise_var: float = 1.0) -> np.ndarray:
    """Exact interference-plus-noise covariance of one subband (Eq. 10 without targets).

    R_in = sigma^2 I + sum_j INR_j a_j a_j^H for white-in-band jammers of
    per-element power INR_j at directions sin(az_j).
    """
    R = noise_var * np.eye(N, dtype=np.complex128)
    for s, p in zip(jam_sin, jam_inr):
        a = steering(N, spatial_frequency(float(s), ratio, dl))
        R += p * np.outer(a, a.conj())
    return R


def sinr(w: np.ndarray, a: np.ndarray, R_in: np.ndarray) -> float:
    """Output SINR of correlator w for unit-power signal with steering a: |w^H a|^2 / (w^H R_in w)."""
    num = abs(np.vdot(w, a)) ** 2
    den = float(np.vdot(w, R_in @ w).real)
    return num / den


def sinr_loss_db(w_test: np.ndarray, w_ref: np.ndarray, a: np.ndarray, R_in: np.ndarray) -> float:
    """10 log10(SINR(w_ref) / SINR(w_test)): how much output SINR w_test gives up."""
    return 10.0 * math.log10(sinr(w_ref, a, R_in) / sinr(w_test, a, R_in))


def rel_weight_error(w_test: np.ndarray, w_ref: np.ndarray) -> float:
    return float(np.linalg.norm(w_test - w_ref) / np.linalg.norm(w_ref))
