"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI and compare it
with the FP64 oracle on the same complex64 input."""

from __future__ import annotations

import math
import sys

import numpy as np

import oracle

EPS32 = 2.0 ** -24


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def snapshot_dynamic_range(scene) -> float:
    """sqrt(total element-space snapshot power / noise power) = sqrt(1 + N sum INR / sigma^2)."""
    cfg = scene.cfg
    return math.sqrt(1.0 + cfg.N * float(np.sum(scene.jammer_inr)) / cfg.noise_var)


def weight_tol(kappa: float, plain: bool = False, dr: float = 1.0, unit: float = EPS32) -> float:
    """Relative weight tolerance against the FP64 oracle, derived from the FP32 arithmetic.

    * Rounding every stored snapshot to FP32 perturbs the windowed covariance so that the
      MVDR weights move by about 0.5 eps32 sqrt(kappa) (measured with in-window jammers at
      30-50 dB INR): bound 8 eps32 sqrt(kappa).
    * FP32 FFT arithmetic leaves errors of order eps32 times the whole snapshot's norm in
      every bin, so low-power window bins see strong jammers' rounding: the weights move by
      about 0.05 eps32 DR, DR the snapshot dynamic range (measured at N = 256 and 1024):
      bound 0.5 eps32 DR.
    * The plain form also forms the covariance and solves in FP32, which moves the weights
      by about u kappa with u = eps32: bound 4 u kappa.  The mixed forms form it from BF16
      products: u = 2^-16 with each snapshot split into BF16 hi + lo (the lo*lo product is
      dropped), u = 2^-8 with one BF16 product.
    The floor is the 1e-5 relative weight error the method is held to.
    """
    base = max(1e-5, 0.5 * EPS32 * dr)
    if plain:
        return max(base, 4.0 * unit * kappa)
    return max(base, 8.0 * EPS32 * math.sqrt(kappa))


def windowed_interference(scene, k, bins, ratio):
    """S D R_in D^H S^T of one window: sigma^2 (S D)(S D)^H + sum_j INR_j (S D a_j)(S D a_j)^H,
    the same matrix as forming the N x N R_in first, in O(W^2 N) (the N x N form takes seconds
    per window at N = 4096)."""
    cfg = scene.cfg
    D = np.exp(-2j * np.pi * np.outer(np.asarray(bins, dtype=np.float64), np.arange(cfg.N)) / cfg.M)
    D /= math.sqrt(cfg.M)
    R = cfg.noise_var * (D @ D.conj().T)
    for s, p in zip(np.sin(scene.jammer_az), scene.jammer_inr):
        a = D @ oracle.steering(cfg.N, oracle.spatial_frequency(float(s), ratio, cfg.dl))
        R += p * np.outer(a, a.conj())
    return R


# relative weight error ||w - w_oracle|| / ||w_oracle|| every pair of the extended-precision
# forms must stay within (with SINR loss <= 0.1 dB)
WEIGHT_ERR_BAR = 1e-5


def compare_beamform(scene, ref, res, subbands=None, plain=False, sinr_bar_db=0.1,
                     check_sinr=True, fp32_fft=True, tol_scale=1.0, unit=EPS32, ext=False,
                     pairs=False):
    """Check GPU outputs ``res`` (tensors) against oracle dict ``ref`` (windowed_mvdr with
    return_windows).  Returns a dict of error statistics.

    pairs: also return "per_pair", a list of (oracle pivot ratio, SINR loss, weight error).
    ext: the extended-precision forms (fused / graph / learned): every pair's relative weight
    error must be <= 1e-5 and its SINR loss <= 0.1 dB, with no widening; the FP32 bound of
    weight_tol is still computed and logged (max_err_over_f32_tol) for comparison."""
    cfg = scene.cfg
    T, K = len(scene.win), cfg.K
    ks = list(range(K)) if subbands is None else list(subbands)
    starts = res["starts"].cpu().numpy()
    w_g = res["weights"].cpu().numpy().astype(np.complex128)
    z_g = res["out"].cpu().numpy().astype(np.complex128)
    info = res["info"].cpu().numpy()
    ratio = oracle.subband_freq_ratio(K, cfg.beta, cfg.half_bin)
    assert np.all(info[:, ks] == 0), "Cholesky failures reported"
    assert np.array_equal(starts[:, ks], ref["start"]), "window starts differ"
    worst_w, worst_ratio, worst_z, worst_loss = 0.0, 0.0, 0.0, 0.0
    per_pair = []   # (pivot ratio of the oracle's LDL^H, SINR loss dB, relative weight error)
    dr = snapshot_dynamic_range(scene) if fp32_fft else 1.0
    for ik, k in enumerate(ks):
        for t in range(T):
            W = int(scene.win[t])
            wo = ref["w"][t, ik, :W]
            wg = w_g[t, k, :W]
            assert np.all(w_g[t, k, W:] == 0), "weights not zero padded"
            R = ref["R"][t][ik]
            kappa = float(np.linalg.cond(R))
            piv = np.abs(np.diag(np.linalg.cholesky(R))) ** 2
            piv_ratio = float(piv.max() / piv.min())
            err = oracle.rel_weight_error(wg, wo)
            tol = weight_tol(kappa, plain, dr, unit)
            if ext:
                assert err <= WEIGHT_ERR_BAR, \
                    f"pair t={t} k={k}: weight error {err:.3e} > 1e-5 (kappa {kappa:.3e})"
            elif tol_scale is not None:   # None: the error is reported, not bounded
                assert err <= tol * tol_scale, \
                    f"pair t={t} k={k}: weight error {err:.3e} > {tol:.3e} (kappa {kappa:.3e})"
            worst_w = max(worst_w, err)
            worst_ratio = max(worst_ratio, err / tol)
            # apply step: GPU output vs the GPU's own weights on the oracle's test snapshots.
            # The GPU's snapshots carry the FP32 rounding of two FFTs (~1e-6 of |y|), so the
            # bound is 1e-5 ||w|| max ||y||; a wrong index or conjugation gives O(1).
            Yt = ref["Yw"][t][ik][:, cfg.L:cfg.L + cfg.Lt]
            if cfg.Lt and tol_scale is not None:
                zc = wg.conj() @ Yt
                scale = np.linalg.norm(wg) * np.max(np.linalg.norm(Yt, axis=0))
                dz = float(np.max(np.abs(z_g[t, k] - zc)) / scale)
                assert dz <= 1e-5, f"pair t={t} k={k}: output error {dz:.3e}"
                worst_z = max(worst_z, dz)
            if check_sinr and scene.jammer_az.size:
                bins = oracle.window_bins(int(ref["start"][t, ik]), W, cfg.M)
                Rin = windowed_interference(scene, k, bins, ratio[k])
                a = ref["a"][t, ik, :W]
                loss = abs(oracle.sinr_loss_db(wg, wo, a, Rin))
                if sinr_bar_db is not None:   # None: the loss is reported, not bounded
                    assert loss <= sinr_bar_db, f"pair t={t} k={k}: SINR loss {loss:.3e} dB"
                worst_loss = max(worst_loss, loss)
                per_pair.append((piv_ratio, loss, err))
    key = "max_err_over_f32_tol" if ext else "max_err_over_tol"
    st = {"max_weight_err": worst_w, key: worst_ratio, "max_out_err": worst_z,
          "max_sinr_loss_db": worst_loss}
    if pairs:
        st["per_pair"] = per_pair
    return st


def loss_by_pivot_ratio(per_pair, edges=(1, 10, 100, 1e3, 1e4, 1e5, 1e7, 1e12)):
    """Worst SINR loss and weight error of the pairs in each band of LDL^H pivot ratio (the
    routing statistic of the mixed forms), as text for the test log."""
    r = np.asarray(per_pair, dtype=np.float64).reshape(-1, 3)
    out = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        m = (r[:, 0] >= lo) & (r[:, 0] < hi)
        if m.any():
            out.append(f"[{lo:.0e},{hi:.0e}): n={int(m.sum())} loss<={r[m, 1].max():.2e} dB "
                       f"err<={r[m, 2].max():.2e}")
    return "; ".join(out)
