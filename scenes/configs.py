"""Workload shapes and scene recipes.

Five workloads, all on a half-wavelength uniform linear array with fractional
bandwidth f_s/f_c = 0.2 and unit-variance receiver noise:

* ``small``      N=16,   M=32,   K=16,  W=5,  L=Lt=64,   1 target, 1 jammer (complex128)
* ``gpu``        N=256,  M=512,  K=128, W=9,  L=Lt=256,  8 targets, 3 jammers
* ``batch``      N=1024, M=2048, K=256, W in {5,9,17,33}, L=Lt=512, 64 targets, 6 jammers
* ``precision``  N=4096, M=8192, K=512, W=64, L=Lt=1024, 32 targets, 8 jammers
* ``learned``    evaluation scenes of the ``batch`` shape; training scenes of the ``gpu`` shape

Target angles are uniform in [-60, 60] degrees from broadside; jammer angles
likewise but rejected when they fall within 2/N of a target in sin-space.
"""

from __future__ import annotations

import dataclasses
from typing import Optional, Sequence, Tuple


@dataclasses.dataclass(frozen=True)
class SceneConfig:
    name: str
    N: int                      # array elements (ULA)
    M: int                      # spatial FFT size (power of two, >= N)
    K: int                      # subbands = time-FFT length (power of two)
    L: int                      # training snapshots (blocks) per subband
    Lt: int                     # test snapshots per subband
    T: int                      # targets (beams per subband)
    W: Optional[int] = None     # fixed window width, or None to draw from W_choices
    W_choices: Tuple[int, ...] = ()
    beta: float = 0.2           # fractional bandwidth f_s / f_c
    dl: float = 0.5             # element spacing over the centre wavelength
    half_bin: bool = False      # subband centres of Eq. 1 (half-bin offsets)
    noise_var: float = 1.0      # receiver noise power sigma^2 per element and sample
    loading_factor: float = 10.0  # diagonal loading = factor * noise_var
    n_jammers: int = 0
    target_az_deg: Optional[Sequence[float]] = None   # fixed angles (else random)
    target_snr_db: Optional[Sequence[float]] = None
    jammer_az_deg: Optional[Sequence[float]] = None
    jammer_inr_db: Optional[Sequence[float]] = None
    az_range_deg: Tuple[float, float] = (-60.0, 60.0)
    snr_range_db: Tuple[float, float] = (-10.0, 10.0)
    inr_range_db: Tuple[float, float] = (20.0, 40.0)
    seed: int = 0
    complex128: bool = False

    @property
    def B(self) -> int:
        return self.L + self.Lt

    @property
    def S(self) -> int:
        return self.B * self.K

    @property
    def delta(self) -> float:
        return self.loading_factor * self.noise_var

    def replace(self, **kw) -> "SceneConfig":
        return dataclasses.replace(self, **kw)


SMALL = SceneConfig(
    name="small", N=16, M=32, K=16, L=64, Lt=64, T=1, W=5,
    n_jammers=1, target_az_deg=(10.0,), target_snr_db=(0.0,),
    jammer_az_deg=(-30.0,), jammer_inr_db=(30.0,), seed=1, complex128=True)

GPU = SceneConfig(
    name="gpu", N=256, M=512, K=128, L=256, Lt=256, T=8, W=9,
    n_jammers=3, inr_range_db=(20.0, 40.0), seed=2)

BATCH = SceneConfig(
    name="batch", N=1024, M=2048, K=256, L=512, Lt=512, T=64, W=None,
    W_choices=(5, 9, 17, 33), n_jammers=6, inr_range_db=(20.0, 50.0), seed=3)

PRECISION = SceneConfig(
    name="precision", N=4096, M=8192, K=512, L=1024, Lt=1024, T=32, W=64,
    n_jammers=8, inr_range_db=(20.0, 60.0), seed=4)

LEARNED_EVAL = BATCH.replace(name="learned_eval", seed=5_900_000)
LEARNED_TRAIN = GPU.replace(name="learned_train", seed=5_000_000)

CONFIGS = {c.name: c for c in (SMALL, GPU, BATCH, PRECISION, LEARNED_EVAL, LEARNED_TRAIN)}


def config_by_name(name: str) -> SceneConfig:
    return CONFIGS[name]
