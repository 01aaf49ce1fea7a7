"""Seeded synthetic array scenes for windowed beamspace MVDR.

This module only *synthesises inputs*: element-space IQ snapshots of a
uniform linear array that see wideband LFM target returns, wideband Gaussian
noise jammers and white receiver noise, following the per-subband signal
model of the paper (Sec. II-A, Eq. 9, with the steering vector of Eq. 7-8 and
the frequency scaling of Eq. 4-5).  It holds none of the beamformer's
arithmetic (no channelizer, beamspace transform, window, covariance or
solve): both the CPU oracle and the GPU library consume what it produces.

Synthesis: for every block b of K samples and every subband k the element
vector is

    X[e, b, k] = sum_src  exp(j * 2*pi * dl * sin(az_src) * (f_k/f_c) * e) * g_src[b, k]
                 + noise[e, b, k],        noise ~ CN(0, sigma^2)

and the time samples are the inverse unitary K-point DFT of each block,
x[e, b*K + tau] = K^-1/2 sum_k X[e, b, k] exp(+j 2 pi tau k / K).  With the
half-bin subband convention (centres of Eq. 1) subband k sits half a bin
higher and every block is additionally multiplied by exp(+j pi tau / K).

Jammers: g ~ CN(0, INR) i.i.d. over (b, k).  Targets: g = sqrt(SNR) * alpha
* (unitary K-point DFT over each block of a unit-power baseband LFM chirp
delayed by a random number of samples), alpha a random unit phasor.

All random numbers come from numpy PCG64 streams derived from the seed, one
stream per element row for the noise, so that a scene does not depend on the
chunking used to build it.
"""

from .configs import SceneConfig, CONFIGS, config_by_name, SMALL, GPU, BATCH, PRECISION, LEARNED_EVAL, LEARNED_TRAIN  # noqa: F401
from .generate import Scene, make_scene, subband_freq_ratio_gen  # noqa: F401
from .generate_torch import make_scene_torch  # noqa: F401
from .upa import UpaSceneConfig, UpaScene, make_upa_scene, UPA, UPA_SMALL, UPA_CONFIGS  # noqa: F401
