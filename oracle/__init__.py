"""Plain FP64 CPU oracle for windowed beamspace MVDR -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never imports, links or calls it, and
it shares no code with the library: it is the slow, obviously-correct
definition the GPU results are compared against.

Everything is complex128 / float64 and follows the paper's equations in their
order (Sec. II-III, Eq. 1-22).  Library primitives (numpy FFT, matmul,
Cholesky, triangular solve) serve as individual steps; there is no blocking,
fusion or reordering beyond what the equations state.

Parity pins: every function is checked in ``tests/test_oracle_*.py`` against
something other than itself -- direct DFT matrices on tiny inputs, closed
forms (Dirichlet kernel, single-interferer null depth, optimum SINR), the
KKT conditions of the MVDR problem, the W = M = N reduction identity, finite
differences for the MLP gradients.  Functions without such a pin carry the
words "parity unpinned" in their docstring.
"""

from .bmvdr import *  # noqa: F401,F403
from . import mlp  # noqa: F401
from . import learned  # noqa: F401
from . import radar  # noqa: F401
from . import upa  # noqa: F401
