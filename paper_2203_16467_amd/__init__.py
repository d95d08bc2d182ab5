"""spff: MI355X-native (gfx950) spectral phase-field fracture solver.

The hot path (FFT-accelerated mechanics CG with the compatibility
projection, bound-constrained CG phase-field solve, alternating-minimisation
load steps) runs in hand-written HIP kernels behind the C ABI declared in
include/spff.h; ``spff`` is the ctypes binding.
"""

from . import spff  # noqa: F401
from .spff import (Problem, create_batch, create_problem, default_config, workspace_bytes,  # noqa: F401
                   SpffError, SpffLibraryError)
