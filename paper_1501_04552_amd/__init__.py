"""MI355X (gfx950) Fourier pseudo-spectral stepper for the real cubic
Klein-Gordon equation, eq. (1) with the scheme of eq. (2).

``kg`` is the ctypes binding of the C interface in ``include/kg.h`` (same
function names); ``Solver`` holds a plan and its torch-allocated workspace.
"""
# PyTorch ships its own HIP runtime; importing it first makes libkg.so bind to
# that same runtime (one runtime per process: torch's device memory and
# streams are then valid inside the library).
import torch  # noqa: F401

from . import kg
from .kg import *  # noqa: F401,F403
from .solver import Solver  # noqa: F401
