"""MI355X-native hot path of gradient-descent borehole acoustic FWI
(Tang, Cheng, Li & Fang, "Borehole acoustic full-waveform inversion").

The compute runs in libbhfwi.so (hand-written HIP for gfx950, C-ABI in
include/bhfwi.h).  This package is the Python binding: ``Survey`` wraps the
C-ABI, ``BoreholeFWI`` is the torch.autograd.Function around the forward and
adjoint kernels, ``fwi`` holds the iteration driver.
"""
from ._lib import (BhfwiError, Survey, load, moduli, moduli_grad, radial_taper,  # noqa: F401
                   semblance, semblance_pick, starting_model, velocities)
from .autograd import BoreholeFWI, Moduli  # noqa: F401
