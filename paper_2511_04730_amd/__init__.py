"""MI355X-native LLOID filtering core (multirate SVD matched filter).

The work runs in liblloid.so (HIP kernels for gfx950) behind the C ABI in
include/lloid.h; this package only marshals arguments to it.
"""
from ._lib import LloidError, load  # noqa: F401
from .plan import LloidPlan, Whitener  # noqa: F401
