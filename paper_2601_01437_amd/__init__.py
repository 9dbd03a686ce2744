"""MI355X (gfx950) library for the linear-method operator of shallow neural
quantum states and the implicitly restarted Lanczos optimisation step.

The compute path is the HIP shared library ``lib/libirlnqs.so`` (C ABI in
``include/irlnqs.h``); this package is its ctypes binding plus a small
convenience class.  Importing it without the built library raises ImportError.
"""
from .binding import *  # noqa: F401,F403
from .binding import EXPORTED, IrlError, LIB_PATH  # noqa: F401
from .system import Batch, System  # noqa: F401
