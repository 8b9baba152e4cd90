"""MI355X (gfx950) temporal component matrices, network hashing and fusion.

The compute runs in ``libtn.so`` (hand-written HIP kernels behind the C ABI of
``include/tn.h``); this package only marshals arguments.  Importing it fails
if the library is not built.
"""
from ._lib import DIRECTED, FORWARD, HLL, TIES_SEQUENTIAL, TNError, lib  # noqa: F401  (loads libtn.so)
from .api import *  # noqa: F401,F403
