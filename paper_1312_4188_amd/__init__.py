"""MI355X (gfx950) first-match packet classifier.

The work happens in ``libfw.so`` (hand-written HIP kernels behind the C
interface in ``include/fw.h``); :mod:`paper_1312_4188_amd.fw` is the thin
Python binding that marshals torch device tensors into that interface.
Importing this package loads nothing; the binding loads the library on first
use and raises if it has not been built.
"""

__all__ = ["fw"]
