"""MI355X-native Keldysh bubble / Schwinger-Dyson library (hot path of arXiv:2405.20996).

The computation lives in libkqft.so (hand-written HIP for gfx950, C ABI in
include/kqft.h); `kqft` is its thin Python binding.
"""
from . import kqft  # noqa: F401
