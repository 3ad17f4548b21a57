"""Seeded synthetic inputs shared by the oracle side and the HIP side.

Holds no arithmetic of the method: only workload sizes and parameters, and the
seeded complex Gaussian noise that is added to the second-order seed vertex.
"""
from .siam import *  # noqa: F401,F403
