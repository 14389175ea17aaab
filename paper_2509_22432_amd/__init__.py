"""MI355X-native flooding step of the Flood complex.

Python binding over libflood.so (C ABI in include/flood.h).  This module
only marshals arguments: every step of the path runs in the library's HIP
kernels (landmarks, grid, flooding, winners, backward) or its host code
(Delaunay, persistence).
PyTorch provides device memory and the current HIP stream.
"""
from .api import (  # noqa: F401
    Complex, FloodFiltration, FloodProblem, delaunay, filtration, fps, fps_batched, lift_2d,
    n_interior, own_samples, persistence, problem_from_complexes,
)
from ._lib import FloodError  # noqa: F401
