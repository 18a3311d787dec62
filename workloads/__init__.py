"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package holds input generation only (meshes, grids, fields, seeds);
none of the transfer arithmetic lives here.
"""
from .gen import *  # noqa: F401,F403
from . import plane  # noqa: F401,E402  (two-dimensional workloads)
from . import unstructured  # noqa: F401,E402  (unstructured fluid background)
