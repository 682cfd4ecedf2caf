"""Seeded synthetic inputs shared by the GPU path's tests/bench and the CPU oracle.

This package only *produces inputs*: banded matrices in LAPACK general-band
(GB) storage, shift grids, masks and point lists.  It contains none of the
arithmetic of sigma_min(zI - A); the oracle and the HIP library each do that on
their own.
"""
from .gen import *  # noqa: F401,F403
