"""stereomesh: MI355X (gfx950) implementation of the iterative piecewise-planar stereo
method of Pillai, Ramalingam and Leonard, "High-Performance and Tunable Stereo
Reconstruction" (ICRA 2016).

The product is the C ABI in ``include/stereomesh.h`` (libstereomesh.so, hand-written
HIP kernels plus host triangulation); ``api`` wraps it for torch tensors.
"""
from ._lib import load, StereoMeshError, LIB_PATH  # noqa: F401

__all__ = ["load", "StereoMeshError", "LIB_PATH"]
