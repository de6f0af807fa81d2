"""MI355X (gfx950) DUGKS step for the conservative Allen-Cahn equation.

The compute path is libdugks.so (HIP kernels behind the C ABI of
include/dugks.h); ``_lib`` binds it with ctypes and ``Solver`` drives one grid
with torch-owned device memory and streams.
"""
from . import _lib  # noqa: F401

__all__ = ["_lib", "build", "inputs", "solver"]
