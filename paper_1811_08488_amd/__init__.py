"""MSPCG for the even-odd preconditioned Moebius domain-wall Dirac equation on MI355X.

The compute path is the C-ABI shared library built from ``csrc/`` (HIP for
gfx950); ``mspcg`` is its ctypes binding.  Importing this package loads
nothing: the binding loads the library on first use and raises if it is
missing.
"""

__all__ = ["mspcg", "synth", "workloads"]
