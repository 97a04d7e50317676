"""MI355X-native PDV multiple-scattering Monte Carlo (libpdv, HIP gfx950).

The simulation runs in libpdv.so (see include/pdv.h); ``pdv`` is its ctypes
binding and ``workloads`` holds seeded synthetic problem statements.
"""
from . import workloads  # noqa: F401

__all__ = ["pdv", "workloads"]
