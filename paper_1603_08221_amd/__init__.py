"""MI355X-native (gfx950 HIP) solver for gas separation in binary mixtures.

Hot path of Wang, Xu & Guo, arXiv:1603.08221: two coupled D2Q9 MRT lattice
Boltzmann populations in a pressure-driven microchannel with diffuse-bounce-back
walls, reduced every step to the separation degree CL. The solver is the C ABI
library ``liblbsep.so`` (header ``include/lbsep.h``); ``lbsep`` is its thin
Python binding and ``workloads`` holds the seeded synthetic channel configurations.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads"]
