"""MI355X (gfx950) implementation of the coupled D1Q3Q3 lattice Boltzmann
scheme of Dubois, Graille & Lallemand (arXiv 1802.02369).

The hot path lives in ``liblbm.so`` (hand-written HIP, C ABI in
``include/lbm.h``); ``lbm`` is its thin Python binding and ``workloads`` the
seeded synthetic inputs.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "lbm"]
