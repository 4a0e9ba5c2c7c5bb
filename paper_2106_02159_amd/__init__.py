"""MI355X-native explicit hyperbolic (Euler) step of Guermond, Kronbichler,
Maier, Popov, Tomas (arXiv:2106.02159): Q1 graph viscosity, low-order update,
local bounds, high-order flux and convex limiting inside SSPRK(3,3), as HIP
kernels behind the C ABI of ``include/ns.h``.

``abi`` is the ctypes binding of ``libns.so``; ``workloads`` holds the seeded
synthetic inputs; ``build`` compiles the library in-tree.
"""
from . import abi, workloads  # noqa: F401
from .abi import Graph, NSError, Solver  # noqa: F401
