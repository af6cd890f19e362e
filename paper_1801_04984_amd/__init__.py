"""MI355X-native space-time Biot slab operator and solver.

The compute path is the HIP library libbiotst.so (C ABI in include/biotst.h);
`native` is its ctypes binding.  Koecher, "Space-Time-Parallel
Poroelasticity Simulation": monolithic dG(r) x (Q2, RT1, DG-Q1) slab
systems solved by blockwise fixed-stress preconditioned GMRES.
"""
from .native import BiotSlab, BiotError, load_library, make_desc, make_opts  # noqa: F401
