"""MI355X (gfx950) implementation of the D2Q9 lattice Boltzmann stream-and-collide
step with the entropic multi-relaxation (KBC) collision and the LBGK baseline.

The compute path is the HIP library ``libkbc.so`` behind the C ABI in
``include/kbc.h``; this package holds its Python binding (``_lib``), a
per-lattice wrapper (``sim.Sim``) and the seeded workload generators
(``inputs``).  Importing the package does not load the library.
"""
__all__ = ["inputs", "sim"]
