"""MI355X-native relativistic lattice Boltzmann solver (arXiv:2011.06856).

The hot path -- the fused stream-and-collide step over a 2D grid with the
off-lattice product quadrature -- runs as hand-written HIP kernels for gfx950
in ``librlbm.so`` behind the C ABI of ``include/rlbm.h``; ``rlbm`` is its
ctypes binding.  Importing this package loads nothing; importing ``rlbm``
loads the library and fails if it is not built.
"""
