"""FP64 CPU oracle for the relativistic lattice Boltzmann method of arXiv:2011.06856.

Test infrastructure: only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import this package.  It shares no code with the GPU
library in ``paper_2011_06856_amd``, and that package never imports it.
"""
from .oracle import (  # noqa: F401
    build, Quadrature, Sim, landau, mj_moment, num_threads, set_threads, site_stats, qs_G, qs_landau,
)
from .closed_forms import (  # noqa: F401
    free_streaming_tube, landau_1d, rel_l2,
)
