"""FP64 CPU oracle of the coupled LB/MD step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU library and its Python binding never do.
"""
from .oracle import (Oracle, OrDesc, lib, tables, feq, philox, gauss3, mode_basis, fluid_normals, jvp,  # noqa: F401
                     jvp_series,
                     set_threads, max_threads)
