"""Plain FP64 CPU oracle of the compressible D2V16 MRT finite-difference lattice
Boltzmann model (Chen, Xu, Zhang, Li; Sec. II-IV of the paper).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.
"""

from .oracle import (  # noqa: F401
    OracleParams,
    build,
    lib_path,
    matrices,
    feq_moments,
    feq_moments_complex,
    node_equilibrium_complex,
    init,
    moments,
    run,
    init_complex,
    run_complex,
    moments_complex,
    max_threads,
)
