"""Oracle for population annealing of the 2D Ising model.

TEST INFRASTRUCTURE ONLY.  A plain, slow, single-threaded CPU implementation
of the method of the paper (Sec. 2, Eqs. part-F, part-Q, tau, Free-En; Sec. 3,
Eq. Ham), written in C (``pa_oracle.c``) and loaded here through ctypes.
Only the tests, the smoke entry point and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP path in
``paper_2006_00561_amd``, and neither imports the other.
"""
from .oracle import (  # noqa: F401
    ECAPACITY,
    EEMPTY,
    EINVAL,
    ENOMEM,
    NEAREST,
    MULTINOMIAL,
    OK,
    POISSON,
    RESIDUAL,
    RNG_PLANES,
    RNG_WORD,
    SYSTEMATIC,
    OraclePA,
    build,
    counts,
    energy,
    family_stats,
    lib,
    multinomial_pick,
    philox4x32_10,
    poisson_draw,
    site_draw,
    sweep_potts_replica,
    sweep_replica,
)
