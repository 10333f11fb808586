"""MI355X-native population annealing of the 2D Ising model.

The hot path (init, checkerboard Metropolis sweeps, energy histogram,
reweighting tables, copy counts, scan and gather-copy, observables, free
energy) runs in the HIP kernels of ``libpa.so``; ``binding`` marshals
arguments to its C ABI (``include/pa.h``).
"""
from .binding import (  # noqa: F401
    PA_BITS,
    PA_ECAPACITY,
    PA_EDEVICE,
    PA_EEMPTY,
    PA_EINVAL,
    PA_ENOMEM,
    PA_ESTATE,
    PA_FERRO,
    PA_INT8,
    PA_OK,
    PA_PMJ,
    MLP,
    Batch,
    PAError,
    Population,
    lib,
    strerror,
    tune_rows_per_lane,
)
