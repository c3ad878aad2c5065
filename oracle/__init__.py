"""FP64 CPU oracle of one GPUPEGAS timestep (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg import this package.  The GPU product path never does.
"""
from .oracle import (  # noqa: F401
    Oracle, OracleConfig, build, lib_path, riemann_gas, riemann_bme, dft3,
    poisson, poisson_isolated, DIAG_FIELDS, FIELD_NAMES, set_threads, get_threads,
)
