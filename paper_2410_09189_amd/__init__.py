"""MI355X real-time TDDFT time step: HIP kernels for gfx950 behind a C ABI
(include/rt_tddft.h) and a thin ctypes binding (rt)."""

from . import rt  # noqa: F401
