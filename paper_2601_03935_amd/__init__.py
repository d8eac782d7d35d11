"""MI355X-native GSIS / DVM hot path for radiative polyatomic gas flows.

The product is ``libgsis.so`` (HIP kernels for gfx950 behind the C ABI in ``include/gsis.h``);
:mod:`paper_2601_03935_amd.gsis` is its ctypes binding.
"""

from .gsis import Solver, GsisError, default_opts, lib  # noqa: F401
