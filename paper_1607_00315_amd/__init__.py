"""sic: sparse inverse covariance estimation on AMD Instinct MI355X (gfx950).

The solver (multilevel block coordinate descent for the l1-regularised
log-det problem) lives in the HIP library ``libsic.so`` behind a C-ABI
(``include/sic.h``, ``include/sic_steps.h``); ``sic`` is its Python binding.
"""

from . import sic  # noqa: F401
