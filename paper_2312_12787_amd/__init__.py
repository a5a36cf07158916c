"""MI355X (gfx950) hot path of the Calderon-ordered Burton-Miller collocation
BEM for 2-D Helmholtz transmission problems (arXiv 2312.12787).

The numerical work runs in the HIP kernels of libbem_hip.so behind the C ABI
of include/bem.h; ``bem`` is its thin ctypes binding.
"""
from .bem import (CALDERON, CALDERON_BETA1, CALDERON_ORIG, CONVENTIONAL, EXPORTS, F32, F64, MAX_RESTART, MIXED,  # noqa: F401
                  STATUS, BemError, Problem, SolveInfo, lib, solve_batch, tune_export, tune_import, tune_reset)
