"""expri: MI355X (gfx950) exponential Rosenbrock-Euler transient solver with
the invert-Krylov matrix-exponential-vector product.

The numerical work lives in libexpri.so (C-ABI in include/expri.h, HIP
kernels in csrc/); this package holds the build step and a thin ctypes
binding that passes PyTorch device memory and streams to it."""
from .binding import (Solver, Opts, RunInfo, ExpriError, STATUS, ENTRY_POINTS, REC_FIELDS,
                      default_opts, load_library, LIB_PATH, symbolic_analysis, frontal_analysis, autotune_runs, Mlp,
                      MLP_PARAMS,
                      MLP_NORM)
