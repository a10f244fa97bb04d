"""Reference oracle for the exponential Rosenbrock-Euler (ER) transient solver
with the invert-Krylov matrix-exponential-vector product (Zhuang et al.,
DAC 2015, "An Algorithmic Framework for Efficient Large-Scale Circuit
Simulation Using Exponential Integrators").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 CPU
statement of what the solver computes, used to check the GPU library.  Only
the test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the GPU library and the library never
calls it.

Modules
  mosfet  -- level-1 (Shichman-Hodges) MOSFET current and Jacobian
  sources -- piecewise-linear source values, slopes, breakpoints
  mevp    -- Algorithm 1 (MEVP_IKS) and the small Hessenberg exponential
  er      -- Algorithm 2 (ER step, error estimate, step control), DC point
  mlp     -- the learned step controller's network: forward, gradient, Adam,
             bfloat16 inference (not part of the paper; its plain definition)

Every function is pinned by tests/test_oracle_*.py against closed forms,
brute force or invariants fixed by the paper and the mathematics.
"""
from .mosfet import mosfet_eval, device_currents
from .sources import source_values, source_slopes, breakpoints
from .mevp import InvertKrylov, hessenberg_phi
from .er import Options, Oracle, Trace
from . import mlp
