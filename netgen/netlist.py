"""Circuit data handed to both the solver library and the oracle.

The paper's problem statement (Background, the circuit DAE) is
    d q(x)/dt + f(x) = B u(t).
For the circuits generated here q(x) = C x with a constant, symmetric,
positive semi-definite (possibly singular) capacitance matrix C, and
    f(x) = G_lin x + I_dev(x),
where G_lin holds every linear conductance (resistors, Norton source
conductances, gmin) and I_dev(x) is the current that the MOSFETs draw out of
each node.  B is the incidence of the independent sources and u(t) holds
their piecewise-linear waveforms.

This module only stores those arrays.  It contains no part of the solution
method: no device evaluation, no PWL interpolation, no factorisation.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

GND = -1   # node id of the ideal ground rail (0 V)
VDD = -2   # node id of the ideal supply rail (Netlist.vdd volts)

NMOS = 1
PMOS = -1

MOSFET_DTYPE = np.dtype([
    ("type", np.int8),     # +1 NMOS, -1 PMOS
    ("d", np.int32),       # drain node (or GND / VDD)
    ("g", np.int32),       # gate node (or GND / VDD)
    ("s", np.int32),       # source node (or GND / VDD)
    ("kp", np.float64),    # process transconductance k' in A/V^2
    ("wl", np.float64),    # W/L ratio
    ("vth", np.float64),   # threshold magnitude in V (PMOS uses |V_tp|)
    ("lam", np.float64),   # channel-length modulation lambda in 1/V
])


@dataclass
class PWL:
    """One source waveform: value v[i] at time t[i]; linear in between,
    constant before t[0] and after t[-1].  t is strictly increasing."""
    t: np.ndarray
    v: np.ndarray

    def __post_init__(self):
        self.t = np.ascontiguousarray(self.t, dtype=np.float64)
        self.v = np.ascontiguousarray(self.v, dtype=np.float64)
        if self.t.ndim != 1 or self.t.shape != self.v.shape or self.t.size < 1:
            raise ValueError("PWL needs equal-length 1-D t and v")
        if self.t.size > 1 and not np.all(np.diff(self.t) > 0):
            raise ValueError("PWL times must be strictly increasing")


@dataclass
class Netlist:
    name: str
    n: int
    G: sp.csr_matrix                 # n x n linear conductance matrix (S)
    C: sp.csr_matrix                 # n x n capacitance matrix (F), symmetric PSD
    B: sp.csr_matrix                 # n x n_src source incidence
    sources: list                    # list[PWL], one per column of B
    mosfets: np.ndarray              # structured array of MOSFET_DTYPE
    vdd: float = 1.0
    T: float = 1e-9                  # transient end time (s)
    tol: float = 1e-6                # error budget E_rr (V)
    probes: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    meta: dict = field(default_factory=dict)

    @property
    def n_src(self) -> int:
        return self.B.shape[1]

    @property
    def n_dev(self) -> int:
        return int(self.mosfets.shape[0])

    def breakpoints(self) -> np.ndarray:
        """Sorted union of every source's PWL corner times."""
        if not self.sources:
            return np.zeros(0)
        return np.unique(np.concatenate([s.t for s in self.sources]))

    def same_pattern(self, other: "Netlist") -> bool:
        """True when G, C and B of both netlists have identical sparsity."""
        def eq(a, b):
            return (a.shape == b.shape and np.array_equal(a.indptr, b.indptr)
                    and np.array_equal(a.indices, b.indices))
        return (self.n == other.n and eq(self.G, other.G) and eq(self.C, other.C)
                and eq(self.B, other.B) and self.n_dev == other.n_dev
                and all(np.array_equal(self.mosfets[k], other.mosfets[k])
                        for k in ("type", "d", "g", "s")))


def canonical_csr(m) -> sp.csr_matrix:
    """CSR with summed duplicates and sorted column indices (int32 indices)."""
    m = sp.csr_matrix(m)
    m.sum_duplicates()
    m.sort_indices()
    m.indptr = m.indptr.astype(np.int32)
    m.indices = m.indices.astype(np.int32)
    m.data = m.data.astype(np.float64)
    return m
