"""Seeded synthetic circuits shared by the solver's tests, its benchmark and
the oracle.  Holds circuit construction only, none of the solution method."""
from .netlist import GND, VDD, NMOS, PMOS, MOSFET_DTYPE, PWL, Netlist, canonical_csr
from .circuits import (Builder, rc_single, rc_ladder, tiny_linear, single_inverter, rc_mesh,
                       inverter_chain, power_grid, batch, batch_member, config, CONFIGS)
