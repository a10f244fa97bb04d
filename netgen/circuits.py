"""Seeded synthetic circuits.

The paper's own circuits (ckt1-ckt8, the FreeCPU parasitics, BSIM3 models)
are not public; these generators stand in for them with the shapes, value
distributions and structure of the workloads the solver is measured on:

* ``rc_mesh``        -- linear power-grid-like RC mesh with pulse loads
                        (singular C on the capless nodes).
* ``inverter_chain`` -- CMOS inverters joined by RC ladders with coupling caps
                        and a ramp input (level-1 MOSFETs, singular C).
* ``batch``          -- many variants of one chain topology (same sparsity,
                        perturbed values) plus chains of uneven length.
* ``rc_single``, ``rc_ladder``, ``tiny_linear``, ``single_inverter`` -- small
  circuits whose exact responses are known in closed form or by brute force.

Every routine draws from ``numpy.random.Generator(PCG64(seed))`` only.  Node
ids are 0-based unknowns; GND (-1) and VDD (-2) are ideal rails.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .netlist import GND, VDD, NMOS, PMOS, MOSFET_DTYPE, PWL, Netlist, canonical_csr

FF = 1e-15
PS = 1e-12
NS = 1e-9


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


class Builder:
    """Collects linear elements, sources and MOSFETs into a Netlist."""

    def __init__(self, vdd: float = 1.0):
        self.n = 0
        self.vdd = vdd
        self._g = ([], [], [])
        self._c = ([], [], [])
        self._b = ([], [], [])
        self.sources: list[PWL] = []
        self.devs: list[tuple] = []

    def node(self) -> int:
        self.n += 1
        return self.n - 1

    def nodes(self, k: int) -> np.ndarray:
        ids = np.arange(self.n, self.n + k, dtype=np.int64)
        self.n += k
        return ids

    @staticmethod
    def _stamp(store, a, b, val):
        r, c, v = store
        if a >= 0:
            r.append(a); c.append(a); v.append(val)
        if b >= 0:
            r.append(b); c.append(b); v.append(val)
        if a >= 0 and b >= 0:
            r.append(a); c.append(b); v.append(-val)
            r.append(b); c.append(a); v.append(-val)

    def resistor(self, a: int, b: int, ohms: float):
        if not ohms > 0:
            raise ValueError("resistance must be positive")
        self._stamp(self._g, a, b, 1.0 / ohms)

    def conductance(self, a: int, b: int, siemens: float):
        self._stamp(self._g, a, b, siemens)

    def resistors(self, a, b, ohms):
        """Many resistors at once: a[i] -- b[i] with ohms[i] (inner nodes only)."""
        a = np.asarray(a, np.int64); b = np.asarray(b, np.int64)
        g = 1.0 / np.asarray(ohms, np.float64)
        if a.size == 0:
            return
        if not (np.all(a >= 0) and np.all(b >= 0) and np.all(np.isfinite(g)) and np.all(g > 0)):
            raise ValueError("bulk resistors need inner nodes and positive resistances")
        r, c, v = self._g
        r.extend(np.concatenate([a, b, a, b]).tolist())
        c.extend(np.concatenate([a, b, b, a]).tolist())
        v.extend(np.concatenate([g, g, -g, -g]).tolist())

    def ground_capacitors(self, nodes, farads):
        """Many capacitors from inner nodes to ground at once."""
        nodes = np.asarray(nodes, np.int64)
        f = np.asarray(farads, np.float64)
        if nodes.size and not (np.all(nodes >= 0) and np.all(f > 0)):
            raise ValueError("bulk capacitors need inner nodes and positive values")
        r, c, v = self._c
        r.extend(nodes.tolist()); c.extend(nodes.tolist()); v.extend(f.tolist())

    def capacitor(self, a: int, b: int, farads: float):
        if not farads > 0:
            raise ValueError("capacitance must be positive")
        self._stamp(self._c, a, b, farads)

    def voltage_source(self, node: int, series_ohms: float, wave: PWL):
        """Voltage source wave(t) in series with series_ohms, entered as its
        Norton equivalent: a conductance 1/R to ground and an injected
        current wave(t)/R."""
        g = 1.0 / series_ohms
        self.conductance(node, GND, g)
        self._b[0].append(node); self._b[1].append(len(self.sources)); self._b[2].append(g)
        self.sources.append(wave)

    def current_load(self, node: int, wave: PWL):
        """Current wave(t) drawn out of node (to ground)."""
        self._b[0].append(node); self._b[1].append(len(self.sources)); self._b[2].append(-1.0)
        self.sources.append(wave)

    def mosfet(self, kind: int, d: int, g: int, s: int, kp: float, wl: float, vth: float,
               lam: float = 0.05):
        self.devs.append((kind, d, g, s, kp, wl, vth, lam))

    def build(self, name: str, T: float, tol: float = 1e-6, probes=(), **meta) -> Netlist:
        n = self.n
        def mat(store, shape):
            r, c, v = store
            return canonical_csr(sp.coo_matrix((np.asarray(v, float), (np.asarray(r), np.asarray(c))),
                                               shape=shape))
        G = mat(self._g, (n, n))
        C = mat(self._c, (n, n))
        B = mat(self._b, (n, len(self.sources)))
        devs = np.array(self.devs, dtype=MOSFET_DTYPE) if self.devs else np.zeros(0, MOSFET_DTYPE)
        return Netlist(name=name, n=n, G=G, C=C, B=B, sources=list(self.sources), mosfets=devs,
                       vdd=self.vdd, T=T, tol=tol, probes=np.asarray(probes, np.int32), meta=meta)


# ----------------------------------------------------------------------------
# Small circuits with known responses
# ----------------------------------------------------------------------------

def rc_single(R: float = 1e3, Cap: float = 1e-12, wave: str = "step", amp: float = 1.0,
              T: float = 5e-9) -> Netlist:
    """One node: a source through R charging C to ground.

    wave="step": the source holds amp for all t (start the transient from
    x = 0 to see the step response),
    wave="ramp": the source is amp * t / T on [0, T]."""
    b = Builder()
    x = b.node()
    if wave == "step":
        src = PWL([0.0], [amp])
    elif wave == "ramp":
        src = PWL([0.0, T], [0.0, amp])
    else:
        raise ValueError(wave)
    b.voltage_source(x, R, src)
    b.capacitor(x, GND, Cap)
    return b.build(f"rc_single_{wave}", T=T, probes=[x], R=R, Cap=Cap, amp=amp, wave=wave)


def rc_ladder(N: int = 16, R: float = 100.0, c: float = 10e-15, Vs: float = 1.0,
              T: float = 2e-10) -> Netlist:
    """Uniform ladder: a constant source Vs through R into node 0, R between
    neighbours, cap c at every node, the far end open.  Its conductance
    matrix is (1/R) tridiag(-1, 2, -1) with the last diagonal entry 1.
    Started from x = 0 this gives the ladder's step response."""
    b = Builder()
    xs = b.nodes(N)
    b.voltage_source(int(xs[0]), R, PWL([0.0], [Vs]))
    for i in range(N - 1):
        b.resistor(int(xs[i]), int(xs[i + 1]), R)
    for i in range(N):
        b.capacitor(int(xs[i]), GND, c)
    return b.build(f"rc_ladder_{N}", T=T, probes=list(range(N)), R=R, c=c, Vs=Vs, N=N)


def tiny_linear(seed: int, n: int = 8, n_capless: int = 3) -> Netlist:
    """A random connected linear RC circuit of n <= 8 nodes with n_capless
    nodes that carry no capacitance (singular C), one coupling cap between two
    capacitive nodes and one PWL voltage source with two ramps."""
    rng = _rng(seed)
    b = Builder()
    xs = b.nodes(n)
    # random spanning tree plus a few extra edges
    order = rng.permutation(n)
    for k in range(1, n):
        a = int(order[k]); p = int(order[rng.integers(0, k)])
        b.resistor(a, p, float(_log_uniform(rng, 10.0, 1e3)))
    for _ in range(n // 2):
        a, c2 = rng.choice(n, 2, replace=False)
        b.resistor(int(a), int(c2), float(_log_uniform(rng, 10.0, 1e3)))
    capless = set(int(i) for i in rng.choice(n, n_capless, replace=False))
    capn = [i for i in range(n) if i not in capless]
    for i in capn:
        b.capacitor(i, GND, float(_log_uniform(rng, 1 * FF, 50 * FF)))
    if len(capn) >= 2:
        a, c2 = rng.choice(capn, 2, replace=False)
        b.capacitor(int(a), int(c2), float(rng.uniform(1 * FF, 5 * FF)))
    drive = int(rng.integers(0, n))
    b.conductance(int(rng.integers(0, n)), GND, 1e-3)
    t1 = float(rng.uniform(10 * PS, 40 * PS)); t2 = t1 + float(rng.uniform(20 * PS, 60 * PS))
    b.voltage_source(drive, 50.0, PWL([0.0, t1, t2], [0.0, 1.0, 0.4]))
    return b.build(f"tiny_linear_{seed}", T=150 * PS, probes=list(range(n)),
                   capless=sorted(capless))


def single_inverter(seed: int = 7, t_ramp: float = 50 * PS, T: float = 150 * PS) -> Netlist:
    """One CMOS inverter driving an RC load; ramp input on its gate."""
    rng = _rng(seed)
    b = Builder()
    gate, out, far = b.node(), b.node(), b.node()
    b.voltage_source(gate, 10.0, PWL([0.0, 10 * PS, 10 * PS + t_ramp], [0.0, 0.0, 1.0]))
    b.capacitor(gate, GND, 1 * FF)
    b.capacitor(out, GND, 0.5 * FF)
    b.conductance(out, GND, 1e-12)
    b.resistor(out, far, 200.0)
    b.capacitor(far, GND, 5 * FF)
    b.mosfet(PMOS, out, gate, VDD, 200e-6, 4.0, 0.3)
    b.mosfet(NMOS, out, gate, GND, 200e-6, 2.0, 0.3)
    return b.build("single_inverter", T=T, probes=[gate, out, far])


# ----------------------------------------------------------------------------
# RC mesh with pulse loads (linear)
# ----------------------------------------------------------------------------

def rc_mesh(seed: int = 1001, side: int = 32, T: float = 5 * NS, stim_seed: int = 2001,
            n_loads: int = 16, cap_frac: float = 0.8) -> Netlist:
    """side x side single-layer mesh.  Edge resistors log-uniform 0.1-10 ohm;
    ground caps log-uniform 1-100 fF on a random cap_frac of the nodes (C is
    singular on the rest); four corner Vdd = 1 V pads through 0.01 ohm;
    n_loads pulse current loads 0 -> 5 mA with 50 ps edges, period
    U(0.2, 1) ns, 50 % duty and start delay U(0, period)."""
    rng = _rng(seed)
    srng = _rng(stim_seed)
    b = Builder()
    ids = b.nodes(side * side).reshape(side, side)
    for i in range(side):
        for j in range(side):
            if j + 1 < side:
                b.resistor(int(ids[i, j]), int(ids[i, j + 1]), float(_log_uniform(rng, 0.1, 10.0)))
            if i + 1 < side:
                b.resistor(int(ids[i, j]), int(ids[i + 1, j]), float(_log_uniform(rng, 0.1, 10.0)))
    n = side * side
    capn = rng.choice(n, int(round(cap_frac * n)), replace=False)
    for k in np.sort(capn):
        b.capacitor(int(k), GND, float(_log_uniform(rng, 1 * FF, 100 * FF)))
    for (i, j) in ((0, 0), (0, side - 1), (side - 1, 0), (side - 1, side - 1)):
        b.voltage_source(int(ids[i, j]), 0.01, PWL([0.0], [1.0]))
    load_nodes = rng.choice(n, n_loads, replace=False)
    edge = 50 * PS
    for node in load_nodes:
        period = float(srng.uniform(0.2 * NS, 1.0 * NS))
        delay = float(srng.uniform(0.0, period))
        ts, vs = [0.0], [0.0]
        t0 = delay
        while t0 < T:
            for (tt, vv) in ((t0, 0.0), (t0 + edge, 5e-3), (t0 + period / 2, 5e-3),
                             (t0 + period / 2 + edge, 0.0)):
                if tt > ts[-1]:
                    ts.append(tt); vs.append(vv)
            t0 += period
        b.current_load(int(node), PWL(ts, vs))
    probes = np.unique(np.concatenate([load_nodes, [ids[side // 2, side // 2]]]))
    return b.build(f"rc_mesh_{side}x{side}", T=T, probes=probes, seed=seed, capless=n - len(capn))


# ----------------------------------------------------------------------------
# CMOS inverter chains with RC ladders (nonlinear)
# ----------------------------------------------------------------------------

def inverter_chain(seed: int = 1002, n_stages: int = 200, n_seg: int = 10, T: float = 4 * NS,
                   t_ramp: float = 2 * NS, stim_seed: int = 2002, base: dict | None = None,
                   variation: dict | None = None) -> Netlist:
    """Chain of CMOS inverters between ideal rails (Vdd = 1 V).

    Stage s drives a ladder of n_seg T-sections (R/2, C to ground, R/2) whose
    far end is the gate of stage s+1, so each stage adds 1 + 2*n_seg nodes and
    the chain has n_stages*(1 + 2*n_seg) + 1 nodes.  Segment R ~ U(5, 50) ohm,
    C ~ U(0.5, 5) fF; coupling caps U(0.1, 1) fF join same-index mid nodes of
    neighbouring ladders.  Drain nodes carry 0.5 fF and gmin = 1e-12 S to
    ground, gate nodes 1 fF.  MOSFETs: V_th U(0.28, 0.32) V, k' U(100, 300)
    uA/V^2, W/L U(1, 8), lambda = 0.05 / V.  The first gate is driven through 10 ohm by a ramp
    0 -> 1 V of duration t_ramp (after an optional delay).

    ``base``: element values of an earlier call (returned in meta['values'])
    to re-use instead of drawing fresh ones; ``variation``: per-instance
    multiplicative R/C factors U(1 - rc, 1 + rc), additive V_th noise
    N(0, vth_sigma) and input delay U(0, delay_max), drawn from
    variation['seed'].
    """
    rng = _rng(seed)
    srng = _rng(stim_seed)
    per_stage = 1 + 2 * n_seg
    if base is None:
        vals = dict(
            R=rng.uniform(5.0, 50.0, (n_stages, n_seg)),
            C=rng.uniform(0.5 * FF, 5 * FF, (n_stages, n_seg)),
            Cc=rng.uniform(0.1 * FF, 1 * FF, (max(n_stages - 1, 0), n_seg)),
            vth=rng.uniform(0.28, 0.32, (n_stages, 2)),
            kp=rng.uniform(100e-6, 300e-6, (n_stages, 2)),
            wl=rng.uniform(1.0, 8.0, (n_stages, 2)),
            delay=0.0,
        )
    else:
        vals = {k: (np.array(v, copy=True) if isinstance(v, np.ndarray) else v) for k, v in base.items()}
    if variation is not None:
        vr = _rng(variation["seed"])
        rc = variation.get("rc", 0.1)
        vals["R"] = vals["R"] * vr.uniform(1 - rc, 1 + rc, vals["R"].shape)
        vals["C"] = vals["C"] * vr.uniform(1 - rc, 1 + rc, vals["C"].shape)
        vals["Cc"] = vals["Cc"] * vr.uniform(1 - rc, 1 + rc, vals["Cc"].shape)
        vals["vth"] = vals["vth"] + vr.normal(0.0, variation.get("vth_sigma", 0.02), vals["vth"].shape)
        vals["delay"] = float(vr.uniform(0.0, variation.get("delay_max", 0.5 * NS)))
    b = Builder(vdd=1.0)
    gate = b.node()
    delay = float(vals["delay"])
    if delay > 0:
        wave = PWL([0.0, delay, delay + t_ramp], [0.0, 0.0, 1.0])
    else:
        wave = PWL([0.0, t_ramp], [0.0, 1.0])
    b.voltage_source(gate, 10.0, wave)
    b.capacitor(gate, GND, 1 * FF)
    mids_prev = None
    outs = []
    for s in range(n_stages):
        out = b.node()
        outs.append(out)
        b.capacitor(out, GND, 0.5 * FF)
        b.conductance(out, GND, 1e-12)
        b.mosfet(PMOS, out, gate, VDD, vals["kp"][s, 0], vals["wl"][s, 0], vals["vth"][s, 0])
        b.mosfet(NMOS, out, gate, GND, vals["kp"][s, 1], vals["wl"][s, 1], vals["vth"][s, 1])
        prev = out
        mids = []
        for k in range(n_seg):
            mid = b.node(); end = b.node()
            half = vals["R"][s, k] / 2
            b.resistor(prev, mid, half)
            b.capacitor(mid, GND, vals["C"][s, k])
            b.resistor(mid, end, half)
            mids.append(mid)
            prev = end
        if mids_prev is not None:
            for k in range(n_seg):
                b.capacitor(mids_prev[k], mids[k], vals["Cc"][s - 1, k])
        mids_prev = mids
        gate = prev
        b.capacitor(gate, GND, 1 * FF)
    assert b.n == n_stages * per_stage + 1
    probes = [0] + outs[:: max(1, n_stages // 20)] + [b.n - 1]
    return b.build(f"inverter_chain_{n_stages}", T=T, probes=sorted(set(probes)),
                   values=vals, seed=seed, n_stages=n_stages)


def power_grid(seed: int = 1003, side: int = 512, T: float = 2 * NS, stim_seed: int = 2003,
               n_drivers: int = 2000, via_pitch: int = 8, cap_frac: float = 0.7) -> Netlist:
    """Post-layout-style power grid: two side x side resistive layers.

    Layer 0 (top) holds nodes 0 .. side^2 - 1, layer 1 (bottom) the next
    side^2, both row-major.  In-layer edge resistors are log-uniform
    0.1-10 ohm; ground caps log-uniform 1-100 fF sit on a random cap_frac of
    the grid nodes (C is singular on the rest); vias U(0.5, 2) ohm join the
    layers at every via_pitch-th row and column; four corner Vdd = 1 V pads
    on the top layer through 0.01 ohm.  n_drivers CMOS inverters (the chain's
    level-1 parameter ranges) sit on distinct random bottom-layer nodes: the
    PMOS source on the grid node, the NMOS source on ground, a private gate
    node (1 fF) driven through 10 ohm by a ramp, and a private output node with
    a U(5, 20) fF load, 0.5 fF and gmin = 1e-12 S.  Each input makes one
    0 <-> 1 V edge of 50 ps at U(0.1, 1.5) ns, in a random direction.  Node
    ids: the grid first, then (gate, output) per driver."""
    rng = _rng(seed)
    srng = _rng(stim_seed)
    b = Builder(vdd=1.0)
    per = side * side
    grid = b.nodes(2 * per).reshape(2, side, side)
    for layer in range(2):
        g = grid[layer]
        b.resistors(g[:, :-1].ravel(), g[:, 1:].ravel(), _log_uniform(rng, 0.1, 10.0, side * (side - 1)))
        b.resistors(g[:-1, :].ravel(), g[1:, :].ravel(), _log_uniform(rng, 0.1, 10.0, side * (side - 1)))
    vi = np.arange(0, side, via_pitch)
    top = grid[0][np.ix_(vi, vi)].ravel()
    bot = grid[1][np.ix_(vi, vi)].ravel()
    b.resistors(top, bot, rng.uniform(0.5, 2.0, top.size))
    capn = np.sort(rng.choice(2 * per, int(round(cap_frac * 2 * per)), replace=False))
    b.ground_capacitors(capn, _log_uniform(rng, 1 * FF, 100 * FF, capn.size))
    for (i, j) in ((0, 0), (0, side - 1), (side - 1, 0), (side - 1, side - 1)):
        b.voltage_source(int(grid[0, i, j]), 0.01, PWL([0.0], [1.0]))
    sites = grid[1].ravel()[np.sort(rng.choice(per, n_drivers, replace=False))]
    vth = rng.uniform(0.28, 0.32, (n_drivers, 2))
    kp = rng.uniform(100e-6, 300e-6, (n_drivers, 2))
    wl = rng.uniform(1.0, 8.0, (n_drivers, 2))
    cload = rng.uniform(5 * FF, 20 * FF, n_drivers)
    edge = 50 * PS
    t_edge = srng.uniform(0.1 * NS, 1.5 * NS, n_drivers)
    rising = srng.random(n_drivers) < 0.5
    outs = []
    for k in range(n_drivers):
        gate, out = b.node(), b.node()
        lo, hi = (0.0, 1.0) if rising[k] else (1.0, 0.0)
        b.voltage_source(gate, 10.0, PWL([0.0, t_edge[k], t_edge[k] + edge], [lo, lo, hi]))
        b.capacitor(gate, GND, 1 * FF)
        b.capacitor(out, GND, 0.5 * FF + cload[k])
        b.conductance(out, GND, 1e-12)
        b.mosfet(PMOS, out, gate, int(sites[k]), kp[k, 0], wl[k, 0], vth[k, 0])
        b.mosfet(NMOS, out, gate, GND, kp[k, 1], wl[k, 1], vth[k, 1])
        outs.append(out)
    probes = np.unique(np.concatenate([sites[:: max(1, n_drivers // 16)], np.asarray(outs[:: max(1, n_drivers // 16)]),
                                       [grid[0, side // 2, side // 2], grid[1, side // 2, side // 2]]]))
    return b.build(f"power_grid_2x{side}x{side}", T=T, probes=probes, seed=seed, side=side,
                   n_drivers=n_drivers, sites=sites)


def batch(seed: int = 1004, n_variants: int = 256, n_uneven: int = 64, stages_lo: int = 50,
          stages_hi: int = 400, n_stages: int = 200, T: float = 4 * NS) -> list:
    """n_variants perturbed copies of one inverter-chain topology (identical
    sparsity; per-instance R/C x U(0.9, 1.1), V_th + N(0, 20 mV), input delay
    U(0, 0.5 ns)) followed by n_uneven chains of U{stages_lo..stages_hi}
    stages, each with its own values and pattern."""
    rng = _rng(seed)
    base = inverter_chain(seed=seed, n_stages=n_stages, T=T).meta["values"]
    out = []
    for i in range(n_variants):
        out.append(inverter_chain(seed=seed, n_stages=n_stages, T=T, base=base,
                                  variation=dict(seed=3000 + i)))
    lengths = rng.integers(stages_lo, stages_hi + 1, n_uneven)
    for j, L in enumerate(lengths):
        out.append(inverter_chain(seed=3000 + n_variants + j, n_stages=int(L), T=T))
    return out


def batch_member(i: int, seed: int = 1004, n_variants: int = 256, n_uneven: int = 64, stages_lo: int = 50,
                 stages_hi: int = 400, n_stages: int = 200, T: float = 4 * NS) -> Netlist:
    """Instance i of batch(...) with the same arguments, built alone."""
    if i < n_variants:
        base = inverter_chain(seed=seed, n_stages=n_stages, T=T).meta["values"]
        return inverter_chain(seed=seed, n_stages=n_stages, T=T, base=base, variation=dict(seed=3000 + i))
    j = i - n_variants
    if not 0 <= j < n_uneven:
        raise IndexError(i)
    lengths = _rng(seed).integers(stages_lo, stages_hi + 1, n_uneven)
    return inverter_chain(seed=3000 + n_variants + j, n_stages=int(lengths[j]), T=T)


CONFIGS = {
    1: "rc_mesh 32x32, 1,024 nodes, linear, 16 pulse loads, T = 5 ns",
    2: "inverter chain, 200 stages x 10-segment ladders, 4,201 nodes, 400 MOSFETs, T = 4 ns",
    3: "power grid 2 x 512 x 512 + 2,000 inverter drivers, 528,288 nodes, 4,000 MOSFETs, T = 2 ns",
    4: "batch of 256 chain variants (shared sparsity) + 64 chains of 50-400 stages, T = 4 ns",
}


def config(cid: int, **kw):
    """The seeded workloads: 1 = RC mesh, 2 = inverter chain, 3 = power grid, 4 = batch."""
    if cid == 1:
        return rc_mesh(seed=1001, stim_seed=2001, **kw)
    if cid == 2:
        return inverter_chain(seed=1002, stim_seed=2002, **kw)
    if cid == 3:
        return power_grid(seed=1003, stim_seed=2003, **kw)
    if cid == 4:
        return batch(seed=1004, **kw)
    raise ValueError(f"unknown config {cid}")
