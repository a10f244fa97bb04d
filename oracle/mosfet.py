"""Level-1 (Shichman-Hodges) MOSFET with channel-length modulation, no body
effect.

The paper evaluates BSIM3 devices to obtain the nonlinear current F and its
linearisation G_k at x_k (Algorithm 2, "derive C_k, G_k, F_k from device
models").  The level-1 model replaces BSIM3 here.  For an NMOS with drain a,
gate g, source b and V_a >= V_b:

    V_ov = V_gb - V_th
    cutoff      V_ov <= 0             I = 0
    triode      V_ab <  V_ov          I = K (V_ov V_ab - V_ab^2 / 2) (1 + lam V_ab)
    saturation  V_ab >= V_ov          I = K V_ov^2 / 2 (1 + lam V_ab)

with K = k' W/L.  The current and its first derivatives are continuous at
both region boundaries.  When V_d < V_s the terminals swap roles (I reverses).  A
PMOS is the mirror image: I_p(V_d, V_g, V_s) = -I_n(-V_d, -V_g, -V_s) with
the threshold magnitude |V_tp|.  I is the current entering the drain
terminal; the device draws I out of the drain node and returns it to the
source node.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

GND = -1
VDD = -2


def _forward(va, vg, vb, K, vth, lam):
    """Current from terminal a to terminal b (requires va >= vb) and its
    partial derivatives with respect to (va, vg, vb)."""
    vov = vg - vb - vth
    vds = va - vb
    f = np.zeros_like(va)
    f_ov = np.zeros_like(va)     # df/dV_ov
    f_ds = np.zeros_like(va)     # df/dV_ab
    on = vov > 0
    lin = on & (vds < vov)
    sat = on & ~lin
    q = 1.0 + lam * vds
    P = vov * vds - 0.5 * vds ** 2
    f[lin] = (K * P * q)[lin]
    f_ov[lin] = (K * vds * q)[lin]
    f_ds[lin] = (K * ((vov - vds) * q + P * lam))[lin]
    f[sat] = (0.5 * K * vov ** 2 * q)[sat]
    f_ov[sat] = (K * vov * q)[sat]
    f_ds[sat] = (0.5 * K * vov ** 2 * lam)[sat]
    return f, f_ds, f_ov, -f_ov - f_ds


def mosfet_eval(kind, vd, vg, vs, kp, wl, vth, lam):
    """Drain current I (into the drain terminal) and dI/dVd, dI/dVg, dI/dVs
    for arrays of devices.  kind is +1 (NMOS) or -1 (PMOS)."""
    kind = np.asarray(kind, dtype=np.float64)
    sgn = np.where(kind > 0, 1.0, -1.0)
    # the mirror image maps a PMOS onto an NMOS
    vd = sgn * np.asarray(vd, float)
    vg = sgn * np.asarray(vg, float)
    vs = sgn * np.asarray(vs, float)
    K = np.asarray(kp, float) * np.asarray(wl, float)
    vth = np.asarray(vth, float)
    lam = np.asarray(lam, float) + np.zeros_like(K)
    fwd = vd >= vs
    # forward: I = f(vd, vg, vs);  reverse: I = -f(vs, vg, vd)
    a = np.where(fwd, vd, vs)
    b = np.where(fwd, vs, vd)
    f, fa, fg, fb = _forward(a, vg, b, K, vth, lam)
    I = np.where(fwd, f, -f)
    dId = np.where(fwd, fa, -fb)
    dIg = np.where(fwd, fg, -fg)
    dIs = np.where(fwd, fb, -fa)
    # undo the mirror: I_p = -I_n(-v) so dI_p/dv = dI_n/dv' evaluated at -v
    return sgn * I, dId, dIg, dIs


def _terminal_voltage(x, node, vdd):
    v = np.zeros(node.shape, dtype=np.float64)
    inner = node >= 0
    v[inner] = x[node[inner]]
    v[node == VDD] = vdd
    return v


def device_currents(net, x):
    """I_dev(x): current drawn out of every node by the MOSFETs, and the
    Jacobian J_dev = dI_dev/dx as an n x n CSR matrix."""
    n = net.n
    dev = net.mosfets
    if dev.shape[0] == 0:
        return np.zeros(n), sp.csr_matrix((n, n))
    d, g, s = dev["d"].astype(np.int64), dev["g"].astype(np.int64), dev["s"].astype(np.int64)
    vd = _terminal_voltage(x, d, net.vdd)
    vg = _terminal_voltage(x, g, net.vdd)
    vs = _terminal_voltage(x, s, net.vdd)
    I, dId, dIg, dIs = mosfet_eval(dev["type"], vd, vg, vs, dev["kp"], dev["wl"], dev["vth"],
                                   dev["lam"])
    Idev = np.zeros(n)
    rows, cols, vals = [], [], []
    for node, sign in ((d, 1.0), (s, -1.0)):
        inner = node >= 0
        np.add.at(Idev, node[inner], sign * I[inner])
        for col, der in ((d, dId), (g, dIg), (s, dIs)):
            ok = inner & (col >= 0)
            rows.append(node[ok]); cols.append(col[ok]); vals.append(sign * der[ok])
    J = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    return Idev, J
