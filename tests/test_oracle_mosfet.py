"""Pins of the oracle's level-1 MOSFET model (hand values, finite
differences, continuity, charge conservation)."""
import numpy as np
import pytest

import netgen
from oracle import mosfet_eval, device_currents


def test_hand_value_saturation_no_clm():
    # k' = 200 uA/V^2, W/L = 2, Vgs = Vds = 1 V, Vth = 0.3 V: I = K/2 (0.7)^2 = 98 uA
    I, *_ = mosfet_eval([1], [1.0], [1.0], [0.0], 200e-6, 2.0, 0.3, 0.0)
    assert I[0] == pytest.approx(98e-6, rel=1e-14)


def test_hand_value_with_clm_and_triode():
    # saturation with lambda = 0.05: 98 uA * (1 + 0.05 * 1)
    I, *_ = mosfet_eval([1], [1.0], [1.0], [0.0], 200e-6, 2.0, 0.3, 0.05)
    assert I[0] == pytest.approx(98e-6 * 1.05, rel=1e-14)
    # triode Vgs = 1, Vds = 0.2: K (0.7*0.2 - 0.02)(1 + 0.01) = 4e-4 * 0.12 * 1.01
    I, *_ = mosfet_eval([1], [0.2], [1.0], [0.0], 200e-6, 2.0, 0.3, 0.05)
    assert I[0] == pytest.approx(4e-4 * 0.12 * 1.01, rel=1e-14)
    # cutoff
    I, *_ = mosfet_eval([1], [1.0], [0.29], [0.0], 200e-6, 2.0, 0.3, 0.05)
    assert I[0] == 0.0


def test_pmos_is_mirror_and_reverse_is_antisymmetric():
    # PMOS source at 1 V, gate 0, drain 0: the mirror of an NMOS with Vgs = Vds = 1
    Ip, *_ = mosfet_eval([-1], [0.0], [0.0], [1.0], 200e-6, 2.0, 0.3, 0.05)
    In, *_ = mosfet_eval([1], [1.0], [1.0], [0.0], 200e-6, 2.0, 0.3, 0.05)
    assert Ip[0] == pytest.approx(-In[0], rel=1e-15)
    # swapping drain and source reverses the current
    a, *_ = mosfet_eval([1], [0.3], [1.0], [0.1], 1e-4, 3.0, 0.3, 0.05)
    b, *_ = mosfet_eval([1], [0.1], [1.0], [0.3], 1e-4, 3.0, 0.3, 0.05)
    assert a[0] == pytest.approx(-b[0], rel=1e-15)


@pytest.mark.parametrize("kind", [1, -1])
def test_jacobian_matches_central_differences(kind):
    rng = np.random.default_rng(4)
    N = 4000
    vd, vg, vs = (rng.uniform(-0.2, 1.2, N) for _ in range(3))
    kp, wl, vth, lam = 150e-6, 3.0, 0.3, 0.05
    I, dd, dg, ds = mosfet_eval(np.full(N, kind), vd, vg, vs, kp, wl, vth, lam)
    eps = 1e-7
    for k, der in enumerate((dd, dg, ds)):
        up = [vd.copy(), vg.copy(), vs.copy()]
        dn = [vd.copy(), vg.copy(), vs.copy()]
        up[k] += eps
        dn[k] -= eps
        fd = (mosfet_eval(np.full(N, kind), *up, kp, wl, vth, lam)[0]
              - mosfet_eval(np.full(N, kind), *dn, kp, wl, vth, lam)[0]) / (2 * eps)
        scale = np.maximum(np.abs(der), 1e-6)
        assert np.max(np.abs(fd - der) / scale) < 1e-5


def test_current_and_derivatives_continuous_at_region_boundaries():
    K, vth, lam = 200e-6 * 2, 0.3, 0.05
    d = 1e-9
    for (vd0, vg0, vs0) in [(0.5, 0.3, 0.0),      # cutoff / on boundary
                            (0.4, 0.7, 0.0),      # triode / saturation boundary
                            (0.2, 0.8, 0.2)]:     # drain-source swap point
        lo = np.array(mosfet_eval([1], [vd0 - d], [vg0], [vs0], K, 1.0, vth, lam)).ravel()
        hi = np.array(mosfet_eval([1], [vd0 + d], [vg0], [vs0], K, 1.0, vth, lam)).ravel()
        assert np.max(np.abs(hi - lo)) < 1e-9
        lo = np.array(mosfet_eval([1], [vd0], [vg0 - d], [vs0], K, 1.0, vth, lam)).ravel()
        hi = np.array(mosfet_eval([1], [vd0], [vg0 + d], [vs0], K, 1.0, vth, lam)).ravel()
        assert np.max(np.abs(hi - lo)) < 1e-9


def test_device_currents_conserve_charge_and_match_jacobian():
    net = netgen.single_inverter()
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.uniform(0, 1, net.n)
        I, J = device_currents(net, x)
        # every device is between unknown nodes and rails: the rail currents
        # balance the node currents, so check the Jacobian by differences
        eps = 1e-7
        for j in range(net.n):
            e = np.zeros(net.n); e[j] = eps
            fd = (device_currents(net, x + e)[0] - device_currents(net, x - e)[0]) / (2 * eps)
            assert np.allclose(fd, J.toarray()[:, j], rtol=1e-5, atol=1e-12)
    # a MOSFET between two unknown nodes draws from one what it returns to the other
    b = netgen.Builder()
    a, g, c = b.node(), b.node(), b.node()
    b.mosfet(1, a, g, c, 1e-4, 2.0, 0.3)
    net2 = b.build("pair", T=1e-12)
    I, _ = device_currents(net2, np.array([0.8, 1.0, 0.1]))
    assert I.sum() == pytest.approx(0.0, abs=1e-20) and I[0] > 0 and I[1] == 0.0
