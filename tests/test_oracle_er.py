"""Pins of the oracle's exponential Rosenbrock-Euler transient (Algorithm 2)
against closed-form and brute-force responses, the DC invariant, the order of
the local error estimator and the step-control invariants."""
import numpy as np
import pytest

import netgen
from oracle import Oracle, Options
from tests.exact import ladder_step, linear_exact


def test_single_rc_step_and_ramp_are_exact():
    R, Cap = 1e3, 1e-12
    net = netgen.rc_single(R=R, Cap=Cap, wave="step")
    tr = Oracle(net).run(np.zeros(1))
    t = np.array(tr.t)
    x = np.array(tr.x)[:, 0]
    assert np.max(np.abs(x - (1 - np.exp(-t / (R * Cap))))) < 1e-13
    assert max(tr.m) == 1
    net = netgen.rc_single(R=R, Cap=Cap, wave="ramp")
    tr = Oracle(net).run(np.zeros(1))
    t = np.array(tr.t)
    x = np.array(tr.x)[:, 0]
    a = 1.0 / net.T
    assert np.max(np.abs(x - a * (t - R * Cap * (1 - np.exp(-t / (R * Cap)))))) < 1e-13


def test_rc_ladder_matches_modal_closed_form():
    N, R, c = 16, 100.0, 10e-15
    net = netgen.rc_ladder(N=N, R=R, c=c)
    tr = Oracle(net, Options(tol=1e-12)).run(np.zeros(N))
    X = np.array(tr.x)
    assert np.max(np.abs(X - ladder_step(N, R, c, 1.0, np.array(tr.t)))) < 1e-12
    # at the default tolerance the error stays within the Krylov budget
    tr = Oracle(net).run(np.zeros(N))
    assert np.max(np.abs(np.array(tr.x) - ladder_step(N, R, c, 1.0, np.array(tr.t)))) < 1e-6


@pytest.mark.parametrize("seed", range(10))
def test_singular_C_circuits_match_kron_reduced_exact(seed):
    net = netgen.tiny_linear(seed)
    o = Oracle(net, Options(tol=1e-12))
    x0 = o.dc()
    tr = o.run(x0)
    ex = linear_exact(net, x0, np.array(tr.t))
    assert np.max(np.abs(np.array(tr.x) - ex)) < 1e-12
    # every source corner inside (0, T) is a step end
    corners = [p for s in net.sources for p in s.t if 0 < p < net.T]
    assert set(corners) <= set(tr.t)


def test_literal_and_combined_modes_agree():
    net = netgen.tiny_linear(1)
    x0 = Oracle(net).dc()
    a = Oracle(net, Options(mode="combined")).run(x0)
    b = Oracle(net, Options(mode="literal")).run(x0)
    assert a.t == b.t
    assert np.max(np.abs(np.array(a.x) - np.array(b.x))) < 5e-7


def test_dc_invariant_and_linear_long_step_lands_on_dc():
    for net in (netgen.config(1), netgen.inverter_chain(n_stages=12), netgen.single_inverter()):
        o = Oracle(net)
        x0 = o.dc()
        r = o.residual_current(x0, 0.0)
        # scale: the largest current any single conductance carries
        scale = max(np.max(np.abs(o.B @ np.array([s.v[0] for s in net.sources]))),
                    np.max(abs(o.G) @ np.abs(x0)))
        assert np.max(np.abs(r)) <= 1e-10 * scale
    # linear: one step of 1000 s from x = 0 with a constant source lands on G^{-1} B u
    net = netgen.rc_ladder(N=12)
    tr = Oracle(net).replay(np.zeros(12), [1e3])
    assert np.max(np.abs(tr.x[-1] - 1.0)) < 1e-12
    net = netgen.config(1)
    G = net.G.toarray(); u = np.array([s.v[0] for s in net.sources])
    assert np.allclose(Oracle(net).dc(), np.linalg.solve(G, net.B @ u), rtol=0, atol=1e-12)


def test_dc_blocks_are_topological():
    net = netgen.inverter_chain(n_stages=6, n_seg=2)
    blocks = Oracle(net).dc_blocks()
    where = {}
    for b, mem in enumerate(blocks):
        for i in mem:
            where[int(i)] = b
    assert sorted(where) == list(range(net.n))
    for d in net.mosfets:
        if d["g"] >= 0 and d["d"] >= 0:
            assert where[int(d["g"])] <= where[int(d["d"])]


def test_error_estimate_is_third_order_in_h():
    # e_rr = (I - e^{hJ}) G^{-1} dF with dF = O(|x_{k+1} - x_k|^2) = O(h^2)
    net = netgen.single_inverter()
    o = Oracle(net)
    x0 = o.dc()
    tr = o.run(x0, T=40e-12)
    x, t = np.array(tr.x[-1]), tr.t[-1]
    hs = 1e-12 * 2.0 ** -np.arange(4, 9)
    errs = []
    for h in hs:
        o2 = Oracle(net, Options(tol=1e-12, eps_krylov=1e-14))
        o2.replay(x, [t + h], t0=t)
        errs.append(o2.trace.err[-1])
    local = np.diff(np.log(errs)) / np.diff(np.log(hs))
    # the local order rises towards 3 as h leaves the stiff regime
    assert np.all(np.diff(local) > -0.05)
    assert 2.8 < local[-1] < 3.15


def test_step_control_invariants_on_nonlinear_run():
    net = netgen.inverter_chain(n_stages=6, T=1.2e-9, t_ramp=0.3e-9)
    o = Oracle(net)
    x0 = o.dc()
    tr = o.run(x0, keep=None)
    # one LU per accepted step, none on rejection
    assert tr.lu_count == len(tr.t)
    assert sum(tr.rejects) > 0
    assert all(e <= o.E_rr for e in tr.err)
    assert tr.t[-1] == net.T
    assert np.all(np.diff(tr.t) > 0)
    # a rejection halves the step (alpha = 1/2) and nothing else changes it
    h_max = net.T / 20
    for hu, ht, i in zip(tr.h, tr.h_try, tr.rejects):
        assert hu == ht * 0.5 ** i and ht <= h_max
    # growth: after a first-try accept the next unclipped try doubles
    corners = set(p for s in net.sources for p in s.t if 0 < p < net.T) | {net.T}
    grew = 0
    for k in range(len(tr.t) - 1):
        if tr.rejects[k] == 0 and tr.t[k + 1] not in corners and tr.h_try[k] * 2 <= h_max:
            if tr.t[k] not in corners:
                assert tr.h_try[k + 1] == 2 * tr.h_try[k]
                grew += 1
    assert grew > 0


def test_replay_of_own_grid_agrees_and_is_deterministic():
    net = netgen.inverter_chain(n_stages=4, T=0.8e-9, t_ramp=0.2e-9)
    o = Oracle(net)
    x0 = o.dc()
    a = o.run(x0)
    b = Oracle(net).replay(x0, a.t)
    # run() builds each basis at the first trial h and reuses it after a
    # rejection; replay() builds it at the accepted h: equal to the Krylov tolerance
    assert np.max(np.abs(np.array(a.x) - np.array(b.x))) < 10 * 0.1 * net.tol
    c = Oracle(net).replay(x0, a.t)
    assert np.array_equal(np.array(b.x), np.array(c.x))


def test_erc_with_zero_gamma_is_er_and_correction_is_small():
    # ER-C subtracts gamma h phi_2(hJ) C^{-1} dF: gamma = 0 reproduces ER exactly,
    # and on a switching chain the correction stays of the order of the error budget
    net = netgen.inverter_chain(seed=77, n_stages=6, T=0.5e-9, t_ramp=0.2e-9)
    x0 = Oracle(net).dc()
    ts = Oracle(net).run(x0, keep=None).t
    er = Oracle(net).replay(x0, ts, keep="all")
    erc0 = Oracle(net, Options(erc=True, gamma=0.0)).replay(x0, ts, keep="all")
    assert np.array_equal(np.array(er.x), np.array(erc0.x))
    erc = Oracle(net, Options(erc=True, gamma=0.1)).replay(x0, ts, keep="all")
    diff = np.max(np.abs(np.array(erc.x) - np.array(er.x)))
    assert 0.0 < diff <= 20 * net.tol


def _one_node_nmos_circuit():
    """One node x: a capacitor to ground, a voltage source through R, and an
    NMOS with its drain on x, its gate on the supply rail and its source on
    ground.  The source falls linearly, so p and z are both non-zero."""
    b = netgen.Builder()
    x = b.node()
    R, Cap, kp, wl, vth, lam = 1e3, 1e-15, 200e-6, 2.0, 0.3, 0.05
    b.voltage_source(x, R, netgen.PWL([0.0, 10e-12], [0.2, 0.1]))
    b.capacitor(x, -1, Cap)
    b.mosfet(1, x, -2, -1, kp, wl, vth, lam)
    net = b.build("one_node_nmos", T=10e-12)
    return net, dict(g=1.0 / R, Cap=Cap, K=kp * wl, vov=1.0 - vth, lam=lam, u0=0.2, slope=-0.1 / 10e-12)


def _nmos_current(x, K, vov, lam):
    """Level-1 drain current of the grounded-source NMOS with V_gs = vov + V_th,
    V_ds = x >= 0, and its derivative in x (written out for this test)."""
    if x < vov:
        P = vov * x - 0.5 * x * x
        return K * P * (1 + lam * x), K * ((vov - x) * (1 + lam * x) + P * lam)
    return 0.5 * K * vov * vov * (1 + lam * x), 0.5 * K * vov * vov * lam


@pytest.mark.parametrize("h", [0.3e-12, 1e-12, 4e-12])
def test_one_step_of_er_and_erc_on_one_node_matches_scalar_closed_form(h):
    # With one unknown every matrix is a scalar and the Krylov space is exact
    # at m = 1.  The ER step (the closed forms after the ER equation), the
    # local error estimate and the ER-C correction (section on the modified
    # correction term: x_{k+1,c} = x_{k+1} - gamma h phi_2(hJ) C^{-1} dF) are
    # evaluated here from scalars, with phi_2(q) = (e^q - 1 - q) / q^2.
    net, c = _one_node_nmos_circuit()
    x0 = 0.9
    g, Cap, K, vov, lam = c["g"], c["Cap"], c["K"], c["vov"], c["lam"]
    I0, a = _nmos_current(x0, K, vov, lam)
    Gk = g + a
    q = -h * Gk / Cap                        # h J_k
    r = g * c["u0"] - g * x0 - I0
    w, p = r / Gk, g * c["slope"] / Gk
    z = Cap * p / Gk
    x1 = x0 + h * p - np.expm1(q) * (w - z)
    I1, _ = _nmos_current(x1, K, vov, lam)
    dF = a * (x1 - x0) - (I1 - I0)
    err = abs(-np.expm1(q) * dF / Gk)
    phi2 = (np.expm1(q) - q) / (q * q)
    gamma = 0.1
    x1c = x1 - gamma * h * phi2 * dF / Cap
    # the correction is far above rounding, so its sign and size are visible
    assert abs(x1c - x1) > 1e-8 * abs(x1)

    er = Oracle(net, Options(tol=1.0)).replay(np.array([x0]), [h])
    assert er.x[-1][0] == pytest.approx(x1, rel=1e-12, abs=0)
    assert er.err[-1] == pytest.approx(err, rel=1e-10, abs=0)
    erc = Oracle(net, Options(tol=1.0, erc=True, gamma=gamma)).replay(np.array([x0]), [h])
    assert erc.x[-1][0] == pytest.approx(x1c, rel=1e-12, abs=0)
    # the step is accepted on the estimate of the uncorrected state
    assert erc.err[-1] == pytest.approx(err, rel=1e-10, abs=0)


def test_erc_step_on_three_nodes_matches_dense_phi_functions():
    # The single inverter has a capacitor on each of its three nodes, so C is
    # invertible and J = -C^{-1} G_k can be formed.  phi_1 and phi_2 of hJ come
    # from one dense exponential of the block matrix [[hJ, I, 0], [0, 0, I],
    # [0, 0, 0]], whose first block row holds e^{hJ}, phi_1(hJ), phi_2(hJ).
    import scipy.linalg
    from oracle.mosfet import device_currents
    from oracle.sources import source_values, source_slopes
    net = netgen.single_inverter()
    n = net.n
    o = Oracle(net)
    x0 = o.run(o.dc(), T=30e-12).x[-1]
    t0 = 30e-12
    h, gamma = 2e-12, 0.1
    C = net.C.toarray()
    assert np.linalg.matrix_rank(C) == n
    I0, Jd = device_currents(net, x0)
    Gk = net.G.toarray() + Jd.toarray()
    J = -np.linalg.solve(C, Gk)
    Z = np.zeros((3 * n, 3 * n))
    Z[:n, :n] = h * J
    Z[:n, n:2 * n] = np.eye(n)
    Z[n:2 * n, 2 * n:] = np.eye(n)
    E = scipy.linalg.expm(Z)
    eJ, phi1, phi2 = E[:n, :n], E[:n, n:2 * n], E[:n, 2 * n:]
    u = source_values(net, t0)
    s = source_slopes(net, t0, h)
    r = net.B @ u - net.G @ x0 - I0
    g_k = np.linalg.solve(C, r)
    b_k = np.linalg.solve(C, net.B @ s)
    # the ER step as the paper writes it, before any cancellation of C^{-1}
    x1 = x0 + h * phi1 @ g_k + h * h * phi2 @ b_k
    I1, _ = device_currents(net, x1)
    dF = Jd @ (x1 - x0) - (I1 - I0)
    err = np.max(np.abs(h * phi1 @ np.linalg.solve(C, dF)))
    x1c = x1 - gamma * h * phi2 @ np.linalg.solve(C, dF)
    assert np.max(np.abs(x1c - x1)) > 1e-6
    opts = dict(tol=1.0, eps_krylov=1e-16)
    er = Oracle(net, Options(**opts)).replay(x0, [t0 + h], t0=t0)
    erc = Oracle(net, Options(erc=True, gamma=gamma, **opts)).replay(x0, [t0 + h], t0=t0)
    assert np.max(np.abs(er.x[-1] - x1)) <= 1e-11
    assert er.err[-1] == pytest.approx(err, rel=1e-8)
    assert np.max(np.abs(erc.x[-1] - x1c)) <= 1e-11
