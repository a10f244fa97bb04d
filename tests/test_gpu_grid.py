"""The multifrontal engine (one circuit too large for one workgroup) against
the oracle, run on an MI355X through the C-ABI.

Bars as for the one-workgroup engine: normwise backward error of the solves
<= 1e-12 (the linear-solve bar is 1e-10); MEVP results within the sum of the
two residual bounds (each side's product is within its rho <= eps of the
exact one); relative waveform error <= 1e-6 at every accepted time of a
replayed grid; DC within 1e-10 V."""
import os

import numpy as np
import pytest

import netgen
from oracle import Oracle, InvertKrylov, device_currents

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.fail(f"missing {path}: run tests/golden/make_golden.py {name}")
    return np.load(path, allow_pickle=False)


def rel_wave_err(x, ref):
    return np.max(np.abs(np.asarray(x) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1.0)


def grid96():
    return netgen.power_grid(side=96, n_drivers=60)


def chain12():
    return netgen.inverter_chain(seed=77, n_stages=12, T=1.5e-9, t_ramp=0.2e-9)


def backward_error(net, x, b, y):
    _, Jd = device_currents(net, x)
    G = (net.G + Jd).tocsr()
    return np.abs(G @ y - b).max() / (abs(G).sum(1).max() * np.abs(y).max() + np.abs(b).max())


def test_grid_engine_is_picked_and_factor_solve_meet_the_bar():
    import paper_1511_04515_amd as E
    net = grid96()
    g = _golden("grid96")
    s = E.Solver(net)  # n = 18,552 > 9,216: the multifrontal engine
    assert s.classes()[0][0]["workgroups"] == 0
    x = g["x0"] + np.random.default_rng(1).normal(0, 0.05, net.n)
    s.factor(s.to_device([x]))
    b = np.random.default_rng(2).standard_normal(net.n)
    ys = s.zeros()
    s.solve(s.to_device([b]), ys)
    berr = backward_error(net, x, b, ys[0].cpu().numpy())
    print(f"grid96 solve backward error {berr:.2e}", flush=True)
    assert berr <= 1e-12
    s.close()


def test_grid_engine_solve_with_a_root_front_over_288_pivots():
    # a 2 x 160 x 160 grid: its root front has 319 pivots, so the top height's
    # pivot-block solves take 512-thread workgroups and the others 256; the
    # solve meets the backward-error bar near the DC point (at random node
    # voltages some driver outputs have no conducting device, G_k is nearly
    # singular and the normwise bar says little)
    import paper_1511_04515_amd as E
    from paper_1511_04515_amd import binding as B
    net = netgen.power_grid(side=160, n_drivers=100)
    a = B.frontal_analysis(net)
    root = a["height"] == a["height"].max()
    assert a["nc"][root].max() > 288 and (a["nc"][~root] <= 288).all()
    s = E.Solver(net)
    assert s.classes()[0][0]["workgroups"] == 0
    x0 = s.zeros()
    s.dc(x0)
    x = x0[0].cpu().numpy() + np.random.default_rng(11).normal(0, 0.05, net.n)
    s.factor(s.to_device([x]))
    b = np.random.default_rng(12).standard_normal(net.n)
    ys = s.zeros()
    s.solve(s.to_device([b]), ys)
    y = ys[0].cpu().numpy()
    berr = backward_error(net, x, b, y)
    print(f"grid160 solve backward error {berr:.2e}, max |y| {np.abs(y).max():.2e}", flush=True)
    # |y| stays near 1e4 here; a nearly singular G_k would give |y| near 1e12
    assert np.abs(y).max() < 1e6 and berr <= 1e-12
    s.close()


def test_grid_engine_dc_matches_oracle():
    import paper_1511_04515_amd as E
    net = grid96()
    g = _golden("grid96")
    s = E.Solver(net)
    xs = s.zeros()
    info = s.dc(xs)
    assert info[0]["status"] == 0
    d = np.max(np.abs(xs[0].cpu().numpy() - g["x0"]))
    print(f"grid96 DC: {info[0]['steps']} Newton steps, max |dx| vs oracle {d:.2e} V", flush=True)
    assert d <= 1e-10
    s.close()


@pytest.mark.parametrize("h", [3e-12, 2e-11, 1e-9])
def test_grid_engine_mevp_matches_oracle(h):
    import paper_1511_04515_amd as E
    import scipy.sparse.linalg as spla
    net = grid96()
    g = _golden("grid96")
    x0 = g["x0"]
    _, Jd = device_currents(net, x0)
    lu = spla.splu((net.G + Jd).tocsc())
    A = lambda q: -lu.solve(net.C @ q)
    v = A(np.random.default_rng(5).standard_normal(net.n))
    eps = 1e-7 * np.linalg.norm(v)
    k = InvertKrylov(A, v, 60)
    d, rho = k.converge(h, eps)
    ref = k.combine(d)
    s = E.Solver(net)
    s.factor(s.to_device([x0]))
    outs = s.zeros()
    m, rho_g = s.mevp(s.to_device([v]), outs, h, eps)
    got = outs[0].cpu().numpy()
    diff = np.max(np.abs(got - ref))
    print(f"h {h:g}: m {m[0]} (oracle {k.m}), rho {rho_g[0]:.3e} ({rho:.3e}), max diff {diff:.2e}", flush=True)
    assert abs(m[0] - k.m) <= 1 and rho_g[0] <= eps
    assert diff <= 2 * eps
    s.close()


def test_grid_engine_replay_matches_oracle_on_grid96():
    import paper_1511_04515_amd as E
    net = grid96()
    g = _golden("grid96")
    s = E.Solver(net, trace_cap=4096)
    xs = s.to_device([g["x0"]])
    info = s.run_schedule(xs, [g["t"]])
    assert info[0]["status"] == 0 and info[0]["steps"] == len(g["t"])
    tr = s.trace(0)
    assert np.array_equal(tr["t"], g["t"])
    err = rel_wave_err(tr["x"], g["replay_probe_x"])
    fin = rel_wave_err(xs[0].cpu().numpy(), g["x_final"])
    print(f"grid96 replay: {len(g['t'])} steps, waveform rel err {err:.2e}, final {fin:.2e}, "
          f"m {tr['m'].tolist()} vs {g['replay_m'].tolist()}", flush=True)
    assert err <= 1e-6 and fin <= 1e-6
    s.close()


def test_grid_engine_forced_on_a_chain_matches_oracle_replay_and_run():
    # the nonlinear chain (device-heavy fronts) through the multifrontal engine
    import paper_1511_04515_amd as E
    g = _golden("chain12")
    net = chain12()
    s = E.Solver(net, trace_cap=4096, engine=2)
    xs = s.to_device([g["x0"]])
    info = s.run_schedule(xs, [g["t"]])
    assert info[0]["status"] == 0
    tr = s.trace(0)
    err = rel_wave_err(tr["x"], g["replay_probe_x"])
    print(f"chain12 through the multifrontal engine: replay rel err {err:.2e}", flush=True)
    assert err <= 1e-6 and rel_wave_err(xs[0].cpu().numpy(), g["x_final"]) <= 1e-6
    # the adaptive run takes the oracle's decisions except where e_rr sits on E_rr
    xs = s.to_device([g["x0"]])
    info = s.run(xs)
    tr = s.trace(0)
    assert info[0]["status"] == 0 and tr["t"][-1] == net.T
    n_ref = len(g["t"])
    common = np.intersect1d(tr["t"], g["t"])
    print(f"adaptive: {len(tr['t'])} steps (oracle {n_ref}), {common.size} shared", flush=True)
    assert abs(len(tr["t"]) - n_ref) <= max(3, n_ref // 50) and common.size > 0.9 * n_ref
    ia = np.searchsorted(tr["t"], common)
    ib = np.searchsorted(g["t"], common)
    assert rel_wave_err(tr["x"][ia], g["run_probe_x"][ib]) <= 1e-5
    assert info[0]["lu_count"] == info[0]["steps"]
    # expri_step repeated with its own h_next is the adaptive run
    xs = s.to_device([g["x0"]])
    t, h, k = 0.0, s.opts.h_init, 0
    while t < net.T and k < 40:
        st = s.step(xs, t, h)[0]
        assert st["t"] == tr["t"][k] and st["h_used"] == tr["h"][k], k
        t, h, k = st["t"], st["h_next"], k + 1
    s.close()


def test_full_power_grid_factor_solve_and_replay():
    # config 3 at its full size (528,288 unknowns), in the configuration the
    # benchmark runs: the oracle's first 20 accepted steps from its DC point,
    # replayed; the solve's backward error on the full system
    import paper_1511_04515_amd as E
    import time
    g = _golden("grid512")
    net = netgen.config(3)
    s = E.Solver(net, trace_cap=4096)
    x0 = g["x0"]
    xs = s.to_device([x0])
    s.factor(xs)
    b = np.random.default_rng(7).standard_normal(net.n)
    ys = s.zeros()
    s.solve(s.to_device([b]), ys)
    berr = backward_error(net, x0, b, ys[0].cpu().numpy())
    t0 = time.perf_counter()
    info = s.run_schedule(xs, [g["t"]])
    el = time.perf_counter() - t0
    tr = s.trace(0)
    err = rel_wave_err(tr["x"], g["replay_probe_x"])
    fin = rel_wave_err(xs[0].cpu().numpy(), g["x_final"])
    print(f"config 3: backward error {berr:.2e}; replay of {len(g['t'])} steps in {el:.2f} s, waveform rel err "
          f"{err:.2e}, final state {fin:.2e}, m {tr['m'].tolist()} vs {g['replay_m'].tolist()}", flush=True)
    assert info[0]["status"] == 0 and np.array_equal(tr["t"], g["t"])
    assert berr <= 1e-12 and err <= 1e-6 and fin <= 1e-6
    s.close()


def test_learned_controller_in_the_multifrontal_engine_on_grid96():
    # the learned controller (trained on chain traces, as the benchmark's) in
    # the multifrontal engine over the first 0.3 ns of the 2 x 96 x 96 grid
    # (about 60 steps of the paper's control reach 0.14 ns, after which its
    # steps settle near 0.3 ps): the run reaches T, every accepted step meets
    # E_rr (the error test still judges every trial), the trace holds finite
    # features, and the final state stays within 100 E_rr of the paper's
    # control
    import paper_1511_04515_amd as E
    from paper_1511_04515_amd import control
    base = netgen.inverter_chain(seed=7000, n_stages=80).meta["values"]
    nets = [netgen.inverter_chain(seed=7000, n_stages=80, base=base, variation=dict(seed=7100 + i))
            for i in range(8)]
    nets += [netgen.inverter_chain(seed=7300 + j, n_stages=L) for j, L in enumerate((60, 110, 150, 190))]
    s = E.Solver(nets, probes=[np.zeros(0, np.int32)] * len(nets), trace_cap=8192)
    x = s.zeros()
    s.dc(x)
    s.run(x, max_steps_per_launch=8192)
    X, T = control.samples_from_traces([s.trace(i) for i in range(len(nets))])
    s.close()
    params, norm, _ = control.train(X, T, epochs=40, batch=4096, lr=1e-3)
    print(f"controller trained on {len(X)} samples", flush=True)

    net = netgen.power_grid(side=96, n_drivers=60, T=0.3e-9)

    def run(ctrl):
        g = E.Solver(net)
        assert g.classes()[0][0]["workgroups"] == 0  # the multifrontal engine
        xg = g.zeros()
        g.dc(xg)
        if ctrl is not None:
            g.load_controller(*ctrl)
        info = g.run(xg)[0]
        tr = g.trace(0)
        sec, _ = g.kernel_time()
        out = xg[0].cpu().numpy()
        g.close()
        print(f"  {'learned' if ctrl is not None else 'paper'}: {sec:.2f} s, {info['steps']} steps", flush=True)
        return info, tr, out, sec

    pi, ptr, px, psec = run(None)
    li, ltr, lx, lsec = run((params, norm))
    gap = np.max(np.abs(lx - px))
    print(f"grid96 to 0.3 ns: paper's control {psec:.2f} s, {pi['steps']} steps, {pi['rejects']} rejections, "
          f"{pi['arnoldi']} Arnoldi; learned {lsec:.2f} s, {li['steps']} steps, {li['rejects']} rejections, "
          f"{li['arnoldi']} Arnoldi; final state gap {gap:.2e} V", flush=True)
    assert pi["status"] == 0 and li["status"] == 0
    assert ptr["t"][-1] == net.T and ltr["t"][-1] == net.T
    assert np.all(ltr["err"] <= 1e-6) and np.all(ptr["err"] <= 1e-6)
    assert np.isfinite(ltr["feat"]).all() and np.isfinite(ptr["feat"]).all()
    assert gap <= 100 * 1e-6


def test_automatic_engine_choice_falls_back_to_the_multifrontal_engine():
    # a 2 x 64 x 64 grid (8,252 unknowns) is under the one-workgroup engine's
    # size bound, but rows of its L and U are longer than that engine's solve
    # passes hold: the automatic choice sets it up on the multifrontal engine
    import paper_1511_04515_amd as E
    net = netgen.power_grid(seed=9003, side=64, T=0.05e-9, stim_seed=9004, n_drivers=30)
    assert net.n <= 9216
    s = E.Solver(net)
    assert s.classes()[0][0]["workgroups"] == 0
    x = s.zeros()
    s.dc(x)
    info = s.run(x)[0]
    assert info["status"] == 0 and s.trace(0)["t"][-1] == net.T
    s.close()
    with pytest.raises(E.ExpriError):
        E.Solver(net, engine=1)
