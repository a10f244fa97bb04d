"""GPU parity of libexpri against the oracle (run on an MI355X).

Every call goes through the C-ABI (ctypes binding).  Tolerances:
  * LU of G_k: ||L U - P G_k P^T|| <= 1e-12 ||G_k||; solves: normwise
    backward error <= 1e-12 (the linear-solve bar is 1e-10);
  * MEVP and one-step results: 1e-10 relative to the vector norm (same
    arithmetic in a different summation order);
  * transient waveforms: max_k ||x_gpu(t_k) - x_ref(t_k)||_inf /
    max(max_k ||x_ref||_inf, 1 V) <= 1e-6 on the replayed grid (both sides take
    the same steps; the observed error is far smaller).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import netgen
from oracle import Oracle, Options, InvertKrylov, device_currents
from tests.exact import ladder_step, linear_exact

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def Solver(nets, **kw):
    import paper_1511_04515_amd as E
    return E.Solver(nets, **kw)


def rel_wave_err(x, ref):
    return np.max(np.abs(np.asarray(x) - np.asarray(ref))) / max(np.max(np.abs(ref)), 1.0)


def lu_residual(s, inst, net, x):
    pat = s.lu_pattern(inst)
    lu = s.lu_values(inst)
    n = net.n
    F = sp.csr_matrix((lu, pat["col"], pat["rowptr"]), shape=(n, n)).toarray()
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    _, Jd = device_currents(net, x)
    perm = pat["perm"]
    Gk = (net.G + Jd).toarray()[np.ix_(perm, perm)]
    return np.linalg.norm(L @ U - Gk) / np.linalg.norm(Gk), Gk, perm


def test_factor_and_solve_match_oracle():
    net = netgen.inverter_chain(seed=3, n_stages=20)
    o = Oracle(net)
    x0 = o.dc()
    x = x0 + np.random.default_rng(1).normal(0, 0.05, net.n)
    s = Solver(net)
    xs = s.to_device([x])
    s.factor(xs)
    r, Gk, perm = lu_residual(s, 0, net, x)
    assert r <= 1e-12
    b = np.random.default_rng(2).standard_normal(net.n)
    ys = s.zeros()
    s.solve(s.to_device([b]), ys)
    y = ys[0].cpu().numpy()
    _, Jd = device_currents(net, x)
    G = (net.G + Jd).tocsr()
    berr = np.abs(G @ y - b).max() / (abs(G).sum(1).max() * np.abs(y).max() + np.abs(b).max())
    assert berr <= 1e-12
    s.close()


@pytest.mark.parametrize("h", [2e-14, 1e-12, 5e-11])
def test_mevp_matches_oracle(h):
    net = netgen.inverter_chain(seed=4, n_stages=20)
    o = Oracle(net)
    x0 = o.dc()
    _, Jd = device_currents(net, x0)
    lu = spla.splu((net.G + Jd).tocsc())
    A = lambda q: -lu.solve(net.C @ q)
    v = A(np.random.default_rng(5).standard_normal(net.n))
    eps = 1e-7 * np.linalg.norm(v)
    k = InvertKrylov(A, v, 60)
    d, rho = k.converge(h, eps)
    ref = k.combine(d)
    s = Solver(net)
    s.factor(s.to_device([x0]))
    outs = s.zeros()
    m, rho_g = s.mevp(s.to_device([v]), outs, h, eps)
    got = outs[0].cpu().numpy()
    assert m[0] == k.m
    assert rho_g[0] == pytest.approx(rho, rel=1e-6, abs=1e-30)
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.linalg.norm(v)
    s.close()


@pytest.mark.parametrize("cfg", [1, 2])
def test_dc_matches_oracle(cfg):
    net = netgen.config(cfg)
    ref = Oracle(net).dc()
    s = Solver(net)
    xs = s.zeros()
    info = s.dc(xs)
    assert info[0]["status"] == 0
    assert np.max(np.abs(xs[0].cpu().numpy() - ref)) <= 1e-10
    s.close()


def _golden(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    if not os.path.exists(path):
        pytest.fail(f"missing {path}: run tests/golden/make_golden.py")
    return np.load(path, allow_pickle=False)


@pytest.mark.parametrize("name,cfg,kw", [("mesh", 1, {}), ("chain", 2, {}), ("chain12", None, {}),
                                         ("chain12_erc", None, dict(erc=1, gamma=0.1))])
def test_replay_parity_full_run(name, cfg, kw):
    g = _golden(name)
    net = netgen.config(cfg) if cfg else netgen.inverter_chain(seed=77, n_stages=12, T=1.5e-9,
                                                               t_ramp=0.2e-9)
    s = Solver(net, trace_cap=4096, **kw)
    xs = s.to_device([g["x0"]])
    info = s.run_schedule(xs, [g["t"]])
    assert info[0]["status"] == 0 and info[0]["steps"] == len(g["t"])
    tr = s.trace(0)
    assert np.array_equal(tr["t"], g["t"])
    err = rel_wave_err(tr["x"], g["replay_probe_x"])
    assert err <= 1e-6
    # the final full state as well
    assert rel_wave_err(xs[0].cpu().numpy(), g["x_final"]) <= 1e-6
    # Krylov sizes agree except where the residual sits on the threshold
    match = np.mean(tr["m"] == g["replay_m"])
    big = g["replay_err"] > 1e-3 * net.tol
    err_rel = np.max(np.abs(tr["err"][big] / g["replay_err"][big] - 1)) if big.any() else 0.0
    print(f"{name}: {len(g['t'])} steps, waveform rel err {err:.2e}, m match {match:.3f}, "
          f"m diff hist {np.bincount(np.abs(tr['m'] - g['replay_m']).astype(int))}, "
          f"e_rr max rel diff {err_rel:.2e}", flush=True)
    # m itself is rounding-sensitive: the residual hovers near eps_K for a few
    # iterations, and a 1e-15 relative perturbation of the oracle's own input
    # changes m on ~20% of the chain's steps; so only its mean is bounded
    assert np.mean(np.abs(tr["m"] - g["replay_m"])) <= 1.0
    assert err_rel <= 1e-3
    s.close()


def test_adaptive_run_follows_oracle_grid():
    g = _golden("chain12")
    net = netgen.inverter_chain(seed=77, n_stages=12, T=1.5e-9, t_ramp=0.2e-9)
    s = Solver(net)
    xs = s.to_device([g["x0"]])
    info = s.run(xs)
    tr = s.trace(0)
    assert info[0]["status"] == 0 and tr["t"][-1] == net.T
    # same controller, same decisions except where err sits on E_rr
    n_ref = len(g["t"])
    assert abs(len(tr["t"]) - n_ref) <= max(3, n_ref // 50)
    common = np.intersect1d(tr["t"], g["t"])
    assert common.size > 0.9 * n_ref
    ia = np.searchsorted(tr["t"], common)
    ib = np.searchsorted(g["t"], common)
    assert rel_wave_err(tr["x"][ia], g["run_probe_x"][ib]) <= 1e-5
    # one LU per accepted step, none on a rejection
    assert info[0]["lu_count"] == info[0]["steps"] and info[0]["rejects"] > 0
    s.close()


def test_closed_forms_on_gpu():
    R, Cap = 1e3, 1e-12
    for wave in ("step", "ramp"):
        net = netgen.rc_single(R=R, Cap=Cap, wave=wave)
        s = Solver(net)
        xs = s.zeros()
        s.run(xs)
        tr = s.trace(0)
        t = tr["t"]
        ex = 1 - np.exp(-t / (R * Cap)) if wave == "step" else (t - R * Cap * (1 - np.exp(-t / (R * Cap)))) / net.T
        assert np.max(np.abs(tr["x"][:, 0] - ex)) < 1e-13
        s.close()
    N, Rl, c = 16, 100.0, 10e-15
    net = netgen.rc_ladder(N=N, R=Rl, c=c)
    s = Solver(net, E_rr=1e-12)
    xs = s.zeros()
    s.run(xs)
    tr = s.trace(0)
    assert np.max(np.abs(tr["x"] - ladder_step(N, Rl, c, 1.0, tr["t"]))) < 1e-12
    s.close()


@pytest.mark.parametrize("seed", range(4))
def test_singular_C_tiny_circuits_on_gpu(seed):
    net = netgen.tiny_linear(seed)
    x0 = Oracle(net).dc()
    s = Solver(net, E_rr=1e-12)
    xs = s.to_device([x0])
    s.run(xs)
    tr = s.trace(0)
    ex = linear_exact(net, x0, tr["t"])
    assert np.max(np.abs(tr["x"] - ex[:, net.probes])) < 1e-12
    s.close()


def test_batch_matches_single_instance_runs():
    base = netgen.inverter_chain(seed=1004, n_stages=30, T=0.8e-9, t_ramp=0.3e-9)
    vals = base.meta["values"]
    nets = [netgen.inverter_chain(seed=1004, n_stages=30, T=0.8e-9, t_ramp=0.3e-9, base=vals,
                                  variation=dict(seed=3000 + i)) for i in range(3)]
    nets.append(netgen.inverter_chain(seed=9, n_stages=17, T=0.8e-9, t_ramp=0.3e-9))
    x0s = [Oracle(n).dc() for n in nets]
    sb = Solver(nets, block_size=512)
    xb = sb.to_device(x0s)
    sb.run(xb)
    for i, net in enumerate(nets):
        s1 = Solver(net, block_size=512)
        x1 = s1.to_device([x0s[i]])
        s1.run(x1)
        a, b = sb.trace(i), s1.trace(0)
        assert np.array_equal(a["t"], b["t"]) and np.array_equal(a["x"], b["x"])
        assert np.array_equal(xb[i].cpu().numpy(), x1[0].cpu().numpy())
        s1.close()
    sb.close()


def test_set_values_matches_a_fresh_setup():
    """expri_set_values on instances of a shared-pattern batch gives, bit for
    bit, the factors, solves and transients of a fresh setup with those
    values; a circuit of another pattern is refused with EPATTERN and solve
    waits for a new factor."""
    import paper_1511_04515_amd as E
    import torch
    kw = dict(seed=1004, n_stages=30, T=0.8e-9, t_ramp=0.3e-9)
    vals = netgen.inverter_chain(**kw).meta["values"]
    var = [netgen.inverter_chain(**kw, base=vals, variation=dict(seed=3000 + i)) for i in range(4)]
    want = [var[0], var[3], var[0]]
    x0s = [Oracle(n).dc() for n in want]
    s = Solver(var[:3], block_size=512)
    s.set_values(1, var[3])
    s.set_values(2, var[0])
    ref = Solver(want, block_size=512)

    xs, xr = s.to_device(x0s), ref.to_device(x0s)
    rng = np.random.default_rng(11)
    bs = s.to_device([rng.standard_normal(n.n) for n in want])
    ys = [torch.empty_like(b) for b in bs]
    yr = [torch.empty_like(b) for b in bs]
    with pytest.raises(E.ExpriError) as ei:
        s.solve(bs, ys)
    assert ei.value.status == -1
    s.factor(xs)
    ref.factor(xr)
    s.solve(bs, ys)
    ref.solve(bs, yr)
    for i in range(3):
        assert np.array_equal(s.lu_values(i), ref.lu_values(i))
        assert np.array_equal(ys[i].cpu().numpy(), yr[i].cpu().numpy())

    s.run(xs)
    ref.run(xr)
    for i in range(3):
        a, b = s.trace(i), ref.trace(i)
        assert np.array_equal(a["t"], b["t"]) and np.array_equal(a["x"], b["x"])
        assert np.array_equal(xs[i].cpu().numpy(), xr[i].cpu().numpy())

    other = netgen.inverter_chain(seed=9, n_stages=17, T=0.8e-9, t_ramp=0.3e-9)
    with pytest.raises(E.ExpriError) as ei:
        s.set_values(0, other)
    assert ei.value.status == -8
    s.close()
    ref.close()


def test_mixed_size_batch_runs_as_concurrent_classes_and_matches_single_runs():
    # chains of 841, 2521 and 6301 nodes take 256 threads, 512 threads with
    # up to 9 rows per thread and 512 threads with up to 18: three launch
    # classes, the transient kernels concurrent on three streams
    nets = [netgen.inverter_chain(seed=40 + i, n_stages=L, T=0.3e-9, t_ramp=0.1e-9)
            for i, L in enumerate((300, 40, 120, 40, 300))]
    sb = Solver(nets)
    classes, ic = sb.classes()
    assert [(c["block_size"], c["max_rows"]) for c in classes] == [(512, 18), (512, 9), (256, 9)]
    assert [c["n_inst"] for c in classes] == [2, 1, 2]
    assert ic.tolist() == [0, 2, 1, 2, 0]
    xb = sb.zeros()
    sb.dc(xb)
    x_dc = [x.clone() for x in xb]
    sb.factor(xb)
    rng = np.random.default_rng(3)
    rhs = sb.to_device([rng.standard_normal(n.n) for n in nets])
    yb = sb.zeros()
    sb.solve(rhs, yb)
    sb.run(xb)
    assert all(c["kernel_s"] > 0 for c in sb.classes()[0])
    for i, net in enumerate(nets):
        s1 = Solver(net)
        c1 = s1.classes()[0][0]
        assert (c1["block_size"], c1["max_rows"]) == (classes[ic[i]]["block_size"], classes[ic[i]]["max_rows"])
        x1 = s1.zeros()
        s1.dc(x1)
        assert np.array_equal(x1[0].cpu().numpy(), x_dc[i].cpu().numpy())
        s1.factor(x1)
        y1 = s1.zeros()
        s1.solve([rhs[i]], y1)
        assert np.array_equal(y1[0].cpu().numpy(), yb[i].cpu().numpy())
        s1.run(x1)
        a, b = sb.trace(i), s1.trace(0)
        assert len(a["t"]) > 5 and np.array_equal(a["t"], b["t"]) and np.array_equal(a["x"], b["x"])
        assert np.array_equal(xb[i].cpu().numpy(), x1[0].cpu().numpy())
        s1.close()
    sb.close()


def test_capped_workgroups_take_instances_in_turn():
    # four workgroups for nine instances in two launch classes: each
    # workgroup runs several instances one after another
    nets = [netgen.inverter_chain(seed=60 + i, n_stages=L, T=0.2e-9, t_ramp=0.1e-9)
            for i, L in enumerate((120, 8, 12, 120, 10, 9, 14, 11, 120))]
    sb = Solver(nets, max_workgroups=4)
    classes, ic = sb.classes()
    assert [c["block_size"] for c in classes] == [512, 256]
    assert [c["n_inst"] for c in classes] == [3, 6]
    assert [c["workgroups"] for c in classes] == [3, 1]
    xb = sb.zeros()
    sb.dc(xb)
    x0 = [x.clone() for x in xb]
    sb.run(xb, max_steps_per_launch=16)  # several launches: instances resume
    for i, net in enumerate(nets):
        s1 = Solver(net)
        x1 = [x0[i].clone()]
        s1.run(x1)
        a, b = sb.trace(i), s1.trace(0)
        assert len(a["t"]) > 0 and np.array_equal(a["t"], b["t"]) and np.array_equal(a["x"], b["x"])
        assert np.array_equal(xb[i].cpu().numpy(), x1[0].cpu().numpy())
        s1.close()
    assert max(len(sb.trace(i)["t"]) for i in range(len(nets))) > 16
    sb.close()


def test_error_paths_keep_last_state():
    import paper_1511_04515_amd as E
    # step below h_min: the chain is active from t = 0 and no trial meets an
    # error budget of 1e-30 V; h_min = 1e-15 s stops it after a few halvings
    net = netgen.inverter_chain(seed=5, n_stages=3, n_seg=2, T=0.2e-9, t_ramp=0.05e-9)
    x0 = Oracle(net).dc()
    s = Solver(net, E_rr=1e-30, eps_krylov=1e-9, h_min=1e-15)
    xs = s.to_device([x0])
    with pytest.raises(E.ExpriError) as ei:
        s.run(xs)
    assert ei.value.status == -5
    assert s.run_info(0)["steps"] == 0
    assert np.array_equal(xs[0].cpu().numpy(), x0)
    s.close()
    # Krylov basis capped below what the residual needs
    net = netgen.config(1)
    s = Solver(net, m_max=2)
    xs = s.to_device([Oracle(net).dc()])
    with pytest.raises(E.ExpriError) as ei:
        s.run(xs)
    assert ei.value.status == -4
    s.close()
    # a node with no conductance: G_k is singular
    b = netgen.Builder()
    a, f = b.node(), b.node()
    b.resistor(a, -1, 100.0)
    b.capacitor(a, -1, 1e-15)
    b.capacitor(f, -1, 1e-15)
    b.voltage_source(a, 10.0, netgen.PWL([0.0, 1e-12], [0.0, 1.0]))
    bad = b.build("floating", T=1e-11)
    s = Solver(bad)
    xs = s.zeros()
    with pytest.raises(E.ExpriError) as ei:
        s.run(xs)
    assert ei.value.status == -3
    s.close()
