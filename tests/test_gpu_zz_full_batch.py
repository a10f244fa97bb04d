"""The benchmark batch at full size, in the launch configuration the benchmark
times (run on an MI355X).

320 instances, 1.39M nodes: 256 variants of a 200-stage inverter chain
(shared sparsity) and 64 chains of 50-400 stages. They run as three
concurrent launch classes (512 threads with up to 18 rows per thread, 512
threads with up to 9, 256 threads), each a work queue over its instances. The oracle cannot run the whole batch in a test, so the
checks are:
  * invariants of every instance: status OK, t = T, one LU per accepted step,
    a finite state;
  * one sampled instance per class equals its single-instance run bit for bit
    (same kernels, so the batch adds no arithmetic of its own);
  * with the learned step controller (the benchmark's default mode), trained
    on disjoint circuits: every instance ends at T, every accepted step meets
    the error budget E_rr (the paper's estimate still judges each step), the
    sampled instances equal their single runs bitwise, and their final states
    stay within 100 E_rr of the paper's control (the observed gap is printed;
    the learned run's accuracy against the oracle is asserted on a fresh
    circuit in test_gpu_controller.py);
  * for each sampled instance, started from the oracle's own DC point, the
    oracle's adaptive run (Algorithm 2) over its first K accepted steps. The
    two controllers take the same decisions except where an error estimate
    sits on E_rr, so the states are compared at the accepted times both grids
    share, to the relative waveform bar of 1e-6.
"""
import numpy as np
import pytest

import netgen
from oracle import Oracle

pytestmark = pytest.mark.gpu

K_REPLAY = 200


def test_full_batch_in_the_benchmark_launch_configuration():
    import paper_1511_04515_amd as E
    import torch
    nets = netgen.config(4)
    assert len(nets) == 320
    # one instance per class: the smallest of the 18-rows class, instance 0 (a
    # shared-pattern variant) and the largest of the 256-thread class
    by_cls = {}
    for i, net in enumerate(nets):
        key = 256 if net.n <= 2048 else 512 if net.n <= 4608 else 1024
        by_cls.setdefault(key, []).append(i)
    picks = [min(by_cls[1024], key=lambda i: nets[i].n), 0, max(by_cls[256], key=lambda i: nets[i].n)]
    ref_x0 = {i: Oracle(nets[i]).dc() for i in picks}

    s = E.Solver(nets, trace_cap=8192)
    classes, _ = s.classes()
    assert [(c["block_size"], c["max_rows"], c["n_inst"]) for c in classes] == [(512, 18, 36), (512, 9, 275),
                                                                                  (256, 9, 9)]
    xs = s.zeros()
    s.dc(xs)
    for i in picks:
        xs[i].copy_(torch.from_numpy(ref_x0[i]))
    x0 = [x.clone() for x in xs]
    info = s.run(xs, max_steps_per_launch=8192)
    for i, (net, r) in enumerate(zip(nets, info)):
        assert r["status"] == 0 and r["t"] == net.T, i
        assert r["lu_count"] == r["steps"] > 0, i
        # work counters within what the trials allow (two MEVPs of at most
        # m_max = 60 Arnoldi steps per trial)
        assert 0 < r["arnoldi"] <= 120 * r["trials"], (i, r)
        assert r["arnoldi"] <= r["mgs_terms"] <= 60 * r["arnoldi"], (i, r)
        assert np.all(np.isfinite(xs[i].cpu().numpy())), i

    for i in picks:
        net = nets[i]
        s1 = E.Solver(net, trace_cap=8192)
        x1 = [x0[i].clone()]
        s1.run(x1, max_steps_per_launch=8192)
        a, b = s.trace(i), s1.trace(0)
        assert np.array_equal(a["t"], b["t"]) and np.array_equal(a["x"], b["x"]), i
        assert np.array_equal(xs[i].cpu().numpy(), x1[0].cpu().numpy()), i
        s1.close()

        ref = Oracle(net).run(ref_x0[i], keep=net.probes, max_steps=K_REPLAY)
        rt = np.array(ref.t)
        common = np.intersect1d(a["t"], rt)
        ia = np.searchsorted(a["t"], common)
        ib = np.searchsorted(rt, common)
        err = np.max(np.abs(a["x"][ia] - np.array(ref.x)[ib])) if common.size else np.inf
        print(f"instance {i} (n = {net.n}): {len(a['t'])} steps; {common.size} of the oracle's first "
              f"{rt.size} accepted times shared, max |dx| there {err:.2e} V", flush=True)
        assert common.size >= min(10, rt.size), i
        # the relative waveform bar at every shared accepted time
        rel = err / max(np.max(np.abs(np.array(ref.x)[ib])), 1.0)
        assert rel <= 1e-6, (i, err)

    # the learned step controller on the same batch, from the same states
    from paper_1511_04515_amd import control
    tnets = _training_set()
    st = E.Solver(tnets, probes=[np.zeros(0, np.int32)] * len(tnets), trace_cap=8192)
    xt = st.zeros()
    st.dc(xt)
    st.run(xt, max_steps_per_launch=8192)
    X, T = control.samples_from_traces([st.trace(i) for i in range(len(tnets))])
    st.close()
    params, norm, _ = control.train(X, T, epochs=40, batch=4096, lr=1e-3)
    s.load_controller(params, norm, safety=0.85)
    xl = [x.clone() for x in x0]
    info_l = s.run(xl, max_steps_per_launch=8192)
    E_rr = s.opts.E_rr
    for i, (net, r) in enumerate(zip(nets, info_l)):
        assert r["status"] == 0 and r["t"] == net.T, i
        tr = s.trace(i)
        assert tr["t"][-1] == net.T and np.all(tr["err"] <= E_rr), i
    print(f"learned: {sum(r['steps'] for r in info_l)} accepted steps, "
          f"{sum(r['rejects'] for r in info_l)} rejections (paper's control: "
          f"{sum(r['steps'] for r in info)}, {sum(r['rejects'] for r in info)})", flush=True)
    for i in picks:
        s1 = E.Solver(nets[i], trace_cap=8192)
        s1.load_controller(params, norm, safety=0.85)
        x1 = [x0[i].clone()]
        s1.run(x1, max_steps_per_launch=8192)
        a, b = s.trace(i), s1.trace(0)
        assert np.array_equal(a["t"], b["t"]) and np.array_equal(a["x"], b["x"]), i
        assert np.array_equal(xl[i].cpu().numpy(), x1[0].cpu().numpy()), i
        s1.close()
        gap = np.max(np.abs(xl[i].cpu().numpy() - xs[i].cpu().numpy()))
        print(f"instance {i}: final state, learned vs paper's control: max |dx| {gap:.2e} V", flush=True)
        # the two controllers take different grids, so their states at T
        # differ by the difference of their accumulated local errors (each
        # step within E_rr); the accuracy of the learned run against the
        # oracle is asserted on a fresh circuit in test_gpu_controller.py
        assert gap <= 100 * E_rr, (i, gap)
    s.close()


def _training_set():
    # circuits disjoint from the batch (seeds 7000+)
    base = netgen.inverter_chain(seed=7000, n_stages=80).meta["values"]
    nets = [netgen.inverter_chain(seed=7000, n_stages=80, base=base, variation=dict(seed=7100 + i))
            for i in range(8)]
    nets += [netgen.inverter_chain(seed=7300 + j, n_stages=L) for j, L in enumerate((60, 110, 150, 190))]
    return nets
