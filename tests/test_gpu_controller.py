"""The learned step controller end to end on an MI355X: trace features from
plain runs, training on the GPU, and what the trained network gains on a
circuit it has not seen.

Gain is time to solution at equal accuracy: the kernel time of the whole
transient with the learned controller against the paper's alpha/beta rule on
the same fresh circuit, both with E_rr = 1e-6 V; accuracy is the final state
against the oracle's adaptive run with a 10x tighter budget (a stored result
of tests/golden/make_golden.py); the local error test judges every step in
both modes."""
import os

import numpy as np
import pytest

import netgen

pytestmark = pytest.mark.gpu


def _training_set():
    base = netgen.inverter_chain(seed=7000, n_stages=80).meta["values"]
    nets = [netgen.inverter_chain(seed=7000, n_stages=80, base=base, variation=dict(seed=7100 + i))
            for i in range(8)]
    nets += [netgen.inverter_chain(seed=7300 + j, n_stages=L) for j, L in enumerate((60, 110, 150, 190))]
    return nets


def _run(E, net, ctrl=None, safety=1.0, **kw):
    s = E.Solver([net], probes=[np.zeros(0, np.int32)], trace_cap=8192, **kw)
    x = s.zeros()
    s.dc(x)
    if ctrl is not None:
        s.load_controller(*ctrl, safety=safety)
    info = s.run(x, max_steps_per_launch=8192)[0]
    sec, _ = s.kernel_time()
    tr = s.trace(0)
    out = x[0].cpu().numpy()
    s.close()
    return info, sec, out, tr


def test_trace_features_are_recorded_and_finite():
    import paper_1511_04515_amd as E
    info, _, _, tr = _run(E, netgen.inverter_chain(seed=9, n_stages=20, T=0.5e-9, t_ramp=0.2e-9))
    f = tr["feat"]
    assert f.shape == (info["steps"], 8) and np.isfinite(f).all()
    # m_{k-1}/60, log10 h_{k-1} (nominal size) and rejections_{k-1} repeat the previous record
    assert np.allclose(f[1:, 1], tr["m"][:-1] / 60.0)
    landed = (tr["rejects"] == 0) & (tr["h"] < tr["h_try"])
    nominal = np.where(landed, tr["h_try"], tr["h"])
    assert np.allclose(f[1:, 2], np.log10(nominal[:-1]))
    assert np.array_equal(f[1:, 7], tr["rejects"][:-1])
    # the log10 of the error budget ratio and of the Krylov residual likewise
    assert np.allclose(f[1:, 6], np.log10(np.maximum(tr["err"][:-1] / 1e-6, 1e-30)))
    assert np.allclose(f[1:, 3], np.log10(np.maximum(tr["rho"][:-1], 1e-30)))


def test_learned_controller_beats_plain_control_on_a_fresh_circuit():
    import paper_1511_04515_amd as E
    from paper_1511_04515_amd import control
    nets = _training_set()
    s = E.Solver(nets, probes=[np.zeros(0, np.int32)] * len(nets), trace_cap=8192)
    x = s.zeros()
    s.dc(x)
    s.run(x, max_steps_per_launch=8192)
    X, T = control.samples_from_traces([s.trace(i) for i in range(len(nets))])
    s.close()
    params, norm, losses = control.train(X, T, epochs=40, batch=4096, lr=1e-3)
    assert losses[-1] < 0.2 * losses[0]
    fresh = netgen.inverter_chain(seed=6000, n_stages=120)
    # the oracle's run at a 10x tighter budget (E_rr = 1e-7 V) to T
    g = np.load(os.path.join(os.path.dirname(__file__), "golden", "fresh120_tight.npz"), allow_pickle=False)
    assert g["t_final"] == fresh.T
    ref = g["x_final"]
    plain, t_plain, x_plain, _ = _run(E, fresh)
    learned, t_learned, x_learned, tr = _run(E, fresh, (params, norm), safety=0.85)
    e_plain = np.abs(x_plain - ref).max()
    e_learned = np.abs(x_learned - ref).max()
    print(f"plain: {t_plain:.2f} s, {plain['steps']} steps, {plain['rejects']} rejections, "
          f"{plain['arnoldi']} Arnoldi, error {e_plain:.1e}; learned: {t_learned:.2f} s, {learned['steps']} steps, "
          f"{learned['rejects']} rejections, {learned['arnoldi']} Arnoldi, error {e_learned:.1e}", flush=True)
    assert learned["status"] == 0 and tr["t"][-1] == fresh.T
    assert learned["rejects"] < 0.5 * plain["rejects"]
    assert t_learned < 0.95 * t_plain
    # equal accuracy: the learned run is no further from the tight oracle
    # reference than the paper's control, up to where each grid falls
    assert e_learned <= max(1.5 * e_plain, 1e-6)
