"""The autotuner (expri_opts.autotune, run on an MI355X): each distinct
pattern's launch configuration (block size, rows-per-thread bound, solve
slots per lane) is measured once per process and cached by pattern hash, and
a tuned batch computes exactly what a context with that configuration given
explicitly computes (the same kernels on the same schedule; the variants'
agreement with the oracle is tested in test_gpu_variants.py)."""
import numpy as np
import pytest

import netgen

pytestmark = pytest.mark.gpu


def test_autotune_measures_each_pattern_once_and_matches_the_explicit_configuration():
    import paper_1511_04515_amd as E
    nets = [netgen.inverter_chain(seed=70 + i, n_stages=L, T=0.2e-9, t_ramp=0.1e-9)
            for i, L in enumerate((30, 120, 250))]
    nets.append(netgen.inverter_chain(seed=70, n_stages=30, T=0.2e-9, t_ramp=0.1e-9))  # shares pattern 0
    r0 = E.autotune_runs()
    s = E.Solver(nets, autotune=1)
    r1 = E.autotune_runs()
    assert r1 > r0
    cfg = [s.config(k) for k in range(len(nets))]
    print("tuned:", [(net.n, c) for net, c in zip(nets, cfg)], flush=True)
    assert cfg[3] == cfg[0]
    for c, net in zip(cfg, nets):
        assert c["block_size"] in (256, 512, 1024) and net.n <= c["max_rows"] * c["block_size"]
        assert c["slots_l"] in (1, 2, 4, 8) and c["slots_u"] in (1, 2, 4, 8)

    # the same patterns again: taken from the cache, no trial runs
    s2 = E.Solver(nets[:3], autotune=1)
    assert E.autotune_runs() == r1
    assert [s2.config(k) for k in range(3)] == cfg[:3]
    s2.close()

    xs = s.zeros()
    s.dc(xs)
    x0 = [x.clone() for x in xs]
    info = s.run(xs)
    assert all(i["status"] == 0 for i in info)
    for k, net in enumerate(nets[:3]):
        c = cfg[k]
        single = None
        for slots in (0, 1, 2, 4, 8):
            t = E.Solver(net, block_size=c["block_size"], solve_slots=slots)
            if t.config(0) == c:
                single = t
                break
            t.close()
        assert single is not None, c
        x1 = [x0[k].clone()]
        single.run(x1)
        a, b = s.trace(k), single.trace(0)
        assert len(a["t"]) > 5 and np.array_equal(a["t"], b["t"]) and np.array_equal(a["x"], b["x"])
        assert np.array_equal(xs[k].cpu().numpy(), x1[0].cpu().numpy())
        single.close()
    s.close()
