"""expri_run_noalloc, the transient whose workspace is the library's static
scratch array (for callers that cannot allocate), against expri_run on the
same circuits: identical traces and final states, on two calls in a row, the
second with a smaller input; a context whose workspace exceeds the array is
refused (run on an MI355X)."""
import numpy as np
import pytest

import netgen
from oracle import Oracle

pytestmark = pytest.mark.gpu


def _nets(stages, T):
    return [netgen.inverter_chain(seed=800 + i, n_stages=L, T=T, t_ramp=0.1e-9) for i, L in enumerate(stages)]


def _compare(nets):
    import paper_1511_04515_amd as E
    x0s = [Oracle(n).dc() for n in nets]
    ref = E.Solver(nets)
    xr = ref.to_device(x0s)
    ref.run(xr)
    got = E.Solver(nets)
    assert got.workspace_bytes() <= 64 << 20
    xg = got.to_device(x0s)
    info = got.run_noalloc(xg)
    for i in range(len(nets)):
        assert info[i]["status"] == 0 and info[i]["t"] == nets[i].T
        a, b = got.trace(i), ref.trace(i)
        assert len(a["t"]) > 5 and np.array_equal(a["t"], b["t"]) and np.array_equal(a["x"], b["x"]), i
        assert np.array_equal(xg[i].cpu().numpy(), xr[i].cpu().numpy()), i
    ref.close()
    return got


def test_noalloc_run_equals_run_twice_second_smaller():
    # two launch classes (512 and 256 threads), then one small chain
    first = _compare(_nets((150, 30, 60), 0.3e-9))
    second = _compare(_nets((25,), 0.2e-9))
    # the first context still runs: its scratch contents were overwritten by
    # the second call, and each call initialises what it reads
    nets = _nets((150, 30, 60), 0.3e-9)
    x0s = [Oracle(n).dc() for n in nets]
    xa = first.to_device(x0s)
    first.run_noalloc(xa)
    import paper_1511_04515_amd as E
    ref = E.Solver(nets)
    xr = ref.to_device(x0s)
    ref.run(xr)
    for i in range(len(nets)):
        assert np.array_equal(xa[i].cpu().numpy(), xr[i].cpu().numpy())
    ref.close()
    first.close()
    second.close()


def test_noalloc_refuses_a_workspace_beyond_the_scratch_array():
    import paper_1511_04515_amd as E
    nets = [netgen.config(2)] * 16
    s = E.Solver(nets, probes=[np.zeros(0, np.int32)] * 16)
    assert s.workspace_bytes() > 64 << 20
    with pytest.raises(E.ExpriError) as ei:
        s.run_noalloc(s.zeros())
    assert ei.value.status == -1
    s.close()
