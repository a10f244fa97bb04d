"""Writes the stored oracle results the GPU parity tests compare against.

Calls only the oracle and the seeded circuit generators:

    python tests/golden/make_golden.py            # all
    python tests/golden/make_golden.py mesh       # one

Files (numpy .npz, no pickles): for each workload the DC point, the accepted
time grid and per-step counters of the adaptive oracle run, and the probe
voltages of the oracle's replay of that grid (the reference of the GPU
replay-parity tests).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import netgen  # noqa: E402
from oracle import Oracle, Options  # noqa: E402

WORKLOADS = {
    # RC mesh 32x32, 1,024 nodes, linear, pulse loads, 5 ns
    "mesh": lambda: netgen.config(1),
    # inverter chain, 200 stages, 4,201 nodes, 4 ns
    "chain": lambda: netgen.config(2),
    # a short chain that switches fully inside its window (edge-case coverage)
    "chain12": lambda: netgen.inverter_chain(seed=77, n_stages=12, T=1.5e-9, t_ramp=0.2e-9),
    # the same chain with the ER-C correction (gamma = 0.1)
    "chain12_erc": lambda: netgen.inverter_chain(seed=77, n_stages=12, T=1.5e-9, t_ramp=0.2e-9),
}
# chains sized into each band of the kernel's (threads, rows per thread)
# variants: 841 -> (256, 4), 1,051 -> (256, 6), 1,891 -> (256, 9),
# 2,521 -> (512, 6), 4,201 -> (512, 9), 5,251 -> (512, 12), 6,301 -> (512, 18)
# (and (1024, 9) when that block size is forced)
VARIANT_STAGES = (40, 50, 90, 120, 200, 250, 300)


def variant_chain(L: int):
    return netgen.inverter_chain(seed=500 + L, n_stages=L, T=0.25e-9, t_ramp=0.1e-9)


for _L in VARIANT_STAGES:
    WORKLOADS[f"variant{_L}"] = (lambda L=_L: variant_chain(L))
OPTIONS = {"chain12_erc": lambda: Options(erc=True, gamma=0.1)}


def make(name: str):
    net = WORKLOADS[name]()
    opts = OPTIONS.get(name, Options)()
    t0 = time.time()
    o = Oracle(net, opts)
    x0 = o.dc()
    run = o.run(x0, keep=net.probes)
    t_run = time.time() - t0
    rep = Oracle(net, OPTIONS.get(name, Options)()).replay(x0, run.t, keep="all")
    X = np.array(rep.x)
    out = dict(
        x0=x0, t=np.array(run.t), h=np.array(run.h), h_try=np.array(run.h_try),
        m=np.array(run.m), m_err=np.array(run.m_err), rejects=np.array(run.rejects),
        err=np.array(run.err), rho=np.array(run.rho), probes=np.asarray(net.probes),
        run_probe_x=np.array(run.x),
        replay_probe_x=X[:, net.probes], replay_m=np.array(rep.m), replay_m_err=np.array(rep.m_err),
        replay_err=np.array(rep.err), replay_rho=np.array(rep.rho),
        x_final=X[-1], lu_count=run.lu_count, arnoldi=run.arnoldi_iters, seconds=t_run,
    )
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(f"{name}: {len(run.t)} steps, {sum(run.rejects)} rejections, {t_run:.1f} s -> {path}")


# power grids (the post-layout-style grid of two resistive layers with
# inverter drivers): the oracle's first K accepted steps from its DC point
GRIDS = {
    # 2 x 96 x 96 + 60 drivers, 18,552 nodes, the first 60 accepted steps
    "grid96": (lambda: netgen.power_grid(side=96, n_drivers=60), 60),
    # the full grid: 2 x 512 x 512 + 2,000 drivers, 528,288 nodes, first 20 steps
    "grid512": (lambda: netgen.config(3), 20),
}


def make_grid(name: str):
    build, K = GRIDS[name]
    net = build()
    t0 = time.time()
    o = Oracle(net)
    x0 = o.dc()
    t_dc = time.time() - t0
    run = o.run(x0, keep=net.probes, max_steps=K)
    rep = Oracle(net).replay(x0, run.t, keep=net.probes)
    t_all = time.time() - t0
    out = dict(
        x0=x0, t=np.array(run.t), h=np.array(run.h), h_try=np.array(run.h_try),
        m=np.array(run.m), m_err=np.array(run.m_err), rejects=np.array(run.rejects),
        err=np.array(run.err), rho=np.array(run.rho), probes=np.asarray(net.probes),
        run_probe_x=np.array(run.x), replay_probe_x=np.array(rep.x), replay_m=np.array(rep.m),
        replay_err=np.array(rep.err), x_final=rep.x_final, lu_count=run.lu_count,
        dc_seconds=t_dc, seconds=t_all,
    )
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(f"{name}: n = {net.n}, {len(run.t)} steps, {sum(run.rejects)} rejections, DC {t_dc:.1f} s, "
          f"total {t_all:.1f} s -> {path}")


# the fresh circuit of the learned-controller test: the oracle's adaptive run
# at a 10x tighter budget (E_rr = 1e-7 V), its final state the accuracy
# reference of the GPU runs at E_rr = 1e-6 V
def make_tight(name: str = "fresh120_tight"):
    net = netgen.inverter_chain(seed=6000, n_stages=120)
    t0 = time.time()
    o = Oracle(net, Options(tol=1e-7))
    x0 = o.dc()
    run = o.run(x0, keep=None)
    out = dict(x0=x0, t_final=run.t[-1], steps=len(run.t), x_final=run.x_final, seconds=time.time() - t0)
    path = os.path.join(HERE, f"{name}.npz")
    np.savez_compressed(path, **out)
    print(f"{name}: {len(run.t)} steps at E_rr = 1e-7 V, {time.time() - t0:.1f} s -> {path}")


if __name__ == "__main__":
    for name in (sys.argv[1:] or list(WORKLOADS) + list(GRIDS) + ["fresh120_tight"]):
        if name == "fresh120_tight":
            make_tight(name)
        else:
            (make_grid if name in GRIDS else make)(name)
