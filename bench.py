"""Benchmark of the exponential Rosenbrock-Euler transient on one MI355X.

Workload (default "batch"): 256 variants of a 200-stage CMOS inverter chain
(4,201 nodes each, identical sparsity; R/C x U(0.9,1.1), V_th + N(0, 20 mV),
input delay U(0, 0.5 ns)) plus 64 chains of U{50..400} stages, 4 ns
transients at E_rr = 1e-6 V, every instance stepped by the GPU library in
one launch.  A bench step is one whole transient of the batch from its DC
point (computed on the GPU, untimed) to T, with the learned step controller
(trained first, untimed, on traces of disjoint circuits).  value = accepted
ER steps summed over instances per second of wall time.

Also reported: the same batch under the paper's step control (time to
solution of both), the library on the single 200-stage chain ("plain", one
instance, the paper's control), the roofline figures of the transient kernel
(algorithmic bytes per launch / its HIP-event duration), and the oracle's CPU
throughput on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--workload batch|chain|mesh|grid]
                    [--controller learned|plain] [--grid-steps K]
"""
from __future__ import annotations

import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Rosenbrock-Euler steps/s; batched+learned vs plain at 1e-6 rel err"
HBM_PEAK_GBS = 8000.0

# HBM traffic of the transient kernel on the default run (batch workload,
# learned control), from two rocprofv3 --pmc passes over this script:
# FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB, the factors being what the same
# counters read for a plain 1 GiB device copy (--copy-bytes).  It is reported
# only while the kernel sources hash to the value it was measured on.
PMC_TRAFFIC = {"sources": ("paper_1511_04515_amd/csrc/engine.hip", "paper_1511_04515_amd/csrc/layout.hpp",
                           "paper_1511_04515_amd/csrc/mlp.hpp", "paper_1511_04515_amd/csrc/devcommon.hpp",
                           "paper_1511_04515_amd/csrc/mosfet.hpp"),
               "sha256_16": "783f2eb571a083d8", "workload": "batch", "controller": "learned", "safety": 0.85,
               "kernel": "k_run<512, 9>",
               "fetch_kib": 12498834521.3, "fetch_factor": 2.0,
               "write_kib": 2322903977.8, "write_factor": 1.0}


def pmc_traffic_bytes(workload, learned, safety, nlaunch, kernel):
    import hashlib
    h = hashlib.sha256()
    for f in PMC_TRAFFIC["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if (h.hexdigest()[:16] != PMC_TRAFFIC["sha256_16"] or workload != PMC_TRAFFIC["workload"]
            or not learned or safety != PMC_TRAFFIC["safety"] or nlaunch != 1 or kernel != PMC_TRAFFIC["kernel"]):
        return None
    return 1024.0 * (PMC_TRAFFIC["fetch_kib"] * PMC_TRAFFIC["fetch_factor"]
                     + PMC_TRAFFIC["write_kib"] * PMC_TRAFFIC["write_factor"])


def workload(name):
    import netgen
    if name == "batch":
        nets = netgen.config(4)
        desc = ("batch: 256 variants of a 200-stage inverter chain (4,201 nodes, shared sparsity) "
                "+ 64 chains of 50-400 stages; level-1 MOSFETs; T = 4 ns; E_rr = 1e-6 V")
    elif name == "variants":
        nets = netgen.config(4)[:256]
        desc = ("the batch's 256 variants of a 200-stage inverter chain (4,201 nodes, shared sparsity); "
                "T = 4 ns; E_rr = 1e-6 V")
    elif name == "chain":
        nets = [netgen.config(2)]
        desc = "one 200-stage inverter chain (4,201 nodes, 400 MOSFETs); T = 4 ns; E_rr = 1e-6 V"
    elif name == "mesh":
        nets = [netgen.config(1)]
        desc = "RC mesh 32x32 (1,024 nodes), 16 pulse loads; T = 5 ns; E_rr = 1e-6 V"
    else:
        raise SystemExit(f"unknown workload {name}")
    return nets, desc


def algorithmic_bytes(sym, net, info, share=1, parts=False):
    """Bytes an ideal implementation moves for the recorded work of one
    instance: 8-byte values, 4-byte indices, the indices of a sparsity
    pattern amortised over the `share` instances of the batch that hold it
    (one read of the index arrays serves all of them).  Per LU: refactor
    (values read and written, pattern) and assembly of G_k and the device
    table; per step: the three right-hand sides (G_lin SpMV, three L/U solve
    pairs, C SpMV, vector traffic); per Arnoldi step: C SpMV + L/U solve pair +
    vector traffic; one read of v_i per Gram-Schmidt product; one read of each
    combined basis column; per trial: re-stamp, the dF solve pair and the
    basis start.  parts=True also returns the bytes of the Arnoldi SpMV +
    solves (the SpTRSV/SpMV phase)."""
    n = net.n
    zLU = sym["lu_col"].size
    zG = net.G.nnz
    zC = net.C.nnz
    D = net.n_dev
    ix = 4.0 / max(share, 1)
    b = info["lu_count"] * ((16 + ix) * zLU + (8 + ix) * zG + 100 * D)
    b += info["steps"] * ((8 + ix) * zG + 3 * (8 + ix) * zLU + (8 + ix) * zC + 80 * n)
    spmv_sptrsv = info["arnoldi"] * ((8 + ix) * zC + (8 + ix) * zLU)
    b += spmv_sptrsv + info["arnoldi"] * 40 * n
    b += info["mgs_terms"] * 8 * n
    b += info["comb_terms"] * 8 * n
    b += info["trials"] * (64 * n + 100 * D + (8 + ix) * zLU)
    return (b, spmv_sptrsv) if parts else b


def pattern_key(net):
    """Identity of a circuit's sparsity pattern (G, C, B, device terminals)."""
    import hashlib
    h = hashlib.sha256()
    for m in (net.G, net.C, net.B):
        h.update(np.asarray(m.indptr, np.int64).tobytes())
        h.update(np.asarray(m.indices, np.int64).tobytes())
    for k in ("d", "g", "s"):
        h.update(np.asarray(net.mosfets[k], np.int64).tobytes())
    return (net.n, h.hexdigest())


def _oracle_sample(args):
    """Worker of cpu_baseline: the oracle's first `steps` accepted ER steps of
    one batch instance from its DC point (the DC solve is not timed)."""
    idx, steps = args
    import netgen
    from oracle import Oracle
    net = netgen.batch_member(idx)
    x0 = Oracle(net).dc()
    t = time.perf_counter()
    tr = Oracle(net).run(x0, keep=None, max_steps=steps)
    return len(tr.t), time.perf_counter() - t, net.n


def cpu_baseline(n_inst=32, steps=100):
    """The oracle (NumPy/SciPy FP64, one thread per process) on a sample of
    the benchmark batch, one instance per process over the host's cores:
    every 10th instance, its first `steps` accepted steps.  value = accepted
    steps summed over the sample / the wall time of the timed runs (each
    worker's timed runs, summed over the workers, spread over `cores`)."""
    import multiprocessing as mp
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    cores = max(1, min(avail, 16, n_inst))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    picks = list(range(0, 320, 320 // n_inst))[:n_inst]
    t = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_oracle_sample, [(i, steps) for i in picks], chunksize=1)
    wall = time.perf_counter() - t
    n_steps = sum(r[0] for r in res)
    busy = sum(r[1] for r in res)
    # the timed runs only (DC solves and interpreter start-up excluded):
    # their summed duration spread over the worker processes
    eff = busy / cores
    return {"value": n_steps / eff, "unit": "instance-steps/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "nproc": avail,
            "single_core_value": n_steps / busy,
            "sample": f"{len(picks)} instances of the benchmark batch (every {320 // n_inst}th: "
                      f"{sum(1 for i in picks if i < 256)} shared-pattern 200-stage chains, "
                      f"{sum(1 for i in picks if i >= 256)} uneven chains), the first {steps} accepted "
                      f"ER steps of each from its DC point: {n_steps} steps, {busy:.1f} s of oracle time "
                      f"on {cores} processes ({wall:.1f} s wall including DC solves and start-up), "
                      f"NumPy/SciPy FP64, one thread per process"}


def grid_measurement(k_steps, log):
    """The single post-layout power grid (2 x 512 x 512 layers + 2,000 inverter
    drivers, 528,288 unknowns) on the multifrontal engine: DC (untimed), then
    k_steps adaptive ER steps of Algorithm 2 from t = 0 timed one by one
    (expri_step with its own h_next); building blocks timed by HIP events:
    one solve pair (forward + backward over the fronts), one numeric
    refactorisation, one C SpMV.  The solve's algorithmic bytes are the
    stored factor entries read once (8 B each) plus the solution and update
    vectors; the refactor's work is its flop count."""
    import numpy as np
    import torch
    import netgen
    import paper_1511_04515_amd as E
    net = netgen.config(3)
    fa = E.frontal_analysis(net, leaf=16)["stats"]
    s = E.Solver(net, probes=[np.zeros(0, np.int32)])
    xs = s.zeros()
    s.dc(xs)
    torch.cuda.synchronize()
    t, h = 0.0, s.opts.h_init
    per, ms_used = [], []
    for _ in range(k_steps):
        t0 = time.perf_counter()
        st = s.step(xs, t, h)[0]
        per.append(time.perf_counter() - t0)
        t, h = st["t"], st["h_next"]
        ms_used.append(st["m"])
    solve_s = s.diag_time(0, reps=10)
    refac_s = s.diag_time(7, reps=3)
    spmv_s = s.diag_time(2, reps=50)
    s.close()
    n = net.n
    solve_bytes = 8.0 * fa["lu_entries"] + 8.0 * 4 * n
    spmv_bytes = 12.0 * net.C.nnz + 16.0 * n
    med = float(np.median(per))
    log(f"grid: {k_steps} steps, median {1e3 * med:.1f} ms/step; solve pair {1e3 * solve_s:.2f} ms, "
        f"refactor {1e3 * refac_s:.1f} ms, C SpMV {1e3 * spmv_s:.3f} ms")
    return {"workload": "power grid 2 x 512 x 512 + 2,000 level-1 inverter drivers (528,288 unknowns, "
                        "4,000 MOSFETs), T = 2 ns, E_rr = 1e-6 V, multifrontal engine",
            "steps_timed": k_steps, "t_reached": t, "steps_per_s": 1.0 / med, "ms_per_step_median": 1e3 * med,
            "krylov_m": ms_used,
            "factor_entries": fa["lu_entries"], "fronts": fa["fronts"], "refactor_flops": fa["flops"],
            "solve_pair_ms": 1e3 * solve_s,
            "solve_roofline": {"bound": "hbm", "bytes": solve_bytes, "achieved": solve_bytes / solve_s / 1e9,
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": solve_bytes / solve_s / 1e9 / HBM_PEAK_GBS},
            "spmv_ms": 1e3 * spmv_s,
            "spmv_roofline": {"bound": "hbm", "bytes": spmv_bytes, "achieved": spmv_bytes / spmv_s / 1e9,
                              "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": spmv_bytes / spmv_s / 1e9 / HBM_PEAK_GBS},
            "refactor_ms": 1e3 * refac_s,
            "refactor_roofline": {"bound": "mfma", "achieved": fa["flops"] / refac_s / 1e12, "peak": 78.6,
                                  "unit": "TFLOP/s", "frac": fa["flops"] / refac_s / 1e12 / 78.6}}


def grid_to_T(ctrl, log, t_end=0.1e-9):
    """The power grid (config 3, from its DC point) up to t_end under the
    paper's step control and under the learned controller (the network
    trained on chain traces): time to solution by HIP events, accepted steps,
    rejections, Arnoldi iterations, and the largest difference of the two
    final states."""
    import numpy as np
    import netgen
    import paper_1511_04515_amd as E
    net = netgen.config(3, T=t_end)
    out, finals = {}, {}
    for mode in ("plain", "learned"):
        log(f"grid to {1e9 * t_end:.2f} ns ({mode}) ...")
        s = E.Solver(net, probes=[np.zeros(0, np.int32)])
        x = s.zeros()
        s.dc(x)
        if mode == "learned":
            s.load_controller(*ctrl)
        try:
            info = s.run(x)[0]
        except E.ExpriError:
            info = s.run_info(0)
        sec, _ = s.kernel_time()
        finals[mode] = x[0].cpu().numpy()
        s.close()
        out[mode] = {"seconds": sec, "accepted_steps": info["steps"], "rejected_trials": info["rejects"],
                     "arnoldi_iterations": info["arnoldi"], "status": info["status"]}
        log(f"grid to T ({mode}): {sec:.2f} s, {info['steps']} steps, {info['rejects']} rejections, "
            f"{info['arnoldi']} Arnoldi")
    out["t_end"] = t_end
    out["learned_vs_plain_time_to_solution"] = out["plain"]["seconds"] / out["learned"]["seconds"]
    out["final_state_max_abs_diff_V"] = float(np.max(np.abs(finals["learned"] - finals["plain"])))
    return out


def controller_training_set():
    """Circuits for the learned controller's training traces, disjoint from
    every benchmarked circuit (seeds 7000+): 16 variants of a 100-stage chain
    and 8 chains of 50-200 stages."""
    import numpy as np
    import netgen
    base = netgen.inverter_chain(seed=7000, n_stages=100).meta["values"]
    nets = [netgen.inverter_chain(seed=7000, n_stages=100, base=base, variation=dict(seed=7100 + i))
            for i in range(16)]
    rng = np.random.default_rng(7200)
    nets += [netgen.inverter_chain(seed=7300 + j, n_stages=int(L)) for j, L in enumerate(rng.integers(50, 201, 8))]
    return nets


def train_controller(log):
    """Plain runs of the training set -> step traces -> GPU training."""
    import numpy as np
    import torch
    import paper_1511_04515_amd as E
    from paper_1511_04515_amd import control
    nets = controller_training_set()
    t0 = time.perf_counter()
    s = E.Solver(nets, probes=[np.zeros(0, np.int32)] * len(nets), trace_cap=8192)
    x = s.zeros()
    s.dc(x)
    s.run(x, max_steps_per_launch=8192)
    X, T = control.samples_from_traces([s.trace(i) for i in range(len(nets))])
    s.close()
    t1 = time.perf_counter()
    params, norm, losses = control.train(X, T, epochs=40, batch=4096, lr=1e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"controller: {len(X)} samples from {len(nets)} training circuits ({t1 - t0:.1f} s), "
        f"trained in {t2 - t1:.1f} s, loss {losses[0]:.3f} -> {losses[-1]:.3f}")
    return params, norm, {"train_samples": int(len(X)), "train_circuits": len(nets),
                          "trace_seconds": t1 - t0, "train_seconds": t2 - t1,
                          "loss_first": float(losses[0]), "loss_last": float(losses[-1])}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch")
    ap.add_argument("--controller", default="learned", choices=("learned", "plain"))
    ap.add_argument("--safety", type=float, default=0.85,
                    help="factor on the learned controller's step (0.85: fastest on its training circuits)")
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="measure each pattern's launch configuration at set-up (untimed) instead of the rule")
    ap.add_argument("--private-patterns", action="store_true",
                    help="give every instance its own copy of the symbolic data (index arrays not shared)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--grid-steps", type=int, default=20,
                    help="adaptive steps of the single 528,288-node power grid (config 3) to time; 0 = skip")
    ap.add_argument("--no-compare", action="store_true", help="skip the plain-control run of the same batch")
    ap.add_argument("--grid-to-T", action="store_true",
                    help="also run the power grid's first 0.1 ns under the paper's control and under the "
                         "learned controller (with the grid workload, or after the batch)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only copy one device buffer of this many bytes to another (twice) and exit: the "
                         "calibration of the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the solver is not sharded "
              f"across GPUs", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1511_04515_amd as E

    if args.copy_bytes:
        torch.cuda.set_device(0)
        a = torch.ones(args.copy_bytes // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        for _ in range(2):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_bytes, "copies": 2}), flush=True)
        return

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    torch.cuda.set_device(0)
    if args.workload == "grid":
        # the single 528,288-node power grid alone (its own JSON line)
        g = grid_measurement(args.grid_steps or 20, log)
        if args.grid_to_T:
            params, norm, _ = train_controller(log)
            g["to_T"] = grid_to_T((params, norm), log)
        print(json.dumps({"metric": "Rosenbrock-Euler steps/s (single power grid, multifrontal engine)",
                          "value": g["steps_per_s"], "unit": "steps/s", "n_gpus": 1,
                          "steps": g["steps_timed"], "warmup": 0, "ms_per_step": g["ms_per_step_median"],
                          "higher_is_better": True, "scaling": "strong", "vs_baseline": None, "dtype": "f64",
                          "data": "synthetic (seeded netgen power grid)",
                          "config": {"workload": g["workload"]}, "grid": g}), flush=True)
        return
    nets, desc = workload(args.workload)
    syms = {}
    for net in nets:
        key = (net.n, net.G.nnz, net.n_dev)
        if key not in syms:
            syms[key] = E.symbolic_analysis(net)
    ctrl, ctrl_info = None, None
    if args.controller == "learned":
        params, norm, ctrl_info = train_controller(log)
        ctrl = (params, norm)
    t_setup = time.perf_counter()
    s = E.Solver(nets, probes=[np.zeros(0, np.int32)] * len(nets), trace_cap=8192,
                 block_size=args.block_size, private_patterns=int(args.private_patterns),
                 autotune=int(args.autotune))
    t_setup = time.perf_counter() - t_setup
    launch_cfg = {}
    for k in range(len(nets)):
        c = s.config(k)
        key = f"{c['block_size']}x{c['max_rows']} slots {c['slots_l']}/{c['slots_u']}"
        launch_cfg[key] = launch_cfg.get(key, 0) + 1
    log(f"set-up {t_setup:.1f} s ({'autotuned' if args.autotune else 'rule'}); launch configurations {launch_cfg}")
    x0 = s.zeros()
    s.dc(x0)
    xs = [x.clone() for x in x0]

    def one_run():
        for x, x_init in zip(xs, x0):
            x.copy_(x_init)
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = s.run(xs, max_steps_per_launch=8192)
        torch.cuda.synchronize()
        return time.perf_counter() - t, info, s.kernel_time()

    mode = "learned" if ctrl else "plain"
    if ctrl:
        s.load_controller(*ctrl, safety=args.safety)
    log(f"{args.workload}: {len(nets)} instances, {sum(n.n for n in nets)} nodes, launch classes "
        f"{[(c['block_size'], c['n_inst']) for c in s.classes()[0]]}, "
        f"{mode} step control")
    for w in range(args.warmup):
        el, _, _ = one_run()
        log(f"warmup {w}: {el:.2f} s")
    torch.cuda.synchronize()
    times, infos, ktimes, cls_times = [], [], [], []
    for k in range(args.steps):
        el, info, kt = one_run()
        times.append(el)
        infos.append(info)
        ktimes.append(kt)
        cls_times.append([c["kernel_s"] for c in s.classes()[0]])
        log(f"step {k}: {el:.2f} s, {sum(i['steps'] for i in info)} accepted ER steps")
    # the median run gives ms_per_step, value and the kernel times alike
    order = sorted(range(len(times)), key=lambda k: times[k])
    med = order[len(order) // 2]
    steps_run = [sum(i["steps"] for i in info) for info in infos]
    value = steps_run[med] / times[med]
    info = infos[med]

    # roofline of the transient kernel: one launch per launch class and run
    # (the classes run concurrently); the dominant kernel is the class with
    # the most algorithmic bytes, timed by HIP events on its own stream
    classes, inst_class = s.classes()
    share = {}
    for net in nets:
        share[pattern_key(net)] = share.get(pattern_key(net), 0) + 1
    cbytes = [0.0] * len(classes)
    sp_bytes = 0.0
    for k, (net, inf) in enumerate(zip(nets, info)):
        b, bsp = algorithmic_bytes(syms[(net.n, net.G.nnz, net.n_dev)], net, inf, share[pattern_key(net)],
                                   parts=True)
        cbytes[inst_class[k]] += b
        sp_bytes += bsp
    q = int(np.argmax(cbytes))
    ksec, nlaunch = ktimes[med]
    class_s = cls_times[med]
    per_launch_bytes = cbytes[q] / max(nlaunch, 1)
    per_launch_s = class_s[q] / max(nlaunch, 1)
    achieved = per_launch_bytes / per_launch_s / 1e9
    kname = f"k_run<{classes[q]['block_size']}, {classes[q]['max_rows']}>"
    traffic = pmc_traffic_bytes(args.workload, ctrl is not None, args.safety, nlaunch, kname)
    # the SpTRSV/SpMV phase (Arnoldi C SpMV + L/U solves) from the in-kernel
    # phase timers: its time summed over instances, spread over the resident
    # workgroups
    wgs = sum(c["workgroups"] for c in classes)
    sp_s = sum(inf["phase_s"]["arnoldi_solve"] for inf in info)
    sp_GBps = sp_bytes / max(sp_s / wgs, 1e-30) / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
            "launches_per_step": nlaunch, "bytes_per_launch": per_launch_bytes,
            "launch_ms": 1e3 * per_launch_s, "timing": f"median of {len(times)} runs (run {med})",
            "classes": [{"kernel": f"k_run<{c['block_size']}, {c['max_rows']}>", "instances": c["n_inst"],
                         "workgroups": c["workgroups"],
                         "launch_ms": 1e3 * cs / max(nlaunch, 1),
                         "bytes_per_launch": b / max(nlaunch, 1),
                         "GBps": b / max(cs, 1e-30) / 1e9} for c, b, cs in zip(classes, cbytes, class_s)],
            "concurrent_ms": 1e3 * ksec / max(nlaunch, 1),
            "all_classes_GBps": sum(cbytes) / max(ksec, 1e-30) / 1e9,
            "spmv_sptrsv": {"bytes": sp_bytes, "phase_s_summed": sp_s, "resident_workgroups": wgs,
                            "GBps": sp_GBps, "frac": sp_GBps / HBM_PEAK_GBS,
                            "what": "Arnoldi C SpMV + L/U solve bytes (indices amortised per pattern) / "
                                    "(phase time summed over instances / resident workgroups)"}}
    if traffic is not None:
        roof["traffic_GBps"] = traffic / per_launch_s / 1e9
        roof["traffic_frac"] = roof["traffic_GBps"] / HBM_PEAK_GBS
    phases = {}
    for inf in info:
        for k, v in inf["phase_s"].items():
            phases[k] = phases.get(k, 0.0) + v
    out = {
        "metric": METRIC, "value": value, "unit": "instance-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * times[med],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded netgen circuits)",
        "config": {"workload": desc, "instances": len(nets), "nodes": int(sum(n.n for n in nets)),
                   "accepted_steps_per_run": int(sum(i["steps"] for i in info)),
                   "rejected_trials_per_run": int(sum(i["rejects"] for i in info)),
                   "arnoldi_iterations_per_run": int(sum(i["arnoldi"] for i in info)),
                   "controller": (f"learned: MLP 8-64-64-2, bfloat16 inference in the transient kernel, "
                                  f"trained on the GPU (float32) from traces of disjoint circuits, "
                                  f"safety {args.safety}") if ctrl else "plain (the paper's alpha/beta rule)",
                   "block_sizes": {f"k_run<{c['block_size']}, {c['max_rows']}>": c["n_inst"] for c in classes},
                   "launch_configurations": launch_cfg, "autotuned": bool(args.autotune),
                   "setup_s": t_setup},
        "time_to_solution_s": times[med],
        "run_seconds": times,
        "roofline": roof,
        "phase_share": {k: v / max(sum(phases.values()), 1e-30) for k, v in phases.items()},
    }
    if ctrl_info:
        out["controller_training"] = ctrl_info
    if ctrl_info and not args.no_compare:
        # the same batch under the paper's step control, for the learned-vs-plain comparison
        s.load_controller(None)
        el, inf_p, _ = one_run()
        steps_p = sum(i["steps"] for i in inf_p)
        out["plain_control_batch"] = {"value": steps_p / el, "unit": "instance-steps/s", "seconds": el,
                                      "accepted_steps": int(steps_p),
                                      "rejected_trials": int(sum(i["rejects"] for i in inf_p)),
                                      "arnoldi_iterations": int(sum(i["arnoldi"] for i in inf_p))}
        out["learned_vs_plain_time_to_solution"] = el / times[med]
        log(f"plain step control on the same batch: {el:.2f} s, {steps_p} accepted ER steps")
    s.close()
    if args.workload == "batch" and not args.no_plain:
        nets1, _ = workload("chain")
        s1 = E.Solver(nets1, probes=[np.zeros(0, np.int32)], trace_cap=8192)
        y0 = s1.zeros()
        s1.dc(y0)
        y = [y0[0].clone()]
        torch.cuda.synchronize()
        t = time.perf_counter()
        inf1 = s1.run(y, max_steps_per_launch=8192)
        torch.cuda.synchronize()
        el1 = time.perf_counter() - t
        out["plain"] = {"workload": "one 200-stage chain, same library, the paper's step control",
                        "value": inf1[0]["steps"] / el1, "unit": "steps/s", "seconds": el1}
        out["batched_vs_plain"] = value / out["plain"]["value"]
        s1.close()
        # the paper's ER-C variant on the same chain (correction gamma = 0.1)
        s2 = E.Solver(nets1, probes=[np.zeros(0, np.int32)], trace_cap=8192, erc=1, gamma=0.1)
        z = [y0[0].clone()]
        torch.cuda.synchronize()
        t = time.perf_counter()
        inf2 = s2.run(z, max_steps_per_launch=8192)
        torch.cuda.synchronize()
        el2 = time.perf_counter() - t
        out["plain_erc"] = {"workload": "the same chain with the ER-C correction (gamma 0.1)",
                            "value": inf2[0]["steps"] / el2, "unit": "steps/s", "seconds": el2,
                            "accepted_steps": inf2[0]["steps"], "rejected_trials": inf2[0]["rejects"]}
        s2.close()
    if args.workload == "batch" and args.grid_steps > 0:
        out["grid"] = grid_measurement(args.grid_steps, log)
        if args.grid_to_T and ctrl is not None:
            out["grid"]["to_T"] = grid_to_T(ctrl, log)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
