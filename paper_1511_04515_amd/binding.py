"""Thin ctypes binding of libexpri.so (include/expri.h).

Argument marshalling only: every numerical step runs in the library's gfx950
kernels.  PyTorch provides device memory (state vectors, workspace) and the
HIP stream.  The binding raises when the library is missing; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexpri.so")

GND, VDD = -1, -2
REC_FIXED = 16
REC_FIELDS = ("t", "h", "h_try", "m", "m_err", "rejects", "err", "rho")
N_FEAT = 8  # step features after the fixed fields (see EXPRI_REC_FIXED in expri.h)

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "ESINGULAR", -4: "EKRYLOV", -5: "ESTEPMIN",
          -6: "ENONFINITE", -7: "EHIP", -8: "EPATTERN", -9: "ENOCONV"}

# the names every C-ABI entry point of include/expri.h exports
ENTRY_POINTS = ("expri_default_opts", "expri_setup", "expri_set_values", "expri_workspace_size",
                "expri_bind_workspace",
                "expri_dc", "expri_factor", "expri_solve", "expri_mevp", "expri_run", "expri_run_noalloc",
                "expri_run_schedule", "expri_step", "expri_step_fixed", "expri_trace", "expri_get_run_info",
                "expri_lu_pattern", "expri_lu_values", "expri_kernel_time", "expri_launch_classes",
                "expri_block_size", "expri_diag_time", "expri_symbolic_create",
                "expri_symbolic_array",
                "expri_symbolic_destroy", "expri_frontal_create", "expri_frontal_array", "expri_frontal_stats",
                "expri_frontal_destroy", "expri_last_error", "expri_destroy",
                "expri_mlp_create", "expri_mlp_set_norm", "expri_mlp_fit_norm", "expri_mlp_get",
                "expri_mlp_grad", "expri_mlp_adam_step", "expri_mlp_forward", "expri_mlp_last_error",
                "expri_mlp_destroy", "expri_controller_load", "expri_instance_config", "expri_autotune_runs")

_p = C.c_void_p
_i32p = C.POINTER(C.c_int32)
_f32p = C.POINTER(C.c_float)
_f64p = C.POINTER(C.c_double)


class Csr(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32), ("nnz", C.c_int32),
                ("rowptr", _i32p), ("colidx", _i32p), ("val", _f64p)]


class Mosfets(C.Structure):
    _fields_ = [("n", C.c_int32), ("type", C.POINTER(C.c_int8)), ("d", _i32p), ("g", _i32p),
                ("s", _i32p), ("kp", _f64p), ("wl", _f64p), ("vth", _f64p), ("lam", _f64p)]


class Pwl(C.Structure):
    _fields_ = [("npts", C.c_int32), ("t", _f64p), ("v", _f64p)]


class Circuit(C.Structure):
    _fields_ = [("n", C.c_int32), ("G", Csr), ("C", Csr), ("B", Csr), ("dev", Mosfets),
                ("n_src", C.c_int32), ("src", C.POINTER(Pwl)), ("vdd", C.c_double),
                ("T", C.c_double), ("n_probe", C.c_int32), ("probe", _i32p)]


class Opts(C.Structure):
    _fields_ = [("E_rr", C.c_double), ("eps_krylov", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("h_init", C.c_double), ("h_min", C.c_double),
                ("h_max", C.c_double), ("breakdown", C.c_double), ("piv_tol", C.c_double),
                ("grow_if_rejects_lt", C.c_int32), ("m_max", C.c_int32),
                ("block_size", C.c_int32), ("trace_cap", C.c_int32),
                ("erc", C.c_int32), ("solve_slots", C.c_int32),
                ("max_workgroups", C.c_int32), ("engine", C.c_int32), ("gamma", C.c_double),
                ("private_patterns", C.c_int32), ("autotune", C.c_int32)]


class RunInfo(C.Structure):
    _fields_ = [("t", C.c_double), ("steps", C.c_int32), ("lu_count", C.c_int32),
                ("rejects", C.c_int32), ("arnoldi", C.c_int32), ("status", C.c_int32),
                ("phase_s", C.c_double * 6), ("trials", C.c_int32), ("mgs_terms", C.c_int64),
                ("comb_terms", C.c_int64)]


class StepInfo(C.Structure):
    _fields_ = [("t", C.c_double), ("h_used", C.c_double), ("h_next", C.c_double), ("err_inf", C.c_double),
                ("krylov_res", C.c_double), ("m", C.c_int32), ("m_err", C.c_int32), ("n_reject", C.c_int32),
                ("status", C.c_int32)]


PHASES = ("factor", "rhs", "arnoldi_solve", "mgs", "hess_phi", "trial")


class ExpriError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libexpri.so (raises if it has not been built).  torch is imported
    first: its HIP runtime is then the one libexpri binds to, so the process
    holds a single HIP / HSA runtime (a second copy loaded ahead of torch's
    leaves one of them without a device)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1511_04515_amd.build.build()")
    import torch  # noqa: F401  (see above)
    lib = C.CDLL(path)
    pp = C.POINTER(_p)
    sig = {
        "expri_default_opts": ([C.POINTER(Opts)], C.c_int),
        "expri_setup": ([C.POINTER(_p), C.POINTER(Circuit), C.c_int32, C.POINTER(Opts), _p], C.c_int),
        "expri_set_values": ([_p, C.c_int32, C.POINTER(Circuit)], C.c_int),
        "expri_workspace_size": ([_p, C.POINTER(C.c_size_t)], C.c_int),
        "expri_bind_workspace": ([_p, _p, C.c_size_t], C.c_int),
        "expri_dc": ([_p, pp, C.c_double], C.c_int),
        "expri_factor": ([_p, pp], C.c_int),
        "expri_solve": ([_p, pp, pp], C.c_int),
        "expri_mevp": ([_p, pp, pp, C.c_double, C.c_double, _i32p, _f64p], C.c_int),
        "expri_run": ([_p, pp, C.c_double, C.c_int32], C.c_int),
        "expri_run_noalloc": ([_p, pp, C.c_double, C.c_int32], C.c_int),
        "expri_run_schedule": ([_p, pp, C.c_double, C.POINTER(_f64p), _i32p], C.c_int),
        "expri_step": ([_p, pp, C.c_double, C.c_double, C.c_double, C.POINTER(StepInfo)], C.c_int),
        "expri_step_fixed": ([_p, pp, C.c_double, C.c_double, C.POINTER(RunInfo)], C.c_int),
        "expri_trace": ([_p, C.c_int32, _f64p, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
        "expri_get_run_info": ([_p, C.c_int32, C.POINTER(RunInfo)], C.c_int),
        "expri_lu_pattern": ([_p, C.c_int32, _i32p, _i32p, _i32p, C.POINTER(C.c_int64), _i32p, _i32p,
                              C.POINTER(C.c_int64)], C.c_int),
        "expri_lu_values": ([_p, C.c_int32, _f64p], C.c_int),
        "expri_kernel_time": ([_p, _f64p, _i32p], C.c_int),
        "expri_launch_classes": ([_p, C.c_int32, _i32p, _i32p, _i32p, _i32p, _f64p, _i32p, _i32p], C.c_int),
        "expri_block_size": ([_p, _i32p], C.c_int),
        "expri_diag_time": ([_p, C.c_int32, C.c_int32, C.c_int32, _f64p], C.c_int),
        "expri_instance_config": ([_p, C.c_int32, _i32p], C.c_int),
        "expri_autotune_runs": ([], C.c_int64),
        "expri_symbolic_create": ([C.POINTER(_p), C.POINTER(Circuit)], C.c_int),
        "expri_frontal_create": ([C.POINTER(_p), C.POINTER(Circuit), C.c_int32], C.c_int),
        "expri_frontal_array": ([_p, C.c_char_p, C.POINTER(C.c_int64), C.c_int64, C.POINTER(C.c_int64)], C.c_int),
        "expri_frontal_stats": ([_p, C.POINTER(C.c_double)], C.c_int),
        "expri_frontal_destroy": ([_p], None),
        "expri_symbolic_array": ([_p, C.c_char_p, _i32p, C.c_int64, C.POINTER(C.c_int64)], C.c_int),
        "expri_symbolic_schedule": ([_p, C.c_int32, C.c_int32], C.c_int),
        "expri_symbolic_destroy": ([_p], None),
        "expri_last_error": ([_p], C.c_char_p),
        "expri_destroy": ([_p], None),
        "expri_mlp_create": ([C.POINTER(_p), _f32p, _p], C.c_int),
        "expri_mlp_set_norm": ([_p, _f32p], C.c_int),
        "expri_mlp_fit_norm": ([_p, _p, _p, C.c_int32], C.c_int),
        "expri_mlp_get": ([_p, _f32p, _f32p], C.c_int),
        "expri_mlp_grad": ([_p, _p, _p, C.c_int32, _f32p, _f32p], C.c_int),
        "expri_mlp_adam_step": ([_p, _p, _p, C.c_int32, C.c_float, _f32p], C.c_int),
        "expri_mlp_forward": ([_p, _p, _p, C.c_int32, C.c_int32], C.c_int),
        "expri_mlp_last_error": ([_p], C.c_char_p),
        "expri_mlp_destroy": ([_p], None),
        "expri_controller_load": ([_p, _f32p, _f32p, C.c_double], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def default_opts(**kw) -> Opts:
    o = Opts()
    load_library().expri_default_opts(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    if "E_rr" in kw and "eps_krylov" not in kw:
        o.eps_krylov = 0.1 * o.E_rr
    return o


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class _Marshal:
    """Keeps the numpy buffers of one setup call alive while C reads them."""

    def __init__(self):
        self.keep = []

    def arr(self, a, dtype, ctype):
        a = _arr(a, dtype)
        if a.size == 0:
            a = np.zeros(1, dtype=dtype)
        self.keep.append(a)
        return _ptr(a, ctype)

    def csr(self, m):
        c = Csr()
        c.n_rows, c.n_cols = m.shape
        c.nnz = int(m.nnz)
        c.rowptr = self.arr(m.indptr, np.int32, C.c_int32)
        c.colidx = self.arr(m.indices, np.int32, C.c_int32)
        c.val = self.arr(m.data, np.float64, C.c_double)
        return c

    def circuit(self, net, probes=None):
        k = Circuit()
        k.n = net.n
        k.G = self.csr(net.G)
        k.C = self.csr(net.C)
        k.B = self.csr(net.B)
        d = net.mosfets
        dv = Mosfets()
        dv.n = int(d.shape[0])
        dv.type = self.arr(d["type"], np.int8, C.c_int8)
        dv.d = self.arr(d["d"], np.int32, C.c_int32)
        dv.g = self.arr(d["g"], np.int32, C.c_int32)
        dv.s = self.arr(d["s"], np.int32, C.c_int32)
        dv.kp = self.arr(d["kp"], np.float64, C.c_double)
        dv.wl = self.arr(d["wl"], np.float64, C.c_double)
        dv.vth = self.arr(d["vth"], np.float64, C.c_double)
        dv.lam = self.arr(d["lam"], np.float64, C.c_double)
        k.dev = dv
        srcs = (Pwl * max(len(net.sources), 1))()
        for i, s in enumerate(net.sources):
            srcs[i].npts = len(s.t)
            srcs[i].t = self.arr(s.t, np.float64, C.c_double)
            srcs[i].v = self.arr(s.v, np.float64, C.c_double)
        self.keep.append(srcs)
        k.n_src = len(net.sources)
        k.src = C.cast(srcs, C.POINTER(Pwl))
        k.vdd = float(net.vdd)
        k.T = float(net.T)
        pr = net.probes if probes is None else probes
        pr = _arr(pr, np.int32)
        k.n_probe = int(pr.size)
        k.probe = self.arr(pr, np.int32, C.c_int32)
        return k


def _dev_ptrs(tensors):
    arr = (C.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])
    return C.cast(arr, C.POINTER(C.c_void_p)), arr


class Solver:
    """A set of circuit instances set up on the current GPU.

    circuits: one netgen.Netlist or a list of them (a batch).  opts: an Opts
    structure or keyword overrides of the defaults.  probes: optional list of
    per-instance node-id arrays recorded in the trace (default: each
    netlist's own probes)."""

    def __init__(self, circuits, opts=None, probes=None, **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("expri needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.lib = load_library()
        if not isinstance(circuits, (list, tuple)):
            circuits = [circuits]
        self.nets = list(circuits)
        self.n_inst = len(self.nets)
        self.opts = opts if isinstance(opts, Opts) else default_opts(**(opts or {}), **kw)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = torch.cuda.current_stream()
        m = _Marshal()
        arr = (Circuit * self.n_inst)()
        self.n_probe = []
        for i, net in enumerate(self.nets):
            arr[i] = m.circuit(net, None if probes is None else probes[i])
            self.n_probe.append(arr[i].n_probe)
        self.ctx = C.c_void_p()
        st = self.lib.expri_setup(C.byref(self.ctx), arr, self.n_inst, C.byref(self.opts),
                                  C.c_void_p(self.stream.cuda_stream))
        del m
        self._check(st)
        size = C.c_size_t()
        self._check(self.lib.expri_workspace_size(self.ctx, C.byref(size)))
        self.ws_bytes = int(size.value)
        self._ws = None
        if self.ws_bytes > 0:  # (the multifrontal engine owns its memory and reports none)
            self._ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
            base = self._ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            self._check(self.lib.expri_bind_workspace(self.ctx, C.c_void_p(aligned), C.c_size_t(self.ws_bytes)))
        bs = C.c_int32()
        self._check(self.lib.expri_block_size(self.ctx, C.byref(bs)))
        self.bs = bs.value

    # -- helpers ---------------------------------------------------------
    def _check(self, st):
        if st != 0:
            msg = self.lib.expri_last_error(self.ctx).decode() if self.ctx else ""
            raise ExpriError(st, msg)

    def zeros(self):
        """One zero state vector per instance (float64, on the GPU)."""
        return [self.torch.zeros(net.n, dtype=self.torch.float64, device=self.device) for net in self.nets]

    def to_device(self, arrays):
        return [self.torch.as_tensor(np.asarray(a, dtype=np.float64), device=self.device).contiguous()
                for a in arrays]

    def _vecs(self, xs):
        if len(xs) != self.n_inst:
            raise ValueError("need one vector per instance")
        for x, net in zip(xs, self.nets):
            if x.dtype != self.torch.float64 or not x.is_cuda or x.numel() != net.n or not x.is_contiguous():
                raise ValueError("state vectors must be contiguous float64 GPU tensors of length n")
        return _dev_ptrs(xs)

    # -- entry points ----------------------------------------------------
    def set_values(self, inst: int, net, probes=None):
        """Give instance `inst` the values of `net` (same sparsity pattern,
        probe count and PWL corner count; see expri_set_values)."""
        if not 0 <= inst < self.n_inst:
            raise IndexError(inst)
        m = _Marshal()
        k = m.circuit(net, probes)
        self._check(self.lib.expri_set_values(self.ctx, inst, C.byref(k)))
        del m
        self.nets[inst] = net

    def dc(self, xs, t0: float = 0.0):
        p, keep = self._vecs(xs)
        self._check(self.lib.expri_dc(self.ctx, p, t0))
        return [self.run_info(i) for i in range(self.n_inst)]

    def factor(self, xs):
        p, keep = self._vecs(xs)
        self._check(self.lib.expri_factor(self.ctx, p))

    def solve(self, bs, ys):
        pb, kb = self._vecs(bs)
        py, ky = self._vecs(ys)
        self._check(self.lib.expri_solve(self.ctx, pb, py))

    def mevp(self, vs, outs, h: float, eps: float):
        pv, kv = self._vecs(vs)
        po, ko = self._vecs(outs)
        m = (C.c_int32 * self.n_inst)()
        rho = (C.c_double * self.n_inst)()
        self._check(self.lib.expri_mevp(self.ctx, pv, po, h, eps, m, rho))
        return list(m), list(rho)

    def run(self, xs, t0: float = 0.0, max_steps_per_launch: int | None = None):
        p, keep = self._vecs(xs)
        ms = self.opts.trace_cap if max_steps_per_launch is None else max_steps_per_launch
        self._check(self.lib.expri_run(self.ctx, p, t0, int(ms)))
        return [self.run_info(i) for i in range(self.n_inst)]

    def run_noalloc(self, xs, t0: float = 0.0, max_steps_per_launch: int | None = None):
        """expri_run with the workspace in the library's static scratch array."""
        p, keep = self._vecs(xs)
        ms = self.opts.trace_cap if max_steps_per_launch is None else max_steps_per_launch
        self._check(self.lib.expri_run_noalloc(self.ctx, p, t0, int(ms)))
        return [self.run_info(i) for i in range(self.n_inst)]

    def workspace_bytes(self) -> int:
        b = C.c_size_t()
        self._check(self.lib.expri_workspace_size(self.ctx, C.byref(b)))
        return b.value

    def run_schedule(self, xs, t_seqs, t0: float = 0.0):
        p, keep = self._vecs(xs)
        seqs = [_arr(s, np.float64) for s in t_seqs]
        sp = (_f64p * self.n_inst)(*[_ptr(s, C.c_double) for s in seqs])
        cnt = (C.c_int32 * self.n_inst)(*[len(s) for s in seqs])
        self._check(self.lib.expri_run_schedule(self.ctx, p, t0, sp, cnt))
        return [self.run_info(i) for i in range(self.n_inst)]

    def step(self, xs, t: float, h: float, tol: float = 0.0):
        """One adaptive step (trial loop at tol) of every instance; a list of
        {t, h_used, h_next, err_inf, krylov_res, m, m_err, n_reject, status}."""
        p, keep = self._vecs(xs)
        info = (StepInfo * self.n_inst)()
        self._check(self.lib.expri_step(self.ctx, p, t, h, tol, info))
        return [{k: getattr(info[i], k) for k, _ in StepInfo._fields_} for i in range(self.n_inst)]

    def step_fixed(self, xs, t: float, h: float):
        p, keep = self._vecs(xs)
        info = (RunInfo * self.n_inst)()
        self._check(self.lib.expri_step_fixed(self.ctx, p, t, h, info))
        return [self._info_dict(info[i]) for i in range(self.n_inst)]

    @staticmethod
    def _info_dict(r):
        return {"t": r.t, "steps": r.steps, "lu_count": r.lu_count, "rejects": r.rejects,
                "arnoldi": r.arnoldi, "status": r.status,
                "phase_s": dict(zip(PHASES, list(r.phase_s))), "trials": r.trials,
                "mgs_terms": r.mgs_terms, "comb_terms": r.comb_terms}

    def run_info(self, inst: int):
        r = RunInfo()
        self._check(self.lib.expri_get_run_info(self.ctx, inst, C.byref(r)))
        return self._info_dict(r)

    def trace(self, inst: int):
        """Accepted-step records of the last run of one instance."""
        n = C.c_int64()
        self._check(self.lib.expri_trace(self.ctx, inst, None, 0, C.byref(n)))
        rec = REC_FIXED + self.n_probe[inst]
        buf = np.zeros((max(n.value, 1), rec))
        self._check(self.lib.expri_trace(self.ctx, inst, _ptr(buf, C.c_double), n.value, C.byref(n)))
        buf = buf[: n.value]
        out = {k: buf[:, i] for i, k in enumerate(REC_FIELDS)}
        out["feat"] = buf[:, len(REC_FIELDS):len(REC_FIELDS) + N_FEAT]
        out["x"] = buf[:, REC_FIXED:]
        return out

    def diag_time(self, what: int, reps: int = 100, arg: int = 8) -> float:
        """Seconds per repetition of one step building block (see expri.h);
        overwrites instance 0's basis and Hessenbergs."""
        sec = C.c_double()
        self._check(self.lib.expri_diag_time(self.ctx, what, reps, arg, C.byref(sec)))
        return sec.value

    def classes(self):
        """(classes, inst_class): the launch classes of the batch as
        [{"block_size", "max_rows", "n_inst", "workgroups", "kernel_s"}],
        (block size, rows-per-thread bound) descending (workgroups: the
        transient kernel's grid; kernel_s: the last transient call's summed
        duration of that class's launches), and the class index of every
        instance."""
        n = C.c_int32()
        self._check(self.lib.expri_launch_classes(self.ctx, 0, None, None, None, None, None, None, C.byref(n)))
        bs = (C.c_int32 * n.value)()
        mr = (C.c_int32 * n.value)()
        cnt = (C.c_int32 * n.value)()
        wg = (C.c_int32 * n.value)()
        ks = (C.c_double * n.value)()
        ic = np.zeros(self.n_inst, np.int32)
        self._check(self.lib.expri_launch_classes(self.ctx, n.value, bs, mr, cnt, wg, ks, _ptr(ic, C.c_int32),
                                                  C.byref(n)))
        return [{"block_size": bs[q], "max_rows": mr[q], "n_inst": cnt[q], "workgroups": wg[q], "kernel_s": ks[q]}
                for q in range(n.value)], ic

    def config(self, inst: int) -> dict:
        """Launch configuration of instance inst: block size, the transient
        kernel's rows-per-thread bound and the solve passes' slots per lane
        (L and U), as the rule or the autotuner chose them."""
        cfg = (C.c_int32 * 4)()
        self._check(self.lib.expri_instance_config(self.ctx, int(inst), cfg))
        return {"block_size": cfg[0], "max_rows": cfg[1], "slots_l": cfg[2], "slots_u": cfg[3]}

    def kernel_time(self):
        """(seconds, launches) of the transient kernel in the last run call."""
        sec = C.c_double()
        n = C.c_int32()
        self._check(self.lib.expri_kernel_time(self.ctx, C.byref(sec), C.byref(n)))
        return sec.value, n.value

    def lu_pattern(self, inst: int):
        nnz = C.c_int64()
        nl = C.c_int32()
        nu = C.c_int32()
        fl = C.c_int64()
        self._check(self.lib.expri_lu_pattern(self.ctx, inst, None, None, None, C.byref(nnz), C.byref(nl),
                                              C.byref(nu), C.byref(fl)))
        n = self.nets[inst].n
        rp = np.zeros(n + 1, np.int32)
        col = np.zeros(max(nnz.value, 1), np.int32)
        perm = np.zeros(n, np.int32)
        self._check(self.lib.expri_lu_pattern(self.ctx, inst, _ptr(rp, C.c_int32), _ptr(col, C.c_int32),
                                              _ptr(perm, C.c_int32), C.byref(nnz), C.byref(nl),
                                              C.byref(nu), C.byref(fl)))
        return {"rowptr": rp, "col": col[: nnz.value], "perm": perm, "n_lev": nl.value,
                "n_ulev": nu.value, "flops": fl.value}

    def lu_values(self, inst: int):
        nnz = self.lu_pattern(inst)["col"].size
        out = np.zeros(nnz)
        self._check(self.lib.expri_lu_values(self.ctx, inst, _ptr(out, C.c_double)))
        return out

    def load_controller(self, params=None, norm=None, safety: float = 0.85):
        """Use a trained network as the step controller of run() (None: the
        paper's alpha/beta rule).  The default safety factor was chosen on
        the controller's own training circuits (fastest of 0.8 to 1.0)."""
        if params is None:
            self._check(self.lib.expri_controller_load(self.ctx, None, None, 1.0))
            return
        p = np.ascontiguousarray(params, np.float32)
        q = np.ascontiguousarray(norm, np.float32)
        if p.size != MLP_PARAMS or q.size != MLP_NORM:
            raise ValueError("expected MLP_PARAMS parameters and MLP_NORM standardisation values")
        self._check(self.lib.expri_controller_load(self.ctx, _ptr(p, C.c_float), _ptr(q, C.c_float),
                                                   C.c_double(safety)))

    def close(self):
        if self.ctx:
            self.torch.cuda.synchronize()
            self.lib.expri_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SYMBOLIC_ARRAYS = ("perm", "lu_rowptr", "lu_col", "lu_diag", "lev_ptr", "lev_rows", "ulev_ptr",
                   "ulev_rows", "row_grp", "grp_pos", "grp_diag", "grp_ptr", "pair_src", "pair_dst",
                   "lu_gidx", "jac_ptr", "jac_code", "node_ptr", "node_code", "g_rowptr", "g_col",
                   "g_src", "c_rowptr", "c_col", "c_src", "b_rowptr", "b_col", "b_src", "dev_node",
                   "block_of")


SCHEDULE_ARRAYS = ("lsched", "usched", "slot_pos", "slot_col", "row_of", "pass_code", "c_ell_col")


def autotune_runs() -> int:
    """Trial contexts the autotuner has run in this process."""
    return int(load_library().expri_autotune_runs())


def symbolic_analysis(net, block_size: int | None = None, solve_slots: int = 0) -> dict:
    """Host-only symbolic analysis of one netlist (no GPU): every integer
    array the kernels are driven by, by name; with block_size also the
    flattened solve schedules built for that launch block size (and
    solve_slots slots per lane, 0 = automatic)."""
    lib = load_library()
    m = _Marshal()
    k = m.circuit(net)
    h = C.c_void_p()
    st = lib.expri_symbolic_create(C.byref(h), C.byref(k))
    if st != 0:
        raise ExpriError(st, "symbolic analysis failed")
    out = {}
    try:
        names = SYMBOLIC_ARRAYS
        if block_size is not None:
            st = lib.expri_symbolic_schedule(h, int(block_size), int(solve_slots))
            if st != 0:
                raise ExpriError(st, "schedule build failed")
            names = SYMBOLIC_ARRAYS + SCHEDULE_ARRAYS
        for name in names:
            n = C.c_int64()
            lib.expri_symbolic_array(h, name.encode(), None, 0, C.byref(n))
            a = np.zeros(max(n.value, 1), np.int32)
            lib.expri_symbolic_array(h, name.encode(), _ptr(a, C.c_int32), n.value, C.byref(n))
            out[name] = a[: n.value]
    finally:
        lib.expri_symbolic_destroy(h)
    return out


FRONTAL_ARRAYS = ("perm", "c0", "nc", "fsz", "parent", "height", "r_ptr", "r_idx", "rel", "f_off", "u_off",
                  "owner", "lev_ptr", "lev_front", "ch_ptr", "ch", "ent_pos", "ent_row", "ent_g", "ent_jptr", "ent_jcode",
                  "g_rowptr", "g_col", "g_src", "c_rowptr", "c_col", "c_src", "b_rowptr", "b_col", "b_src",
                  "dev_node", "node_ptr", "node_code")
FRONTAL_STATS = ("fronts", "front_doubles", "lu_entries", "flops", "max_front", "max_pivots", "heights",
                 "update_doubles")


def frontal_analysis(net, leaf: int = 32) -> dict:
    """Host-only multifrontal analysis of one netlist (no GPU): the arrays of
    the separator tree of fronts by name (int64) and its statistics."""
    lib = load_library()
    m = _Marshal()
    k = m.circuit(net)
    h = C.c_void_p()
    st = lib.expri_frontal_create(C.byref(h), C.byref(k), int(leaf))
    if st != 0:
        raise ExpriError(st, "frontal analysis failed")
    out = {}
    try:
        for name in FRONTAL_ARRAYS:
            n = C.c_int64()
            lib.expri_frontal_array(h, name.encode(), None, 0, C.byref(n))
            a = np.zeros(max(n.value, 1), np.int64)
            lib.expri_frontal_array(h, name.encode(), _ptr(a, C.c_int64), n.value, C.byref(n))
            out[name] = a[: n.value]
        st_ = (C.c_double * 8)()
        lib.expri_frontal_stats(h, st_)
        out["stats"] = dict(zip(FRONTAL_STATS, list(st_)))
    finally:
        lib.expri_frontal_destroy(h)
    return out


MLP_PARAMS = 4866
MLP_NORM = 20


class Mlp:
    """The learned step controller's network on the current GPU (training in
    float32, inference in float32 or bfloat16).  X (n x 8) and T (n x 2) are
    float32 CUDA tensors; params is a float array of MLP_PARAMS values."""

    def __init__(self, params):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("expri needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.torch = torch
        self.lib = load_library()
        p = np.ascontiguousarray(params, np.float32)
        if p.size != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters, got {p.size}")
        self.stream = torch.cuda.current_stream()
        self.h = C.c_void_p()
        self._check(self.lib.expri_mlp_create(C.byref(self.h), _ptr(p, C.c_float),
                                              C.c_void_p(self.stream.cuda_stream)))

    def _check(self, st):
        if st != 0:
            msg = self.lib.expri_mlp_last_error(self.h).decode() if self.h else ""
            raise ExpriError(st, msg)

    def _samples(self, X, T=None):
        for A, w in ((X, 8), (T, 2)):
            if A is not None and (A.dtype != self.torch.float32 or A.dim() != 2 or A.shape[1] != w
                                  or not A.is_cuda or not A.is_contiguous()):
                raise ValueError(f"expected a contiguous float32 CUDA tensor of shape (n, {w})")
        if T is not None and T.shape[0] != X.shape[0]:
            raise ValueError("X and T differ in length")
        return X.shape[0]

    def set_norm(self, norm):
        a = np.ascontiguousarray(norm, np.float32)
        self._check(self.lib.expri_mlp_set_norm(self.h, _ptr(a, C.c_float)))

    def fit_norm(self, X, T):
        n = self._samples(X, T)
        self._check(self.lib.expri_mlp_fit_norm(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), n))

    def params(self):
        out = np.zeros(MLP_PARAMS, np.float32)
        self._check(self.lib.expri_mlp_get(self.h, _ptr(out, C.c_float), None))
        return out

    def norm(self):
        out = np.zeros(MLP_NORM, np.float32)
        self._check(self.lib.expri_mlp_get(self.h, None, _ptr(out, C.c_float)))
        return out

    def grad(self, X, T):
        n = self._samples(X, T)
        loss = np.zeros(1, np.float32)
        g = np.zeros(MLP_PARAMS, np.float32)
        self._check(self.lib.expri_mlp_grad(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), n,
                                            _ptr(loss, C.c_float), _ptr(g, C.c_float)))
        return float(loss[0]), g

    def adam_step(self, X, T, lr: float = 1e-3, want_loss: bool = False):
        n = self._samples(X, T)
        loss = np.zeros(1, np.float32)
        self._check(self.lib.expri_mlp_adam_step(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(T.data_ptr()), n,
                                                 C.c_float(lr), _ptr(loss, C.c_float) if want_loss else None))
        return float(loss[0]) if want_loss else None

    def forward(self, X, bf16: bool = True):
        n = self._samples(X)
        Y = self.torch.empty((n, 2), dtype=self.torch.float32, device=X.device)
        self._check(self.lib.expri_mlp_forward(self.h, C.c_void_p(X.data_ptr()), C.c_void_p(Y.data_ptr()), n,
                                               1 if bf16 else 0))
        return Y

    def close(self):
        if self.h:
            self.torch.cuda.synchronize()
            self.lib.expri_mlp_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
