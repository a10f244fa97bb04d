"""Algorithm 2 of the paper: the exponential Rosenbrock-Euler (ER) transient.

Circuit: C x' = -G_lin x - I_dev(x) + B u(t), C symmetric PSD, maybe singular.

Linearisation at x_k (the chain-rule form in the Rosenbrock-Euler section):
    G_k   = G_lin + J_dev(x_k)            J_dev = dI_dev/dx
    F_k(x) = J_dev(x_k) x - I_dev(x)       so C x' = -G_k x + F_k(x) + B u
    J_k   = -C^{-1} G_k.
The ER step (eq. of x_{k+1}(h_k)) is
    x_{k+1} = x_k + h phi_1(hJ_k) g_k + h^2 phi_2(hJ_k) b_k,
    g_k = C^{-1} r_k,  r_k = B u(t_k) - G_lin x_k - I_dev(x_k),
    b_k = C^{-1} B s_k, s_k = du/dt on the step (u is linear on the step).
The C^{-1} factors cancel against the 1/J denominators of phi_1, phi_2
(J^{-1} C^{-1} = -G^{-1}); with
    w = G_k^{-1} r_k,  p = G_k^{-1} B s_k,  z = G_k^{-1} C p
this gives
    h phi_1(hJ) g_k   = (I - e^{hJ}) w
    h^2 phi_2(hJ) b_k = (e^{hJ} - I) z + h p
    x_{k+1} = x_k + h p + (I - e^{hJ})(w - z).
"combined" mode evaluates (I - e^{hJ}) on the single vector w - z; "literal"
mode evaluates it on w and on z with two MEVPs, as Algorithm 2 computes
phi_1 and phi_2 separately.  They agree to the Krylov tolerance.

Local nonlinear error (eq. of e_rr):
    e_rr = h phi_1(hJ) C^{-1} dF = (I - e^{hJ}) G_k^{-1} dF,
    dF = F_k(x_{k+1}) - F_k(x_k) = J_dev(x_k)(x_{k+1} - x_k) - (I_dev(x_{k+1}) - I_dev(x_k)).
Step control (Algorithm 2): accept when ||e_rr||_inf <= E_rr, otherwise
h <- alpha h and retry with the same LU and Krylov basis; after an accepted
step with i rejections grow by beta when i < 5.

ER-C (the modified correction term, Algorithm 2 with O_pt_c): after the error
estimate, x_{k+1} <- x_{k+1} - gamma h phi_2(hJ) C^{-1} dF, evaluated on the
error MEVP's basis (hessenberg_phi2); the step is accepted on the estimate of
the uncorrected x_{k+1}.

Readings where the paper is silent (each listed in the design notes):
 * steps are clipped to source corners and to T; a clipped step that is
   accepted at its first try lands exactly on the corner;
 * the proposed step h_prop grows as h_prop <- beta h_prop after a first-try
   accept and as (i < 5 ? beta : 1) * h_used after i > 0 rejections, capped at
   h_max (clipping to a corner does not shrink it);
 * eps_K = 0.1 E_rr, residual rho_m in volts; basis reused and extended after
   a rejection when rho_m(h) > eps_K at the new h;
 * h_init = 1e-13 s, h_min = 1e-18 s, h_max = T / 20, m_max = 60.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.sparse.csgraph as csgraph

from .mevp import InvertKrylov, KrylovError
from .mosfet import device_currents
from .sources import source_values, source_slopes, breakpoints


class StepMinError(RuntimeError):
    """The step size fell below h_min."""


class NonFiniteError(RuntimeError):
    """A NaN or Inf appeared in the state."""


@dataclass
class Options:
    tol: float | None = None          # E_rr in volts (default: the netlist's tol)
    eps_krylov: float | None = None   # eps_K (default 0.1 * E_rr)
    alpha: float = 0.5
    beta: float = 2.0
    grow_if_rejects_lt: int = 5
    h_init: float = 1e-13
    h_min: float = 1e-18
    h_max: float | None = None        # default T / 20
    m_max: int = 60
    mode: str = "combined"            # or "literal"
    breakdown: float = 1e-13
    erc: bool = False                 # ER-C: subtract gamma h phi_2(hJ) C^{-1} dF
    gamma: float = 0.1
    max_steps: int = 10_000_000


@dataclass
class Trace:
    t: list = field(default_factory=list)
    h: list = field(default_factory=list)
    m: list = field(default_factory=list)
    m_err: list = field(default_factory=list)
    rejects: list = field(default_factory=list)
    err: list = field(default_factory=list)
    rho: list = field(default_factory=list)
    h_try: list = field(default_factory=list)
    x: list = field(default_factory=list)
    lu_count: int = 0
    arnoldi_iters: int = 0
    x_final: np.ndarray | None = None   # the state at the last accepted time

    def arrays(self):
        return {k: np.asarray(getattr(self, k)) for k in
                ("t", "h", "h_try", "m", "m_err", "rejects", "err", "rho", "x")}


class Oracle:
    def __init__(self, net, opts: Options | None = None):
        self.net = net
        self.o = opts or Options()
        self.E_rr = self.o.tol if self.o.tol is not None else net.tol
        self.eps = self.o.eps_krylov if self.o.eps_krylov is not None else 0.1 * self.E_rr
        self.G = net.G.tocsr()
        self.C = net.C.tocsr()
        self.B = net.B.tocsr()
        self.has_dev = net.n_dev > 0

    # -- pieces ---------------------------------------------------------------
    def stamp(self, x):
        return device_currents(self.net, x)

    def factor(self, Jd):
        Gk = (self.G + Jd).tocsc()
        return spla.splu(Gk)

    def residual_current(self, x, t, I=None):
        """r = B u(t) - G_lin x - I_dev(x)"""
        if I is None:
            I, _ = self.stamp(x)
        return self.B @ source_values(self.net, t) - self.G @ x - I

    # -- DC operating point (Algorithm 2, x(0) = DC_solution) ----------------
    def newton(self, x, t: float = 0.0, g_shunt: float = 0.0, tol: float = 1e-12,
               max_iter: int = 100, vclip: float = 0.3):
        """Damped Newton on B u(t) - G_lin x - I_dev(x) - g_shunt x = 0: each
        update solves (G_k + g_shunt I) dx = r and is scaled down so that
        ||dx||_inf <= vclip; stops when ||dx||_inf <= tol."""
        x = np.array(x, dtype=float)
        shunt = g_shunt * sp.identity(self.net.n, format="csr")
        for _ in range(max_iter):
            I, Jd = self.stamp(x)
            r = self.residual_current(x, t, I) - g_shunt * x
            dx = spla.splu((self.G + Jd + shunt).tocsc()).solve(r)
            big = float(np.max(np.abs(dx))) if dx.size else 0.0
            x = x + (min(1.0, vclip / big) if big > 0 else 1.0) * dx
            if big <= tol:
                return x
        raise RuntimeError(f"DC Newton did not converge (g_shunt = {g_shunt:g})")

    def dc_blocks(self):
        """Strongly connected components of the dependency graph of the DC
        equations (edge i -> j when equation i depends on x_j through G_lin or
        a MOSFET), listed in topological order (sources first).  MOSFET gates
        draw no current, so a gate couples its driver block to the block of
        the gate node in one direction only."""
        n = self.net.n
        dev = self.net.mosfets
        rows = [self.G.tocoo().row]
        cols = [self.G.tocoo().col]
        for eq in ("d", "s"):
            for var in ("d", "g", "s"):
                ok = (dev[eq] >= 0) & (dev[var] >= 0)
                rows.append(dev[eq][ok].astype(np.int64)); cols.append(dev[var][ok].astype(np.int64))
        r = np.concatenate(rows); c = np.concatenate(cols)
        dep = sp.coo_matrix((np.ones(r.size), (r, c)), shape=(n, n)).tocsr()
        nb, label = csgraph.connected_components(dep, directed=True, connection="strong")
        # condensation edges: block(i) depends on block(j)
        bi, bj = label[r], label[c]
        keep = bi != bj
        succ = [set() for _ in range(nb)]
        indeg = np.zeros(nb, dtype=np.int64)
        for a, b in set(zip(bj[keep].tolist(), bi[keep].tolist())):   # b needs a first
            succ[a].add(b)
            indeg[b] += 1
        order, ready = [], sorted(np.flatnonzero(indeg == 0).tolist())
        while ready:
            a = ready.pop()
            order.append(a)
            for b in sorted(succ[a]):
                indeg[b] -= 1
                if indeg[b] == 0:
                    ready.append(b)
        members = [np.flatnonzero(label == b) for b in range(nb)]
        return [members[b] for b in order]

    def dc(self, t: float = 0.0, x0=None, max_iter: int = 100, vclip: float = 0.3):
        """DC operating point.  Newton on each block of dc_blocks() in
        topological order with the earlier blocks held fixed (updates clipped
        to vclip per node), then Newton on the whole system to 1e-12 V."""
        x = np.zeros(self.net.n) if x0 is None else np.array(x0, dtype=float)
        for blk in self.dc_blocks():
            for _ in range(max_iter):
                I, Jd = self.stamp(x)
                r = self.residual_current(x, t, I)[blk]
                Jb = (self.G + Jd)[blk][:, blk].tocsc()
                dx = spla.splu(Jb).solve(r)
                x[blk] += np.clip(dx, -vclip, vclip)
                if np.max(np.abs(dx)) <= 1e-9:
                    break
            else:
                raise RuntimeError("DC block Newton did not converge")
        return self.newton(x, t, 0.0, tol=1e-12)

    # -- one ER step with its trial loop ---------------------------------------
    def _trial_step(self, x, t, h_try, forced=False):
        """Algorithm 2 body for one accepted step starting at (t, x).

        Returns (x_new, h_used, info).  forced=True accepts the first trial
        (replay of a given time grid) but still reports e_rr."""
        o = self.o
        I_k, Jd = self.stamp(x)
        lu = self.factor(Jd)
        self.trace.lu_count += 1
        C = self.C

        def apply_A(vec):                       # -G_k^{-1} C vec
            return -lu.solve(C @ vec)

        r = self.B @ source_values(self.net, t) - self.G @ x - I_k
        s = source_slopes(self.net, t, h_try)
        w = lu.solve(r)
        p = lu.solve(self.B @ s)
        z = lu.solve(C @ p)
        if o.mode == "combined":
            kry = [(1.0, InvertKrylov(apply_A, w - z, o.m_max, o.breakdown))]
        elif o.mode == "literal":
            kry = [(1.0, InvertKrylov(apply_A, w, o.m_max, o.breakdown)),
                   (-1.0, InvertKrylov(apply_A, z, o.m_max, o.breakdown))]
        else:
            raise ValueError(o.mode)
        h = h_try
        i = 0
        while True:
            x1 = x + h * p
            rho = 0.0
            for sign, k in kry:
                d, rk = k.converge(h, self.eps)
                rho = max(rho, rk)
                x1 = x1 + sign * k.combine(d)
            if not np.all(np.isfinite(x1)):
                raise NonFiniteError("non-finite state")
            m_err = 0
            err = 0.0
            if self.has_dev:
                I1, _ = self.stamp(x1)
                dF = Jd @ (x1 - x) - (I1 - I_k)
                ye = lu.solve(dF)
                ke = InvertKrylov(apply_A, ye, o.m_max, o.breakdown)
                de, _ = ke.converge(h, self.eps)
                e = ke.combine(de)
                err = float(np.max(np.abs(e))) if e.size else 0.0
                m_err = ke.m
                self.trace.arnoldi_iters += ke.iterations
                if o.erc:
                    # the ER-C correction (section on the modified correction
                    # term): D = gamma h phi_2(hJ) C^{-1} dF on the error basis
                    x1 = x1 - o.gamma * ke.combine(ke.phi2(h))
            if forced or err <= self.E_rr:
                info = dict(m=max(k.m for _, k in kry), m_err=m_err, rejects=i, err=err, rho=rho,
                            h_try=h_try)
                self.trace.arnoldi_iters += sum(k.iterations for _, k in kry)
                return x1, h, info
            i += 1
            h *= o.alpha
            if h < o.h_min:
                raise StepMinError(f"h = {h:g} < h_min at t = {t:g}")

    def _record(self, t, x, h, info, keep):
        tr = self.trace
        tr.t.append(t); tr.h.append(h)
        tr.m.append(info["m"]); tr.m_err.append(info["m_err"]); tr.rejects.append(info["rejects"])
        tr.err.append(info["err"]); tr.rho.append(info["rho"]); tr.h_try.append(info["h_try"])
        if isinstance(keep, str) and keep == "all":
            tr.x.append(x.copy())
        elif keep is not None:
            tr.x.append(x[keep].copy())

    # -- adaptive transient (Algorithm 2) -----------------------------------
    def run(self, x0, t0: float = 0.0, T: float | None = None, keep="all", max_steps=None):
        """Adaptive ER from (t0, x0) to T.  keep: 'all' | index array | None."""
        o = self.o
        T = self.net.T if T is None else T
        h_max = o.h_max if o.h_max is not None else T / 20
        bps = breakpoints(self.net, T)
        self.trace = Trace()
        x = np.array(x0, dtype=float)
        t = t0
        h_prop = min(o.h_init, h_max)
        steps = 0
        limit = o.max_steps if max_steps is None else max_steps
        while t < T and steps < limit:
            t_bp = bps[np.searchsorted(bps, t, side="right")]
            h_try = min(h_prop, h_max)
            land = False
            if t + h_try * (1.0 + 1e-3) >= t_bp:
                h_try = t_bp - t
                land = True
            x, h_used, info = self._trial_step(x, t, h_try)
            i = info["rejects"]
            t = t_bp if (land and i == 0) else t + h_used
            grow = o.beta if i < o.grow_if_rejects_lt else 1.0
            h_prop = min(h_max, grow * (h_prop if i == 0 else h_used))
            self._record(t, x, h_used, info, keep)
            steps += 1
        self.trace.x_final = x.copy()
        return self.trace

    # -- replay of a given time grid ----------------------------------------
    def replay(self, x0, ts, t0: float = 0.0, keep="all"):
        """Steps x0 through the accepted times ts (t0 < ts[0] < ts[1] ...)."""
        self.trace = Trace()
        x = np.array(x0, dtype=float)
        t = t0
        for tn in ts:
            h = tn - t
            x, _, info = self._trial_step(x, t, h, forced=True)
            t = tn
            self._record(t, x, h, info, keep)
        self.trace.x_final = x.copy()
        return self.trace
