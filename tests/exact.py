"""Exact responses of small linear circuits, written independently of the
oracle (test-side references only).

* ``ladder_step``: closed-form modal solution of the uniform RC ladder.  The
  matrix (1/R) tridiag(-1, 2, -1) with last diagonal 1 has eigenvalues
  (4/R) sin^2((2j-1) pi / (2(2N+1))) and eigenvectors
  q_j(i) = sin(i (2j-1) pi / (2N+1)), i, j = 1..N.
* ``linear_exact``: any linear RC circuit with singular C.  The capless nodes
  are eliminated (Kron reduction), the reduced symmetric-definite pencil is
  diagonalised with a generalised eigensolver, and every linear piece of the
  source is integrated in closed form (homogeneous plus ramp particular part).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl


def ladder_step(N, R, c, Vs, t):
    j = np.arange(1, N + 1)
    lam = 4.0 * np.sin((2 * j - 1) * np.pi / (2 * (2 * N + 1))) ** 2
    i = np.arange(1, N + 1)
    Q = np.sin(np.outer(i, 2 * j - 1) * np.pi / (2 * N + 1))
    a = np.linalg.solve(Q, -Vs * np.ones(N))           # x(0) = 0, x(inf) = Vs
    return Vs + (np.exp(-np.outer(np.asarray(t), lam) / (R * c)) * a) @ Q.T


def _pwl(src, t):
    tp, vp = src.t, src.v
    return float(np.interp(t, tp, vp))


def linear_exact(net, x0, ts):
    """x(t) at the times ts (increasing) for C x' = -G x + B u(t), x(0) = x0
    (x0 consistent on the capless nodes is not required: they are algebraic)."""
    G = net.G.toarray(); C = net.C.toarray(); B = net.B.toarray()
    capm = np.abs(C).sum(1) > 0
    cap = np.flatnonzero(capm); nc = np.flatnonzero(~capm)
    Gcc, Gcn = G[np.ix_(cap, cap)], G[np.ix_(cap, nc)]
    Gnc, Gnn = G[np.ix_(nc, cap)], G[np.ix_(nc, nc)]
    Gr = Gcc - Gcn @ np.linalg.solve(Gnn, Gnc)
    Cr = C[np.ix_(cap, cap)]
    lam, W = sl.eigh(Gr, Cr)                             # W^T Cr W = I

    def b_of(t):
        u = np.array([_pwl(s, t) for s in net.sources])
        b = B @ u
        return b[cap] - Gcn @ np.linalg.solve(Gnn, b[nc]), b

    corners = sorted(set(p for s in net.sources for p in s.t if p > 0))
    grid = sorted(set(corners) | set(float(t) for t in ts))
    xc = np.asarray(x0, float)[cap].copy()
    tcur = 0.0
    out = {}
    for tn in grid:
        if tn > tcur:
            b0, _ = b_of(tcur)
            b1, _ = b_of(tn)
            tau = tn - tcur
            s = (b1 - b0) / tau
            y = W.T @ Cr @ xc
            f0, fs = W.T @ b0, W.T @ s
            e = np.exp(-lam * tau)
            y = y * e + f0 * (1 - e) / lam + fs * (tau / lam - (1 - e) / lam ** 2)
            xc = W @ y
            tcur = tn
        _, b = b_of(tn)
        x = np.zeros(net.n)
        x[cap] = xc
        x[nc] = np.linalg.solve(Gnn, b[nc] - Gnc @ xc)
        out[tn] = x
    return np.array([out[float(t)] for t in ts])


def expm_hJ(G, C, h, v):
    """e^{hJ} v with J = -C^{-1} G for singular C, through the eigenvectors
    of A = -G^{-1} C (J^{-1} on range C): each eigen-component mu != 0 is
    scaled by exp(h / mu) and the kernel of C is removed."""
    A = -np.linalg.solve(G, C)
    mu, W = np.linalg.eig(A)
    c = np.linalg.solve(W, v)
    big = np.abs(mu) > 1e-300
    f = np.zeros_like(mu)
    f[big] = np.exp(h / mu[big])
    return np.real(W @ (f * c))
