"""Algorithm 1 of the paper (MEVP_IKS): Arnoldi on the invert Krylov subspace
K_m(J^{-1}, v) = span{v, -G^{-1}C v, ..., (-G^{-1}C)^{m-1} v}, and the small
Hessenberg exponential that turns the basis into e^{hJ} v (section "MEVP
Using Invert Krylov Subspace").

With A = J^{-1} = -G^{-1} C the Arnoldi relation is
    A V_m = V_m H_m + h_{m+1,m} v_{m+1} e_m^T,
the approximation is e^{hJ} v ~ beta V_m e^{h H_m^{-1}} e_1 (beta = ||v||_2),
and the residual of the approximation (equation of the invert-Krylov error
estimate) is
    r_m(h) = -beta h_{m+1,m} G v_{m+1} e_m^T H_m^{-1} e^{h H_m^{-1}} e_1.
The stopping test uses its G^{-1}-scaled 2-norm
    rho_m(h) = beta h_{m+1,m} |e_m^T H_m^{-1} e^{h H_m^{-1}} e_1|   (volts).

The step needs (I - e^{hJ}) v rather than e^{hJ} v; it is formed from the
augmented matrix [[M, e_1], [0, 0]] with M = h H_m^{-1}, whose exponential
holds y = e^M e_1 in its first column and f = phi_1(M) e_1 in its last, so
    (I - e^{hJ}) v ~ beta V_m d,   d = -M f = e_1 - y
without the cancellation of subtracting two nearly equal n-vectors.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


class KrylovError(RuntimeError):
    """Arnoldi reached m_max without meeting the residual tolerance."""


def hessenberg_phi(Hm: np.ndarray, h_next: float, beta: float, h: float):
    """Small-matrix part of the MEVP at step size h.

    Returns (d, rho): d = (I - e^{M}) e_1 computed as -M phi_1(M) e_1 with
    M = h H_m^{-1}, and the residual norm rho_m(h).  Non-finite results are
    returned as they are; the caller treats them as not converged."""
    m = Hm.shape[0]
    with np.errstate(all="ignore"):
        try:
            Hinv = np.linalg.inv(Hm)             # LU with partial pivoting
        except np.linalg.LinAlgError:
            return np.full(m, np.nan), np.inf
        M = h * Hinv
        aug = np.zeros((m + 1, m + 1))
        aug[:m, :m] = M
        aug[0, m] = 1.0
        if not np.all(np.isfinite(aug)):
            return np.full(m, np.nan), np.inf
        E = scipy.linalg.expm(aug)              # scaling and squaring, Pade
        y = E[:m, 0]
        f = E[:m, m]
        d = -(M @ f)
        rho = beta * h_next * abs((Hinv @ y)[m - 1])
    if not (np.all(np.isfinite(d)) and np.isfinite(rho)):
        return d, np.inf
    return d, rho


def hessenberg_phi2(Hm: np.ndarray, h: float) -> np.ndarray:
    """Small-matrix part of h phi_2(hJ) on the invert Krylov space: with
    M = h H_m^{-1}, returns d2 = -M phi_2(M) e_1 (phi_2(z) = (e^z - 1 - z)/z^2),
    read from the exponential of the augmented matrix
    [[M, e_1, 0], [0, 0, 1], [0, 0, 0]], whose last column holds phi_2(M) e_1.
    With y = G^{-1} b and its basis (beta, V_m, H_m),
        h phi_2(hJ) C^{-1} b ~ beta V_m d2
    (from J^{-1} = -G^{-1} C: h phi_2(hJ) C^{-1} b = y - (1/h)(e^{hJ} - I) A y
    with A = -G^{-1} C, and A y ~ beta V_m H_m e_1)."""
    m = Hm.shape[0]
    with np.errstate(all="ignore"):
        M = h * np.linalg.inv(Hm)
        aug = np.zeros((m + 2, m + 2))
        aug[:m, :m] = M
        aug[0, m] = 1.0
        aug[m, m + 1] = 1.0
        E = scipy.linalg.expm(aug)
        return -(M @ E[:m, m + 1])


class InvertKrylov:
    """Arnoldi state for one start vector v (Algorithm 1).

    apply_A(x) must return -G^{-1} (C x).  The basis and Hessenberg matrix are
    kept so that a later, smaller step size can reuse them (Algorithm 2 reuses
    (V_m, H_m) when it shrinks h) and extend them when the residual asks."""

    def __init__(self, apply_A, v: np.ndarray, m_max: int = 60, breakdown: float = 1e-13):
        self.apply_A = apply_A
        self.m_max = m_max
        self.breakdown = breakdown
        self.n = v.shape[0]
        self.beta = float(np.linalg.norm(v))
        self.V = np.zeros((self.n, m_max + 1))
        self.H = np.zeros((m_max + 1, m_max))
        self.m = 0
        self.exact = self.beta == 0.0
        if not self.exact:
            self.V[:, 0] = v / self.beta
        self.iterations = 0

    def iterate(self):
        """One Arnoldi step: solve -G w = C v_j, then modified Gram-Schmidt
        against v_1..v_j in increasing order, h_{j+1,j} = ||w||, normalise."""
        j = self.m
        w = self.apply_A(self.V[:, j])
        for i in range(j + 1):
            self.H[i, j] = w @ self.V[:, i]
            w = w - self.H[i, j] * self.V[:, i]
        self.H[j + 1, j] = np.linalg.norm(w)
        self.m = j + 1
        self.iterations += 1
        scale = np.max(np.abs(self.H[: j + 2, : j + 1]))
        if self.H[j + 1, j] <= self.breakdown * scale:
            self.exact = True                   # invariant subspace found
            self.H[j + 1, j] = 0.0
        else:
            self.V[:, j + 1] = w / self.H[j + 1, j]

    def phi(self, h: float):
        m = self.m
        return hessenberg_phi(self.H[:m, :m], self.H[m, m - 1], self.beta, h)

    def converge(self, h: float, eps: float):
        """Grow the basis until rho_m(h) <= eps; returns (d, rho)."""
        if self.beta == 0.0:
            return np.zeros(0), 0.0
        if self.m > 0:
            d, rho = self.phi(h)
            if rho <= eps:
                return d, rho
            if self.exact:
                raise KrylovError("invariant subspace with non-finite exponential")
        while True:
            if self.m >= self.m_max:
                raise KrylovError(f"m_max={self.m_max} reached without rho <= {eps:g}")
            self.iterate()
            d, rho = self.phi(h)
            if rho <= eps:
                return d, rho
            if self.exact:
                raise KrylovError("invariant subspace with non-finite exponential")

    def phi2(self, h: float) -> np.ndarray:
        """d2 of hessenberg_phi2 on the current basis (beta V_m d2 ~ h phi_2(hJ) C^{-1} b)."""
        m = self.m
        if self.beta == 0.0 or m == 0:
            return np.zeros(m)
        return hessenberg_phi2(self.H[:m, :m], h)

    def combine(self, d: np.ndarray) -> np.ndarray:
        """beta V_m d"""
        if self.beta == 0.0:
            return np.zeros(self.n)
        return self.beta * (self.V[:, : self.m] @ d)
