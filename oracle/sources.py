"""Piecewise-linear independent sources.

The paper takes u(t) to be piecewise linear over every step [t_k, t_{k+1}]
(the definition of b_k in the Rosenbrock-Euler section), so a step never
crosses a corner of any source waveform.  These helpers evaluate u, its slope
on one linear piece, and the corner times.
"""
from __future__ import annotations

import numpy as np


def _value(t_pts, v_pts, t):
    if t <= t_pts[0]:
        return float(v_pts[0])
    if t >= t_pts[-1]:
        return float(v_pts[-1])
    i = int(np.searchsorted(t_pts, t, side="right")) - 1
    slope = (v_pts[i + 1] - v_pts[i]) / (t_pts[i + 1] - t_pts[i])
    return float(v_pts[i] + (t - t_pts[i]) * slope)


def _slope(t_pts, v_pts, t):
    if t < t_pts[0] or t >= t_pts[-1] or len(t_pts) < 2:
        return 0.0
    i = int(np.searchsorted(t_pts, t, side="right")) - 1
    return float((v_pts[i + 1] - v_pts[i]) / (t_pts[i + 1] - t_pts[i]))


def source_values(net, t):
    """u(t), one entry per source."""
    return np.array([_value(s.t, s.v, t) for s in net.sources], dtype=np.float64)


def source_slopes(net, t, h):
    """du/dt on the linear piece that holds the step [t, t + h] (evaluated at
    its midpoint; the step never crosses a corner)."""
    tm = t + 0.5 * h
    return np.array([_slope(s.t, s.v, tm) for s in net.sources], dtype=np.float64)


def breakpoints(net, T):
    """Sorted source corner times in (0, T), followed by T itself."""
    pts = [p for s in net.sources for p in s.t if 0.0 < p < T]
    return np.array(sorted(set(pts)) + [T], dtype=np.float64)
