"""Exponential quadrature rules (Sec. 2, eq. 3-5).

General rule (eq. 3):
    u^{n+1} = u^n + dt sum_i b_i(A dt) (A u^n + S(t^n + c_i dt)).
s = 1, c_1 = 1/2: b_1 = phi_1, the exponential midpoint rule (eq. 4).
s = 2: b_1 = (c_2 phi_1 - phi_2)/(c_2 - c_1), b_2 = (-c_1 phi_1 + phi_2)/(c_2 - c_1).
Since b_1 + b_2 = phi_1, the two-stage rule regroups exactly into
    u^{n+1} = u^n + dt [phi_1(A dt) w1 + phi_2(A dt) w2],
    w1 = A u^n + (c_2 S_1 - c_1 S_2)/(c_2 - c_1),   w2 = (S_2 - S_1)/(c_2 - c_1),
with S_i = S(t^n + c_i dt); Gauss nodes c = (1 -+ 1/sqrt 3)/2 give eq. 5.
The phi_1 + phi_2 sum is one augmented sweep (Sec. 2); the "two_sweep" mode
evaluates phi_1 w1 and phi_2 w2 by separate interpolations instead.

The caller evaluates S at the quadrature nodes; a missing source is zero.
"""
from __future__ import annotations

import numpy as np

from . import leja


def exp_midpoint_step(A, u, S_half, dt, alpha, tol, max_degree=leja.MAX_DEGREE,
                      rho_max=leja.RHO_MAX, stats=None):
    """u^{n+1} = u^n + dt phi_1(A dt)(A u^n + S(t^n + dt/2))  (eq. 4)."""
    st = stats if stats is not None else {}
    st.setdefault("matvecs", 0)
    st.setdefault("degrees", [])
    w = A(u)
    st["matvecs"] += 1
    if S_half is not None:
        w = w + S_half
    return u + leja.phi_combo(A, w, None, dt, alpha, tol, max_degree, rho_max, st)


def stage_vectors(Au, S1, S2, c1, c2):
    """(w1, w2) of the regrouped two-stage rule; w2 is None without a source."""
    if S1 is None and S2 is None:
        return Au, None
    z = np.zeros_like(Au)
    s1 = z if S1 is None else S1
    s2 = z if S2 is None else S2
    w1 = Au + (c2 * s1 - c1 * s2) / (c2 - c1)
    w2 = (s2 - s1) / (c2 - c1)
    return w1, w2


def exp_quad2_step(A, u, S1, S2, c1, c2, dt, alpha, tol, max_degree=leja.MAX_DEGREE,
                   rho_max=leja.RHO_MAX, stats=None, mode="augmented"):
    """Two-stage exponential quadrature (eq. 3 with s = 2; eq. 5 for Gauss nodes)."""
    if c1 == c2:
        raise ValueError("c1 == c2")
    st = stats if stats is not None else {}
    st.setdefault("matvecs", 0)
    st.setdefault("degrees", [])
    Au = A(u)
    st["matvecs"] += 1
    w1, w2 = stage_vectors(Au, S1, S2, c1, c2)
    if mode == "augmented":
        return u + leja.phi_combo(A, w1, w2, dt, alpha, tol, max_degree, rho_max, st)
    if mode == "two_sweep":
        y = leja.phi_apply(A, 1, dt, w1, alpha, tol, max_degree, rho_max, st)
        if w2 is not None:
            y = y + leja.phi_apply(A, 2, dt, w2, alpha, tol, max_degree, rho_max, st)
        return u + dt * y
    raise ValueError(mode)
