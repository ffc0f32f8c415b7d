"""Exact-in-time reference solutions for the paper's test problems (Sec. 3),
computed without Leja interpolation: the operator's action is assembled into
a sparse matrix and the solution is written with library matrix functions
(scipy's expm_multiply, after Al-Mohy and Higham, and sparse LU solves).

- Case I (no source): u(T) = exp(T A) u0.
- Case II (time-independent source S): u(T) = exp(T A)(u0 - u*) + u*,
  u* = -A^{-1} S the steady state.
- Cases III/IV (eq. 9): each source term is a fixed profile G_i times
  exp(-r_i |t - t_i|), i.e. G_i c_i exp(lam_i (t - a)) on every interval
  [a, b] that contains no t_i (lam_i = +r_i before t_i, -r_i after).  For
  S(t) = sum_i c_i exp(lam_i (t - a)) G_i the variation-of-constants
  integral is exact:  with z_i = c_i (A - lam_i I)^{-1} G_i,
      u(b) = exp((b - a) A)(u(a) + sum_i z_i) - sum_i exp(lam_i (b - a)) z_i
  For lam_i > 0 (every term before its t_i) A - lam_i I is non-singular:
  with constant advection A is a symmetric negative semi-definite diffusion
  part plus a skew-symmetric central advection part, so its eigenvalues have
  Re <= 0.  A negative lam_i (past t_i, end times beyond 0.1) is used only
  where a test checks the result against quadrature.

Test infrastructure only: it reads the operator through oracle.operator.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

import workloads as W
from oracle import integrators, leja
from oracle import operator as O

# (amplitude, centre x, centre y, width, rate r, time t_i) of eq. 9
TDS_TERMS = ((100.0, 0.25, 0.25, 1.5e-2, 10.0, 0.1),
             (70.0, 0.4, -0.4, 2.5e-2, 5.0, 0.3),
             (50.0, -0.6, 0.6, 1.5e-2, 7.5, 0.6))


def op_of(w):
    return O.make_operator(w.Dxx, w.Dxy, w.Dyy, w.ax_field(), w.ay_field(), w.hx, w.hy, w.bc)


def sparse_matrix(op) -> sps.csr_matrix:
    """A as a sparse matrix, from nine applications of the operator to the
    indicator vectors of the 3 x 3 colour classes (i mod 3, j mod 3): the
    nine-point stencil of a node touches one node of each class, so each
    probe reads one matrix entry per (row, class).  Non-periodic grids only."""
    if op.bc != W.DIRICHLET:
        raise ValueError("colour probing needs a non-periodic grid")
    ny, nx = op.shape
    n = nx * ny
    I = np.broadcast_to(np.arange(nx)[None, :], (ny, nx))
    J = np.broadcast_to(np.arange(ny)[:, None], (ny, nx))
    rows, cols, vals = [], [], []
    for cx in range(3):
        for cy in range(3):
            r = O.apply(op, ((I % 3 == cx) & (J % 3 == cy)).astype(float))
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    ii, jj = I + dx, J + dy
                    ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (ii % 3 == cx) & (jj % 3 == cy)
                    rows.append((J * nx + I)[ok])
                    cols.append((jj * nx + ii)[ok])
                    vals.append(r[ok])
    return sps.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))


def tds_profiles(X, Y):
    return [a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / wd) for a, cx, cy, wd, _, _ in TDS_TERMS]


def exact_case_i(M, u0, T):
    return spla.expm_multiply(T * M, u0.ravel()).reshape(u0.shape)


def exact_case_ii(M, u0, S, T):
    us = -spla.spsolve(M.tocsc(), S.ravel())
    return (spla.expm_multiply(T * M, u0.ravel() - us) + us).reshape(u0.shape)


def exact_tds(M, X, Y, u0, t0, t1):
    """u(t1) from u(t0) = u0 under the sources of eq. 9 (see module doc)."""
    G = [g.ravel() for g in tds_profiles(X, Y)]
    cuts = sorted({t0, t1} | {ti for *_, ti in TDS_TERMS if t0 < ti < t1})
    Id = sps.identity(M.shape[0], format="csc")
    u = u0.ravel().copy()
    for a, b in zip(cuts[:-1], cuts[1:]):
        zs = []
        for (_, _, _, _, r, ti), g in zip(TDS_TERMS, G):
            lam = r if b <= ti else -r
            z = spla.spsolve((M - lam * Id).tocsc(), math.exp(-r * abs(a - ti)) * g)
            zs.append((z, lam))
        u = spla.expm_multiply((b - a) * M, u + sum(z for z, _ in zs))
        for z, lam in zs:
            u = u - math.exp(lam * (b - a)) * z
    return u.reshape(u0.shape)


def exact_solution(w, M=None):
    """Exact u(T) of a paper_case workload."""
    if M is None:
        M = sparse_matrix(op_of(w))
    T = w.extra["T"]
    case = w.extra["case"]
    if case == "I":
        return exact_case_i(M, w.u0, T)
    if case == "II":
        return exact_case_ii(M, w.u0, w.S(0.0), T)
    X, Y, _, _ = W.grid_2d(w.nx, w.ny, W.DIRICHLET, box=W.PAPER_BOX)
    return exact_tds(M, X, Y, w.u0, 0.0, T)


def observed_order(steps, errors):
    """Convergence orders between consecutive runs: log(e_k / e_{k+1}) /
    log(n_{k+1} / n_k) for step counts n and errors e."""
    return [math.log(errors[k] / errors[k + 1]) / math.log(steps[k + 1] / steps[k])
            for k in range(len(steps) - 1)]


def oracle_run(w, tol, alpha):
    """The oracle on a paper_case workload: u after w.steps steps of its
    scheme (phi_0 steps for "exp"), and the matvec count."""
    op = op_of(w)
    A = lambda x: O.apply(op, x)
    u, mv = w.u0.copy(), 0
    for k in range(w.steps):
        st = {}
        S1, S2 = w.stage_sources(k)
        if w.scheme == "exp":
            u = leja.phi_apply(A, 0, w.dt, u, alpha, tol, stats=st)
        elif w.scheme == "midpoint":
            u = integrators.exp_midpoint_step(A, u, S1, w.dt, alpha, tol, stats=st)
        else:
            u = integrators.exp_quad2_step(A, u, S1, S2, w.c1, w.c2, w.dt, alpha, tol, stats=st)
        mv += st["matvecs"]
    return u, mv
