"""The paper's test problems (Sec. 3, Cases I-IV) on the CPU: the exact
references of paper_refs.py pinned against dense matrix functions, and the
oracle's behaviour on these problems against them (the Leja half of the
work-precision study and the orders of the two quadrature rules)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import paper_refs as R
import workloads as W
from oracle import bounds
from oracle import operator as O


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_paper_case_inputs():
    """Eq. 6-9 as generated: ring and spiral tensors are v v^T (rank one),
    the advection of each case, the end times and the step rule."""
    for case in W.PAPER_CASES:
        w = W.paper_case(case, 30)
        det = w.Dxx * w.Dyy - w.Dxy ** 2
        assert np.abs(det).max() <= 1e-13 * np.abs(w.Dxx * w.Dyy).max()
        assert (w.ax_c, w.ay_c) == {"I": (0, 0), "II": (1, 1), "III": (1, 1), "IV": (1, 2)}[case]
        assert abs(w.steps * w.dt - w.extra["T"]) < 1e-15
    X, Y, _, _ = W.grid_2d(30, 30, W.DIRICHLET, box=W.PAPER_BOX)
    w = W.paper_case("I", 30)
    assert np.allclose(w.Dxx, Y * Y) and np.allclose(w.Dxy, -X * Y) and np.allclose(w.Dyy, X * X)
    w = W.paper_case("IV", 30)
    assert np.allclose(w.Dxx, (X + 4 * Y) ** 2) and np.allclose(w.Dxy, -X * X - 4 * X * Y)
    assert W.paper_case("I", 30).steps == 1
    w = W.paper_case("III", 30, dt_mult=50.0, T=0.3)
    assert w.dt <= 50.0 * w.extra["dt_cfl"] and w.scheme == "quad2"
    assert abs(w.c1 + w.c2 - 1.0) < 1e-15 and abs(w.c2 - w.c1 - 1.0 / math.sqrt(3.0)) < 1e-15


def test_sparse_assembly_matches_the_operator():
    w = W.paper_case("IV", 23)
    op = R.op_of(w)
    M = R.sparse_matrix(op)
    v = np.random.default_rng(3).standard_normal((23, 23))
    assert rel(M @ v.ravel(), O.apply(op, v).ravel()) < 1e-15
    assert M.nnz <= 9 * 23 * 23


@pytest.mark.parametrize("case", ["III", "IV"])
def test_exact_tds_reference_against_quadrature(case):
    """The closed form for the sources of eq. 9 against dense expm and
    composite Gauss-Legendre quadrature of the variation-of-constants
    integral on panels of width 0.0025 (the stiffest modes of exp((T - s) A)
    decay on a scale of 1/rho ~ 4e-4 here; panel edges include the kink at
    t = 0.1), to T = 0.3: past the first source time, so both signs of lam_i
    occur."""
    n, T = 9, 0.3
    w = W.paper_case(case, n, T=T)
    op = R.op_of(w)
    M = R.sparse_matrix(op)
    X, Y, _, _ = W.grid_2d(n, n, W.DIRICHLET, box=W.PAPER_BOX)
    got = R.exact_tds(M, X, Y, w.u0, 0.0, T)
    Md = M.toarray()
    ref = sla.expm(T * Md) @ w.u0.ravel()
    xg, wg = np.polynomial.legendre.leggauss(16)
    edges = np.linspace(0.0, T, 121)
    for a, b in zip(edges[:-1], edges[1:]):
        for xq, wq in zip(xg, wg):
            s = 0.5 * (b - a) * xq + 0.5 * (a + b)
            ref += 0.5 * (b - a) * wq * (sla.expm((T - s) * Md) @ W.source_tds(X, Y, s).ravel())
    assert rel(got.ravel(), ref) < 1e-11


def test_exact_case_ii_reference():
    """Case II: the steady state u* = -A^{-1} S is a fixed point of the exact
    solution, and the solution at T matches dense expm."""
    w = W.paper_case("II", 10)
    M = R.sparse_matrix(R.op_of(w))
    S = w.S(0.0)
    us = -np.linalg.solve(M.toarray(), S.ravel()).reshape(S.shape)
    assert rel(R.exact_case_ii(M, us, S, 0.85), us) < 1e-12
    ref = (sla.expm(0.85 * M.toarray()) @ (w.u0 - us).ravel()).reshape(S.shape) + us
    assert rel(R.exact_case_ii(M, w.u0, S, 0.85), ref) < 1e-11
    assert rel(R.exact_case_i(M, w.u0, 0.85), (sla.expm(0.85 * M.toarray()) @ w.u0.ravel()).reshape(S.shape)) < 1e-11


@pytest.mark.parametrize("case,n", [("I", 24), ("I", 64), ("II", 24)])
def test_oracle_work_precision_cases_i_ii(case, n):
    """Cases I and II, whose solutions are exact in time (Sec. 3, Fig. 3):
    with tol the accuracy asked of the result, the error against the exact solution stays
    within 10 tol for every tol from 1e-4 to 1e-10, and the matvec count
    rises as tol falls.  Case I at 64^2 is one phi_0 step over the whole
    interval in K = 5 substeps (the chained sweeps share tol), Case II at
    24^2 one midpoint step in K = 8 substeps; a one-term stopping test misses
    this bound by up to 2000 tol."""
    w = W.paper_case(case, n)
    M = R.sparse_matrix(R.op_of(w))
    ref = R.exact_solution(w, M)
    alpha = bounds.gershgorin(R.op_of(w))
    errs, mvs = [], []
    for e in range(4, 11):
        u, mv = R.oracle_run(w, 10.0 ** -e, alpha)
        errs.append(rel(u, ref))
        mvs.append(mv)
    assert all(a <= b for a, b in zip(mvs, mvs[1:])), mvs
    for e, err in zip(range(4, 11), errs):
        assert err <= 10 * 10.0 ** -e, (e, err, errs)


@pytest.mark.parametrize("case", ["III", "IV"])
def test_oracle_orders_on_time_dependent_sources(case):
    """Cases III/IV to T = 0.1 at tol 1e-12: exponential midpoint converges
    with order 2 and exponential Gauss with order 4 (Sec. 2), Gauss being the
    more accurate at every step size."""
    n = 20
    w0 = W.paper_case(case, n)
    M = R.sparse_matrix(R.op_of(w0))
    ref = R.exact_solution(w0, M)
    alpha = bounds.gershgorin(R.op_of(w0))
    res = {}
    for scheme in ("midpoint", "quad2"):
        steps, errs = [], []
        for mult in (80.0, 40.0, 20.0):
            w = W.paper_case(case, n, dt_mult=mult, scheme=scheme)
            u, _ = R.oracle_run(w, 1e-12, alpha)
            steps.append(w.steps)
            errs.append(rel(u, ref))
        res[scheme] = (steps, errs)
    om = R.observed_order(*res["midpoint"])
    og = R.observed_order(*res["quad2"])
    assert all(1.5 <= p <= 2.5 for p in om), om
    assert all(p >= 3.2 for p in og), og
    assert all(g < m for g, m in zip(res["quad2"][1], res["midpoint"][1]))
