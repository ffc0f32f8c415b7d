"""Pins of the oracle's exponential quadrature rules (Sec. 2, eq. 3-5) against
exact solutions: the Fourier closed form of a periodic constant-coefficient
problem, the steady state of a constant source, dense matrix exponentials,
and the convergence orders the paper states."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spla
import scipy.sparse as sps

import workloads as W
from oracle import bounds, integrators, leja
from oracle import operator as O


def op_of(w):
    return O.make_operator(w.Dxx, w.Dxy, w.Dyy, w.ax_field(), w.ay_field(), w.hx, w.hy, w.bc)


def dense(op):
    ny, nx = op.shape
    n = nx * ny
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = O.apply(op, e.reshape(ny, nx)).ravel()
    return M


def fourier_exact(w, T):
    """u(T) = IFFT(exp(lambda T) FFT(u0)) for the constant-coefficient
    periodic stencil, lambda from von Neumann analysis."""
    n = w.nx
    Dxx, Dxy, Dyy = w.Dxx[0, 0], w.Dxy[0, 0], w.Dyy[0, 0]
    k = 2 * np.pi * np.fft.fftfreq(n, d=1.0 / n) / n
    TX, TY = np.meshgrid(k, k)
    lam = (2 * Dxx * (np.cos(TX) - 1) / w.hx ** 2 + 2 * Dyy * (np.cos(TY) - 1) / w.hy ** 2
           - 2 * Dxy * np.sin(TX) * np.sin(TY) / (w.hx * w.hy)
           + 1j * (w.ax_c * np.sin(TX) / w.hx + w.ay_c * np.sin(TY) / w.hy))
    return np.real(np.fft.ifft2(np.exp(lam * T) * np.fft.fft2(w.u0))), lam


def test_periodic_constant_source_free_matches_fourier():
    """The periodic constant-coefficient workload (no source): the midpoint
    step is exp(A dt) exactly, so 10 steps must match the Fourier solution
    to the Leja tolerance."""
    w = W.c1_periodic_constant(n=64, steps=10)
    op = op_of(w)
    A = lambda x: O.apply(op, x)
    alpha, _ = bounds.spectral_bound(op, 0)
    u = w.u0.copy()
    st = {}
    for _ in range(w.steps):
        u = integrators.exp_midpoint_step(A, u, None, w.dt, alpha, w.tol, stats=st)
    ref, lam = fourier_exact(w, w.steps * w.dt)
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    assert err < 2e-9, err
    # exactness in time: one big step of length T equals ten small ones
    u1 = integrators.exp_midpoint_step(A, w.u0, None, w.steps * w.dt, alpha, 1e-12)
    assert np.linalg.norm(u1 - ref) / np.linalg.norm(ref) < 1e-10
    # exact spectral radius of this stencil vs the Gershgorin estimate
    rho = np.max(np.abs(lam))
    assert 1.0 < abs(alpha) / rho < 1.5
    # mass is conserved (column sums of A vanish)
    assert abs(u.sum() - w.u0.sum()) < 1e-12 * abs(w.u0).sum()


def test_constant_source_steady_state_and_exactness():
    """Constant source: u* = -A^{-1} S is a fixed point of both rules and a
    step is exact: u(t) = exp(tA)(u0 - u*) + u*."""
    w = W.c2_dirichlet_circular(n=16, steps=3)
    op = op_of(w)
    A = lambda x: O.apply(op, x)
    M = dense(op)
    S = w.S(0.0)
    ustar = spla.spsolve(sps.csc_matrix(M), -S.ravel()).reshape(S.shape)
    alpha, _ = bounds.spectral_bound(op, 0)
    for step in ("mid", "quad2", "gauss"):
        if step == "mid":
            f = lambda u: integrators.exp_midpoint_step(A, u, S, w.dt, alpha, 1e-12)
        elif step == "quad2":
            f = lambda u: integrators.exp_quad2_step(A, u, S, S, 1 / 3, 2 / 3, w.dt, alpha, 1e-12)
        else:
            c1, c2 = 0.5 - math.sqrt(3) / 6, 0.5 + math.sqrt(3) / 6
            f = lambda u: integrators.exp_quad2_step(A, u, S, S, c1, c2, w.dt, alpha, 1e-12)
        us = f(ustar)
        assert np.linalg.norm(us - ustar) <= 1e-10 * np.linalg.norm(ustar), step
        u1 = f(w.u0)
        ref = (sla.expm(w.dt * M) @ (w.u0 - ustar).ravel()).reshape(S.shape) + ustar
        assert np.linalg.norm(u1 - ref) <= 1e-10 * np.linalg.norm(ref), step


def _tds_problem(n=12):
    X, Y, hx, hy = W.grid_2d(n, n, W.DIRICHLET, box=(-1, 1, -1, 1))
    Dxx, Dxy, Dyy = W.spiral_tensor(X, Y, 1)
    Dxx, Dxy, Dyy = Dxx + 1e-3, Dxy, Dyy + 1e-3
    op = O.make_operator(Dxx, Dxy, Dyy, 1.0, 1.0, hx, hy, W.DIRICHLET)
    u0 = W.gaussian(X, Y, 0.1, -0.2, 0.3)
    S = lambda t: W.source_tds(X, Y, t)
    return op, u0, S


def _integrate(op, u0, S, T, nsteps, scheme, alpha):
    A = lambda x: O.apply(op, x)
    dt = T / nsteps
    u = u0.copy()
    for n in range(nsteps):
        t = n * dt
        if scheme == "mid":
            u = integrators.exp_midpoint_step(A, u, S(t + 0.5 * dt), dt, alpha, 1e-13)
        else:
            c1, c2 = 0.5 - math.sqrt(3) / 6, 0.5 + math.sqrt(3) / 6
            u = integrators.exp_quad2_step(A, u, S(t + c1 * dt), S(t + c2 * dt), c1, c2, dt, alpha, 1e-13)
    return u


def _variation_of_constants(op, u0, S, T):
    """Reference: u(T) = e^{TA} u0 + int_0^T e^{(T-s)A} S(s) ds by composite
    Gauss-Legendre quadrature with dense expm (S is smooth on [0.25, 0.28])."""
    M = dense(op)
    ref = sla.expm((T - 0.25) * M) @ u0.ravel()
    xg, wg = np.polynomial.legendre.leggauss(12)
    edges = np.linspace(0.25, T, 9)
    for a, b in zip(edges[:-1], edges[1:]):
        for xq, wq in zip(xg, wg):
            s = 0.5 * (b - a) * xq + 0.5 * (a + b)
            ref += 0.5 * (b - a) * wq * (sla.expm((T - s) * M) @ S(s).ravel())
    return ref.reshape(u0.shape)


def test_convergence_orders_with_time_dependent_source():
    """Exponential midpoint is second order, exponential Gauss fourth order
    (Sec. 2; Sec. 3 discussion of Figs. 4-5), on spiral-1 diffusion with
    advection and the time-dependent sources of eq. 9, over a window where
    the sources are smooth in t."""
    op, u0, S = _tds_problem()
    alpha, _ = bounds.spectral_bound(op, 0)
    T0, T = 0.25, 0.28
    ref = _variation_of_constants(op, u0, S, T)
    Sshift = lambda t: S(t + T0)
    for scheme, order in (("mid", 2), ("gauss", 4)):
        errs = []
        for nsteps in (2, 4, 8):
            u = _integrate(op, u0, Sshift, T - T0, nsteps, scheme, alpha)
            errs.append(np.linalg.norm(u - ref) / np.linalg.norm(ref))
        rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
        assert all(abs(r - order) < 0.6 for r in rates), (scheme, errs, rates)


def test_gauss_rule_equals_eq5_form():
    """With Gauss nodes the regrouped two-stage rule is eq. 5:
    u + dt phi_1(A dt)(A u + (sqrt3+1)/2 S1 + (1-sqrt3)/2 S2) + dt sqrt3 phi_2(A dt)(S2 - S1)."""
    op, u0, S = _tds_problem(10)
    A = lambda x: O.apply(op, x)
    alpha, _ = bounds.spectral_bound(op, 0)
    c1, c2 = 0.5 - math.sqrt(3) / 6, 0.5 + math.sqrt(3) / 6
    dt = 0.01
    S1, S2 = S(0.3 + c1 * dt), S(0.3 + c2 * dt)
    M = dense(op) * dt
    n = M.shape[0]
    def phil(l, v):
        B = np.zeros((n + l, n + l))
        B[:n, :n] = M
        B[:n, n] = v.ravel()
        for k in range(l - 1):
            B[n + k, n + k + 1] = 1.0
        return sla.expm(B)[:n, n + l - 1].reshape(u0.shape)
    eq5 = (u0 + dt * phil(1, A(u0) + (math.sqrt(3) + 1) / 2 * S1 + (1 - math.sqrt(3)) / 2 * S2)
           + dt * math.sqrt(3) * phil(2, S2 - S1))
    for mode in ("augmented", "two_sweep"):
        u = integrators.exp_quad2_step(A, u0, S1, S2, c1, c2, dt, alpha, 1e-13, mode=mode)
        assert np.linalg.norm(u - eq5) <= 1e-11 * np.linalg.norm(eq5), mode
