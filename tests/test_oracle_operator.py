"""Pins of the oracle's operator A (discretisation of div(D grad u) + div(a u),
Sec. 1 eq. 2) against facts that do not come from its own formula."""
import math

import numpy as np
import pytest
import sympy as sp

import workloads as W
from oracle import operator as O


def dense(op):
    ny, nx = op.shape
    n = nx * ny
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = O.apply(op, e.reshape(ny, nx)).ravel()
    return M


def fourier_symbol(Dxx, Dxy, Dyy, ax, ay, hx, hy, tx, ty):
    """Exact eigenvalue of the constant-coefficient periodic stencil on the
    mode exp(i(tx i + ty j)) (von Neumann analysis of the central stencil)."""
    return (2 * Dxx * (np.cos(tx) - 1) / hx ** 2 + 2 * Dyy * (np.cos(ty) - 1) / hy ** 2
            - 2 * Dxy * np.sin(tx) * np.sin(ty) / (hx * hy)
            + 1j * (ax * np.sin(tx) / hx + ay * np.sin(ty) / hy))


@pytest.mark.parametrize("nx,ny", [(8, 8), (6, 10), (9, 5)])
def test_fourier_modes_are_eigenvectors(nx, ny):
    Dxx, Dxy, Dyy, ax, ay = 0.7525, 0.428683, 0.2575, 0.1, -0.35
    hx, hy = 1.0 / nx, 0.7 / ny
    op = O.make_operator(np.full((ny, nx), Dxx), np.full((ny, nx), Dxy), np.full((ny, nx), Dyy),
                         ax, ay, hx, hy, O.PERIODIC)
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    for kx in range(nx):
        for ky in range(ny):
            tx, ty = 2 * math.pi * kx / nx, 2 * math.pi * ky / ny
            mode = np.exp(1j * (tx * i + ty * j))
            lam = fourier_symbol(Dxx, Dxy, Dyy, ax, ay, hx, hy, tx, ty)
            Au = O.apply(op, mode.real) + 1j * O.apply(op, mode.imag)
            assert np.max(np.abs(Au - lam * mode)) <= 1e-12 * max(1.0, abs(lam))


def test_fourier_spectrum_matches_dense_eigenvalues():
    nx = ny = 8
    c = (0.7525, 0.428683, 0.2575, 0.1, 0.05)
    h = 1.0 / 8
    op = O.make_operator(np.full((8, 8), c[0]), np.full((8, 8), c[1]), np.full((8, 8), c[2]),
                         c[3], c[4], h, h, O.PERIODIC)
    ev = np.linalg.eigvals(dense(op))
    t = 2 * math.pi * np.arange(8) / 8
    TX, TY = np.meshgrid(t, t)
    lam = fourier_symbol(*c, h, h, TX, TY).ravel()
    key = lambda z: (round(z.real, 6), round(z.imag, 6))
    a = np.array(sorted(ev, key=key))
    b = np.array(sorted(lam, key=key))
    assert np.max(np.abs(a - b)) < 1e-9 * np.max(np.abs(b))


def test_periodic_mass_conservation_variable_coefficients():
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(13, 11, seed=3, field_advection=True)
    op = O.make_operator(Dxx, Dxy, Dyy, ax, ay, 1 / 13, 1 / 11, O.PERIODIC)
    u = W.random_vector((11, 13), 1)
    Au = O.apply(op, u)
    assert abs(Au.sum()) <= 1e-13 * np.abs(Au).sum()


@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
def test_symmetric_without_advection(bc):
    Dxx, Dxy, Dyy, _, _ = W.random_fields(12, 9, seed=5, advect=False)
    op = O.make_operator(Dxx, Dxy, Dyy, 0.0, 0.0, 0.08, 0.11, bc)
    M = dense(op)
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    # negative semi-definite for a positive semi-definite tensor field
    assert np.max(np.linalg.eigvalsh(0.5 * (M + M.T))) <= 1e-9 * np.max(np.abs(M))


def test_dirichlet_constant_coefficients_kronecker_form():
    """Constant coefficients, Dirichlet: A equals the textbook Kronecker sum of
    1D second-difference matrices, the Kronecker product of 1D central
    differences for the mixed term, and 1D central differences for advection."""
    nx, ny = 7, 5
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    Dxx, Dxy, Dyy, ax, ay = 0.9, 0.3, 0.4, 0.25, -0.6
    op = O.make_operator(np.full((ny, nx), Dxx), np.full((ny, nx), Dxy), np.full((ny, nx), Dyy),
                         ax, ay, hx, hy, O.DIRICHLET)
    def second(n, h):
        return (np.diag(-2 * np.ones(n)) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1)) / h ** 2
    def central(n, h):
        return (np.diag(np.ones(n - 1), 1) - np.diag(np.ones(n - 1), -1)) / (2 * h)
    Ix, Iy = np.eye(nx), np.eye(ny)
    ref = (Dxx * np.kron(Iy, second(nx, hx)) + Dyy * np.kron(second(ny, hy), Ix)
           + 2 * Dxy * np.kron(central(ny, hy), central(nx, hx))
           + ax * np.kron(Iy, central(nx, hx)) + ay * np.kron(central(ny, hy), Ix))
    M = dense(op)
    assert np.max(np.abs(M - ref)) <= 1e-12 * np.max(np.abs(ref))


def _manufactured(bc):
    x, y = sp.symbols("x y")
    if bc == O.PERIODIC:
        u = sp.sin(2 * sp.pi * x) * sp.cos(4 * sp.pi * y) + sp.cos(2 * sp.pi * (x + y))
        Dxx = 1 + sp.Rational(1, 2) * sp.sin(2 * sp.pi * x) * sp.cos(2 * sp.pi * y)
        Dyy = sp.Rational(3, 4) + sp.Rational(1, 4) * sp.cos(2 * sp.pi * (x - y))
        Dxy = sp.Rational(3, 10) * sp.sin(2 * sp.pi * (x + 2 * y))
        ax = sp.Rational(1, 2) * sp.cos(2 * sp.pi * y)
        ay = -sp.Rational(1, 3) * sp.sin(2 * sp.pi * x)
    else:
        u = sp.sin(sp.pi * x) * sp.sin(2 * sp.pi * y) * sp.exp(x)
        Dxx = 1 + x * y
        Dyy = sp.Rational(1, 2) + x ** 2
        Dxy = sp.Rational(1, 5) * (x - y)
        ax = sp.Rational(1, 2) + y
        ay = -x
    Lu = (sp.diff(Dxx * sp.diff(u, x) + Dxy * sp.diff(u, y), x)
          + sp.diff(Dxy * sp.diff(u, x) + Dyy * sp.diff(u, y), y)
          + sp.diff(ax * u, x) + sp.diff(ay * u, y))
    f = lambda e: sp.lambdify((x, y), e, "numpy")
    return [f(e) for e in (u, Dxx, Dxy, Dyy, ax, ay, Lu)]


@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
def test_manufactured_solution_second_order(bc):
    """A u converges to the exact div(D grad u) + div(a u) at second order
    for smooth variable coefficients (computed symbolically)."""
    fu, fxx, fxy, fyy, fax, fay, fL = _manufactured(bc)
    errs = []
    for n in (32, 64, 128):
        X, Y, hx, hy = W.grid_2d(n, n, bc)
        bcast = lambda v: np.broadcast_to(np.asarray(v, dtype=float), X.shape)
        op = O.make_operator(bcast(fxx(X, Y)), bcast(fxy(X, Y)), bcast(fyy(X, Y)),
                             bcast(fax(X, Y)), bcast(fay(X, Y)), hx, hy, bc)
        e = O.apply(op, fu(X, Y)) - fL(X, Y)
        if bc == O.DIRICHLET:
            e = e[2:-2, 2:-2]  # the boundary face rule is first order locally
        errs.append(np.max(np.abs(e)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


def test_stencil_rows_reproduce_apply():
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(10, 7, seed=9, field_advection=True)
    for bc in (O.PERIODIC, O.DIRICHLET):
        op = O.make_operator(Dxx, Dxy, Dyy, ax, ay, 0.1, 0.13, bc)
        M = dense(op)
        ent = O.stencil_rows(op)
        # row sums of |entries| and diagonal agree with the dense matrix
        assert np.allclose(np.diag(M), ent[0].ravel(), rtol=1e-13, atol=0)
        assert np.allclose(np.abs(M).sum(axis=1), sum(np.abs(e) for e in ent).ravel(), rtol=1e-12)
