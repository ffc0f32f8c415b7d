"""Pins of the oracle's Leja interpolation (Sec. 2) against closed forms,
dense matrix functions (scipy.linalg.expm) and high-precision arithmetic."""
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import leja, phi
from oracle import operator as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [s.strip() for s in fh if s.strip() and not s.startswith("#")]


def test_phi_against_mpmath():
    mpmath.mp.dps = 50
    for z in [-1600.0, -40.0, -3.0, -1.0, -0.999, -0.5, -1e-3, -1e-9, 0.0, 1e-7, 0.3, 2.0]:
        zz = mpmath.mpf(z)
        e = [mpmath.exp(zz)]
        if z == 0.0:
            e += [mpmath.mpf(1), mpmath.mpf(1) / 2, mpmath.mpf(1) / 6]
        else:
            e.append((mpmath.exp(zz) - 1) / zz)
            e.append((mpmath.exp(zz) - 1 - zz) / zz ** 2)
            e.append((mpmath.exp(zz) - 1 - zz - zz ** 2 / 2) / zz ** 3)
        for l in range(4):
            got = float(phi.phi(l, z))
            assert abs(got - float(e[l])) <= 2e-15 * abs(float(e[l])) + 1e-300, (l, z)


def test_phi_recursion():
    z = np.linspace(-50, 5, 1001)
    z = z[z != 0]
    for l in range(3):
        lhs = phi.phi(l + 1, z)
        rhs = (phi.phi(l, z) - 1.0 / math.factorial(l)) / z
        big = np.abs(z) > 1
        assert np.allclose(lhs[big], rhs[big], rtol=1e-13)


def test_leja_first_points_closed_form():
    want = [float(s) for s in load_golden("leja_first_points.txt")]
    got = leja.leja_points(501)[:4]
    assert np.allclose(got, want, rtol=0, atol=4e-16)
    assert got[3] == pytest.approx(-2 / math.sqrt(3), abs=4e-16)


def test_leja_table_is_max_product_on_dense_grid():
    """Every stored point attains the maximum of prod |x - xi_j| over a
    4e5-point grid of [-2, 2] (up to the grid spacing)."""
    xi = leja.leja_points(501)
    grid = np.linspace(-2, 2, 400001)
    F = np.zeros_like(grid)
    for k in range(1, len(xi)):
        F += np.log(np.abs(grid - xi[k - 1]) + 1e-300)
        fk = np.sum(np.log(np.abs(xi[k] - xi[:k])))
        assert fk >= F.max() - 1e-9 * max(1.0, abs(F.max())), k
        # and it is a local maximiser of the product
        for dx in (-1e-9, 1e-9):
            if abs(xi[k] + dx) > 2.0:
                continue
            assert np.sum(np.log(np.abs(xi[k] + dx - xi[:k]))) <= fk + 1e-12, k
    assert np.all(np.abs(xi) <= 2.0)
    assert len(np.unique(xi)) == len(xi)


def test_leja_table_regenerates():
    xi = leja.leja_points(501)
    fresh = leja.generate_leja_points(60)
    assert np.array_equal(fresh, xi[:60])


def test_divided_differences_against_mpmath():
    mpmath.mp.dps = 60
    xi = leja.leja_points(501)
    for l, rho_h, n in [(1, 100.0, 60), (0, 25.0, 40), (2, 400.0, 90)]:
        d = leja.newton_coefficients(l, -rho_h, 1.0, n)
        xs = [mpmath.mpf(float(x)) for x in xi[:n]]
        def g(x):
            z = -rho_h / 2 + rho_h / 4 * x
            if z == 0:
                return mpmath.mpf(1) / math.factorial(l)
            e = mpmath.exp(z)
            return [e, (e - 1) / z, (e - 1 - z) / z ** 2][l]
        dd = [g(x) for x in xs]
        for j in range(1, n):
            for k in range(n - 1, j - 1, -1):
                dd[k] = (dd[k] - dd[k - 1]) / (xs[k] - xs[k - j])
        ref = np.array([float(v) for v in dd])
        # absolute error relative to the largest coefficient, per term
        assert np.max(np.abs(d - ref)) <= 1e-14 * np.max(np.abs(ref)), (l, rho_h)


@pytest.mark.parametrize("l", [0, 1, 2])
@pytest.mark.parametrize("rho_dt", [25.0, 100.0, 400.0, 1600.0])
def test_diagonal_operator_closed_form(l, rho_dt):
    """A diagonal with eigenvalues spread over [-rho dt, 0]: phi_l(A dt) v is
    phi_l(lambda dt) v elementwise; the Leja result is within a few tol."""
    lam = -np.linspace(0.0, 1.0, 3000) * rho_dt
    v = W.random_vector(3000, 7)
    st = {}
    p = leja.phi_apply(lambda x: lam * x, l, 1.0, v, -rho_dt, 1e-10, stats=st)
    ex = phi.phi(l, lam) * v
    assert np.linalg.norm(p - ex) <= 5e-10 * np.linalg.norm(ex), st
    assert st["substeps"] == 1
    # degree grows like sqrt(rho dt) (cost claim of polynomial methods)
    assert st["degrees"][0] < 6.0 * math.sqrt(rho_dt) + 10


@pytest.mark.parametrize("l", [0, 1, 2])
@pytest.mark.parametrize("rho_dt,rho_max", [(1600.0, 1600.0), (1600.0, 400.0), (3000.0, 500.0)])
def test_tolerance_is_the_accuracy_on_a_diagonal_operator(l, rho_dt, rho_max):
    """tol as the accuracy asked of the result (as Sec. 3 uses it): for tol = 1e-4 and
    1e-6, with one sweep and with K = 4 and 6 substeps (phi_0 chains K
    sweeps; phi_1 and phi_2 use the substep recursion), the error against
    the closed form phi_l(lambda dt) v stays within 10 tol, both for a vector
    spread over the whole spectrum and for one concentrated on its smooth end
    (where the Newton terms oscillate most).  A one-term stopping test fails
    this (up to 40 tol on the paper's Case I)."""
    lam = -np.linspace(0.0, 1.0, 3000) * rho_dt
    for v in (W.random_vector(3000, 7), np.exp(lam / (0.01 * rho_dt))):
        ex = phi.phi(l, lam) * v
        for tol in (1e-4, 1e-6):
            st = {}
            p = leja.phi_apply(lambda x: lam * x, l, 1.0, v, -rho_dt, tol, rho_max=rho_max, stats=st)
            assert st["substeps"] == math.ceil(rho_dt / rho_max)
            assert np.linalg.norm(p - ex) <= 10 * tol * np.linalg.norm(ex), (tol, st)


def test_stopping_window():
    """The sweep stops at the first degree m >= STOP_WINDOW whose last
    STOP_WINDOW term norms sum to at most tol ||p_m||: recomputed here from
    the unstopped term sequence of a diagonal operator."""
    lam = -np.linspace(0.0, 1.0, 2000) * 900.0
    v = W.random_vector(2000, 5)
    d = leja.newton_coefficients(1, -900.0, 1.0)
    xi = leja.leja_points()
    c, g = -450.0, 225.0
    y, p, tn, pn = v.copy(), d[0] * v, [], []
    for k in range(300):
        y = (lam * y - (c + g * xi[k]) * y) / g
        p = p + d[k + 1] * y
        tn.append(np.linalg.norm(d[k + 1] * y))
        pn.append(np.linalg.norm(p))
    for tol in (1e-3, 1e-6, 1e-9):
        want = next(m for m in range(leja.STOP_WINDOW, 301)
                    if sum(tn[m - leja.STOP_WINDOW:m]) <= tol * pn[m - 1])
        _, m, conv = leja.newton_sweep(lambda x: lam * x, v, -900.0, 1.0, d, tol)
        assert conv and m == want, (tol, m, want)


def small_op(bc=O.PERIODIC, n=(9, 7), seed=2, scale=1.0):
    nx, ny = n
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=seed, field_advection=True)
    hx = 1.0 / nx if bc == O.PERIODIC else 1.0 / (nx + 1)
    hy = 1.0 / ny if bc == O.PERIODIC else 1.0 / (ny + 1)
    return O.make_operator(scale * Dxx, scale * Dxy, scale * Dyy, ax, ay, hx, hy, bc)


def dense(op):
    ny, nx = op.shape
    n = nx * ny
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = O.apply(op, e.reshape(ny, nx)).ravel()
    return M


def phi_dense(M, l, v):
    """phi_l(M) v from the exponential of the block matrix
    [[M, v, 0], [0, 0, 1], [0, 0, 0]] (l = 1, 2) or expm(M) v (l = 0)."""
    n = M.shape[0]
    if l == 0:
        return sla.expm(M) @ v
    B = np.zeros((n + l, n + l))
    B[:n, :n] = M
    B[:n, n] = v
    for k in range(l - 1):
        B[n + k, n + k + 1] = 1.0
    return sla.expm(B)[:n, n + l - 1]


@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
@pytest.mark.parametrize("l", [0, 1, 2])
def test_small_grid_against_expm(bc, l):
    op = small_op(bc)
    M = dense(op)
    rho = np.max(np.abs(np.linalg.eigvals(M)))
    alpha = -1.1 * rho
    v = W.random_vector(op.shape, 3)
    for dt_mult, rho_max in [(60.0, leja.RHO_MAX), (60.0, 7.0), (300.0, leja.RHO_MAX)]:
        dt = dt_mult / rho
        st = {}
        p = leja.phi_apply(lambda x: O.apply(op, x), l, dt, v, alpha, 1e-12, rho_max=rho_max, stats=st)
        ref = phi_dense(M * dt, l, v.ravel()).reshape(op.shape)
        assert np.linalg.norm(p - ref) <= 1e-10 * np.linalg.norm(ref), (dt_mult, rho_max, st)


def test_augmented_combo_against_block_expm():
    """phi_1(A dt) w1 + phi_2(A dt) w2 through the augmented sweep equals the
    top block of expm([[A dt, w2, w1], [0, 0, 1], [0, 0, 0]])."""
    op = small_op(O.DIRICHLET, (8, 6), seed=4)
    M = dense(op)
    n = M.shape[0]
    rho = np.max(np.abs(np.linalg.eigvals(M)))
    w1 = W.random_vector(op.shape, 11)
    w2 = W.random_vector(op.shape, 12)
    for dt_mult, rho_max in [(40.0, leja.RHO_MAX), (40.0, 9.0), (250.0, 50.0)]:
        dt = dt_mult / rho
        B = np.zeros((n + 2, n + 2))
        B[:n, :n] = M * dt
        B[:n, n] = w2.ravel()
        B[:n, n + 1] = w1.ravel()
        B[n, n + 1] = 1.0
        ref = dt * sla.expm(B)[:n, n + 1].reshape(op.shape)
        st = {}
        y = leja.phi_combo(lambda x: O.apply(op, x), w1, w2, dt, -1.1 * rho, 1e-12,
                           rho_max=rho_max, stats=st)
        assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref), (dt_mult, st)


def test_substep_invariance():
    op = small_op(O.PERIODIC, (10, 10), seed=6)
    A = lambda x: O.apply(op, x)
    rho = np.max(np.abs(np.linalg.eigvals(dense(op))))
    w1 = W.random_vector(op.shape, 1)
    w2 = W.random_vector(op.shape, 2)
    dt = 200.0 / rho
    outs = []
    for K in (1, 2, 3, 5):
        st = {}
        outs.append(leja.phi_combo(A, w1, w2, dt, -1.1 * rho, 1e-12, rho_max=1.1 * rho * dt / K * 1.0000001, stats=st))
        assert st["substeps"] == K
    for o in outs[1:]:
        assert np.linalg.norm(o - outs[0]) <= 1e-10 * np.linalg.norm(outs[0])


def test_zero_vector_and_zero_operator():
    op = small_op()
    A = lambda x: O.apply(op, x)
    z = np.zeros(op.shape)
    st = {}
    p = leja.phi_apply(A, 1, 0.01, z, -100.0, 1e-10, stats=st)
    assert not np.any(p) and st["degrees"] == [0]
    v = W.random_vector(op.shape, 0)
    assert np.array_equal(leja.phi_apply(A, 2, 0.1, v, 0.0, 1e-10), v / 2)
    assert np.allclose(leja.phi_combo(A, v, 2 * v, 0.5, 0.0, 1e-10), 0.5 * (v + v))


def test_null_space_vector_converges_at_the_first_window():
    """A constant vector is in the periodic null space: every Newton term
    after the first vanishes (y_1 = A c / gamma = 0, up to rounding), so the
    sweep stops as soon as the stopping window is full, with
    phi_l(A dt) c = c / l!."""
    op = small_op()
    A = lambda x: O.apply(op, x)
    c = np.full(op.shape, 3.0)
    st = {}
    p = leja.phi_apply(A, 1, 0.05, c, -500.0, 1e-10, stats=st)
    assert st["degrees"] == [leja.STOP_WINDOW]
    assert np.allclose(p, c, rtol=1e-12)


def test_underestimated_bound_is_detected():
    """An interval far too small makes the Newton terms grow: the sweep must
    report non-convergence rather than return a wrong answer silently."""
    lam = -np.linspace(0.0, 1.0, 500) * 400.0
    v = W.random_vector(500, 3)
    p, m, conv = leja.newton_sweep(lambda x: lam * x, v, -40.0, 1.0,
                                   leja.newton_coefficients(1, -40.0, 1.0), 1e-10, 200)
    assert not conv and m <= 200
