"""Pins of the oracle's spectral bounds (Sec. 2: Gershgorin) and power
iteration, plus the counter-based generator and the MLP / feature helpers."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import bounds, features, mlp, rng
from oracle import operator as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(op):
    ny, nx = op.shape
    n = nx * ny
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = O.apply(op, e.reshape(ny, nx)).ravel()
    return M


def test_splitmix64_published_vector():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as fh:
        want = [int(s) for s in fh if s.strip() and not s.startswith("#")]
    assert [int(x) for x in rng.splitmix64(1234567, 5)] == want
    u = rng.uniform_pm1(42, 100000)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.01


@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
def test_gershgorin_against_dense_discs(bc):
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(9, 8, seed=1, field_advection=True)
    op = O.make_operator(Dxx, Dxy, Dyy, 3 * ax, 3 * ay, 0.1, 0.125, bc)
    M = dense(op)
    d = np.diag(M)
    want = np.min(d - (np.abs(M).sum(axis=1) - np.abs(d)))
    assert bounds.gershgorin(op) == pytest.approx(want, rel=1e-13)
    ev = np.linalg.eigvals(M)
    assert np.min(ev.real) >= want * (1 + 1e-12)


@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
def test_power_iteration_matches_largest_eigenvalue(bc):
    Dxx, Dxy, Dyy, _, _ = W.random_fields(14, 12, seed=2, advect=False)
    op = O.make_operator(Dxx, Dxy, Dyy, 0.0, 0.0, 1 / 14, 1 / 12, bc)
    M = dense(op)
    rho = np.max(np.abs(np.linalg.eigvalsh(M)))
    lam, its, conv = bounds.power_iteration(lambda x: O.apply(op, x), op.shape, 5, 50000, 1e-12)
    assert conv
    assert lam == pytest.approx(rho, rel=1e-6)
    alpha, _ = bounds.spectral_bound(op, 1, max_iter=50000, rtol=1e-12, seed=5)
    assert alpha == pytest.approx(-min(1.1 * rho, abs(bounds.gershgorin(op))), rel=1e-6)


def test_power_iteration_periodic_constant_closed_form():
    """Periodic constant coefficients: the exact spectral radius is the max of
    the von Neumann symbol."""
    w = W.c1_periodic_constant(n=32)
    op = O.make_operator(w.Dxx, w.Dxy, w.Dyy, 0.0, 0.0, w.hx, w.hy, w.bc)
    t = 2 * np.pi * np.arange(32) / 32
    TX, TY = np.meshgrid(t, t)
    Dxx, Dxy, Dyy = w.Dxx[0, 0], w.Dxy[0, 0], w.Dyy[0, 0]
    lam = (2 * Dxx * (np.cos(TX) - 1) / w.hx ** 2 + 2 * Dyy * (np.cos(TY) - 1) / w.hy ** 2
           - 2 * Dxy * np.sin(TX) * np.sin(TY) / (w.hx * w.hy))
    rho = np.max(np.abs(lam))
    est, its, conv = bounds.power_iteration(lambda x: O.apply(op, x), op.shape, 1, 100000, 1e-13)
    assert est == pytest.approx(rho, rel=1e-6)


def test_node_eigen_and_features():
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(7, 6, seed=4, field_advection=True)
    kp, kq = features.node_eigen(Dxx, Dxy, Dyy)
    for j in range(6):
        for i in range(7):
            ev = np.linalg.eigvalsh([[Dxx[j, i], Dxy[j, i]], [Dxy[j, i], Dyy[j, i]]])
            assert kq[j, i] == pytest.approx(ev[0], rel=1e-12, abs=1e-15)
            assert kp[j, i] == pytest.approx(ev[1], rel=1e-12)
    f = features.field_features(Dxx, Dxy, Dyy, ax, ay, 0.1, 0.2, 1e-3)
    assert f[0] == pytest.approx(math.log10(kp.max()))
    assert f[5] == pytest.approx(np.hypot(ax, ay).mean())
    assert f[8] == pytest.approx(-3.0)


def test_field_features_every_entry():
    """All nine statistics against a per-node loop over 2 x 2 eigvalsh and
    math.hypot, on fields built so that every entry differs from the others
    (max against mean, k_par against k_perp, |a| against its components, hx
    against hy), with one indefinite node whose negative k_perp is clipped to
    0 (plus 1e-30)."""
    ny, nx = 5, 8
    rng = np.random.default_rng(11)
    Dxx = rng.uniform(0.5, 3.0, (ny, nx))
    Dyy = rng.uniform(0.01, 0.2, (ny, nx))
    Dxy = rng.uniform(-0.05, 0.05, (ny, nx))
    Dxy[2, 3] = 2.0  # Dxx Dyy < Dxy^2 there: k_perp < 0
    ax = rng.uniform(-1.0, 1.0, (ny, nx))
    ay = rng.uniform(-3.0, 3.0, (ny, nx))
    hx, hy, dt = 0.02, 0.125, 3e-4
    kpar, kperp, amag = [], [], []
    for j in range(ny):
        for i in range(nx):
            lo, hi = np.linalg.eigvalsh([[Dxx[j, i], Dxy[j, i]], [Dxy[j, i], Dyy[j, i]]])
            kpar.append(hi)
            kperp.append(max(lo, 0.0) + 1e-30)
            amag.append(math.hypot(ax[j, i], ay[j, i]))
    assert min(kperp) == 1e-30
    want = [math.log10(max(kpar)), math.log10(sum(kpar) / len(kpar)),
            math.log10(max(kperp)), math.log10(sum(kperp) / len(kperp)),
            max(amag), sum(amag) / len(amag), math.log10(hx), math.log10(hy), math.log10(dt)]
    assert len(set(np.round(want, 6))) == 9
    got = features.field_features(Dxx, Dxy, Dyy, ax, ay, hx, hy, dt)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-13)
    # constant advection (scalars) broadcasts over the grid
    got = features.field_features(Dxx, Dxy, Dyy, 0.6, -0.8, hx, hy, dt)
    assert got[4] == pytest.approx(1.0, rel=1e-15) and got[5] == pytest.approx(1.0, rel=1e-15)


def test_mlp_gradient_finite_differences():
    W0 = mlp.init_params(3)
    X = np.random.default_rng(0).standard_normal((5, 9))
    T = np.random.default_rng(1).standard_normal((5, 3))
    Y, cache = mlp.forward(W0, X)
    L, dY = mlp.mse_loss(Y, T)
    g = mlp.backward(W0, cache, dY)
    idx = np.random.default_rng(2).choice(len(W0), 60, replace=False)
    idx = np.concatenate([idx, [0, 575, 576, 639, 640, len(W0) - 1]])
    for k in idx:
        e = 1e-6
        Wp = W0.copy(); Wp[k] += e
        Wm = W0.copy(); Wm[k] -= e
        fd = (mlp.mse_loss(mlp.forward(Wp, X)[0], T)[0] - mlp.mse_loss(mlp.forward(Wm, X)[0], T)[0]) / (2 * e)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def test_mlp_forward_structure_and_adam_first_step():
    assert mlp.n_params() == 9 * 64 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3
    # zero weights: output is the last bias
    W0 = np.zeros(mlp.n_params())
    W0[-3:] = [1.0, -2.0, 0.5]
    Y, _ = mlp.forward(W0, np.ones((4, 9)))
    assert np.array_equal(Y, np.tile([1.0, -2.0, 0.5], (4, 1)))
    # a single path: x0 -> tanh -> tanh -> tanh -> y0
    layers = mlp.unpack(np.zeros(mlp.n_params()))
    layers = [(l[0].copy(), l[1].copy()) for l in layers]
    for Wl, _ in layers:
        Wl[0, 0] = 1.0
    Y, _ = mlp.forward(mlp.pack(layers), np.full((1, 9), 0.7))
    assert Y[0, 0] == pytest.approx(math.tanh(math.tanh(math.tanh(0.7))), rel=1e-15)
    # Adam's first step is lr * g / (|g| + eps) against the gradient
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    Wn, m1, m2 = mlp.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(Wn, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
