"""Spectral bounds for the Leja interval (Sec. 2).

Gershgorin (Sec. 2 names it): every eigenvalue of A lies in a union of row
discs, so the leftmost disc edge
    alpha_G = min_rows ( A_ii - sum_{j != i} |A_ij| )
bounds the real parts from below.  Reading: row discs (the paper does not say
rows or columns), advection entries included.

Power iteration (not in the paper; a tighter estimate of the magnitude of
the eigenvalue of largest modulus):
    v_0 = splitmix64 uniform(-1, 1) vector, normalised;
    w = A v, lambda_k = ||w||, v <- w / lambda_k,
    stop when |lambda_k - lambda_{k-1}| <= rtol * lambda_k or at max_iter.
Reading: alpha = -min(SAFETY * lambda, |alpha_G|) with SAFETY = 1.1, so the
interval never exceeds the rigorous Gershgorin one.
"""
from __future__ import annotations

import numpy as np

from .operator import apply, stencil_rows
from .rng import uniform_pm1

SAFETY = 1.1


def gershgorin(op) -> float:
    ent = stencil_rows(op)
    radius = sum(np.abs(e) for e in ent[1:])
    return float(np.min(ent[0] - radius))


def power_iteration(A, shape, seed: int, max_iter: int, rtol: float):
    """Returns (lambda, iterations, converged)."""
    n = int(np.prod(shape))
    v = uniform_pm1(seed, n).reshape(shape)
    v = v / np.linalg.norm(v)
    lam_prev = 0.0
    lam = 0.0
    for it in range(1, max_iter + 1):
        w = A(v)
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            return 0.0, it, True
        v = w / lam
        if abs(lam - lam_prev) <= rtol * lam:
            return lam, it, True
        lam_prev = lam
    return lam, max_iter, False


def spectral_bound(op, method: int, max_iter: int = 2000, rtol: float = 1e-3, seed: int = 0):
    """method 0: alpha_G.  method 1: -min(SAFETY * lambda_power, |alpha_G|).
    Returns (alpha, iterations)."""
    ag = gershgorin(op)
    if method == 0:
        return ag, 0
    lam, its, _ = power_iteration(lambda x: apply(op, x), op.shape, seed, max_iter, rtol)
    return -min(SAFETY * lam, abs(ag)), its
