"""Scalar phi-functions (Sec. 2): phi_0(z) = exp(z) and
phi_{l+1}(z) = (phi_l(z) - 1/l!) / z, so that
    phi_1(z) = (e^z - 1) / z,   phi_2(z) = (e^z - 1 - z) / z^2,
and phi_l(0) = 1/l!.

Reading (the paper is silent on evaluation near z = 0, where the quotient
form cancels): for |z| < 1 the Taylor series phi_l(z) = sum_k z^k/(k+l)!
is summed to 30 terms (remainder below 1e-30); elsewhere the quotient form
with expm1 is used.
"""
from __future__ import annotations

import math

import numpy as np


def _taylor(z, l, terms=30):
    out = np.zeros_like(z)
    zk = np.ones_like(z)
    for k in range(terms):
        out = out + zk / math.factorial(k + l)
        zk = zk * z
    return out


def phi(l: int, z):
    """phi_l(z) for real z (scalar or array), l in {0, 1, 2, 3}."""
    z = np.asarray(z, dtype=np.float64)
    if l == 0:
        return np.exp(z)
    small = np.abs(z) < 1.0
    zs = np.where(small, 0.0, z)  # avoid 0/0 in the masked branch
    if l == 1:
        big = np.expm1(zs) / np.where(small, 1.0, zs)
    elif l == 2:
        big = (np.expm1(zs) - zs) / np.where(small, 1.0, zs * zs)
    elif l == 3:
        big = (np.expm1(zs) - zs - 0.5 * zs * zs) / np.where(small, 1.0, zs ** 3)
    else:
        raise ValueError("l must be 0..3")
    return np.where(small, _taylor(z, l), big)
