"""Coefficient-field statistics that feed the bound predictor.

Per node the symmetric tensor [[Dxx, Dxy], [Dxy, Dyy]] has eigenvalues
    k_par  = (Dxx + Dyy)/2 + sqrt(((Dxx - Dyy)/2)^2 + Dxy^2),
    k_perp = (Dxx + Dyy)/2 - sqrt(((Dxx - Dyy)/2)^2 + Dxy^2),
the diffusivities along and across the field (the decomposition behind the
paper's ring / spiral tensors, eq. 6-7), and |a| = sqrt(ax^2 + ay^2).

Feature vector (9 values):
  0 log10 max k_par     1 log10 mean k_par
  2 log10 max k_perp'   3 log10 mean k_perp'    (k_perp' = max(k_perp, 0) + 1e-30)
  4 max |a|             5 mean |a|
  6 log10 hx            7 log10 hy              8 log10 dt
"""
from __future__ import annotations

import math

import numpy as np

TINY = 1e-30


def node_eigen(Dxx, Dxy, Dyy):
    m = 0.5 * (Dxx + Dyy)
    r = np.sqrt((0.5 * (Dxx - Dyy)) ** 2 + Dxy ** 2)
    return m + r, m - r


def field_features(Dxx, Dxy, Dyy, ax, ay, hx, hy, dt):
    kpar, kperp = node_eigen(np.asarray(Dxx, np.float64), np.asarray(Dxy, np.float64),
                             np.asarray(Dyy, np.float64))
    kperp = np.maximum(kperp, 0.0) + TINY
    amag = np.hypot(np.broadcast_to(ax, kpar.shape), np.broadcast_to(ay, kpar.shape))
    return np.array([
        math.log10(max(float(kpar.max()), TINY)), math.log10(max(float(kpar.mean()), TINY)),
        math.log10(float(kperp.max())), math.log10(float(kperp.mean())),
        float(amag.max()), float(amag.mean()),
        math.log10(hx), math.log10(hy), math.log10(dt)])
