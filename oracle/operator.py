"""The spatial operator A = div(D grad(.)) + div(a .)  (Sec. 1 eq. 2; Sec. 2
definition of the matrix A below eq. 3).

The paper gives no spatial discretisation.  Reading: the conservative
second-order central nine-point form, with Dyx = Dxy (every tensor in the
paper is symmetric, eq. 6-7):

  (A u)_ij = [Fx_{i+1/2}(u_{i+1,j}-u_ij) - Fx_{i-1/2}(u_ij-u_{i-1,j})] / hx^2
           + [Fy_{j+1/2}(u_{i,j+1}-u_ij) - Fy_{j-1/2}(u_ij-u_{i,j-1})] / hy^2
           + [Dxy_{i+1,j}(u_{i+1,j+1}-u_{i+1,j-1})
              - Dxy_{i-1,j}(u_{i-1,j+1}-u_{i-1,j-1})] / (4 hx hy)      d/dx(Dxy du/dy)
           + [Dxy_{i,j+1}(u_{i+1,j+1}-u_{i-1,j+1})
              - Dxy_{i,j-1}(u_{i+1,j-1}-u_{i-1,j-1})] / (4 hx hy)      d/dy(Dxy du/dx)
           + [ax_{i+1,j} u_{i+1,j} - ax_{i-1,j} u_{i-1,j}] / (2 hx)    d/dx(ax u)
           + [ay_{i,j+1} u_{i,j+1} - ay_{i,j-1} u_{i,j-1}] / (2 hy)    d/dy(ay u)

with face values Fx_{i+1/2} = (Dxx_ij + Dxx_{i+1,j})/2, Fy_{j+1/2} =
(Dyy_ij + Dyy_{i,j+1})/2.

Reading of the advection sign: eq. 2 and the definition of A put +div(a u)
on the right-hand side, which is followed literally.

Boundaries: periodic wraps indices.  Dirichlet means u = 0 on the ghost ring
outside the interior nodes; a face that lies on the boundary takes the
interior node's coefficient (Fx_{-1/2} = Dxx_0j etc.).  Every other ghost
coefficient multiplies a zero ghost value and is never needed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

PERIODIC = 0
DIRICHLET = 1


@dataclass
class Operator:
    Dxx: np.ndarray
    Dxy: np.ndarray
    Dyy: np.ndarray
    ax: np.ndarray
    ay: np.ndarray
    hx: float
    hy: float
    bc: int

    @property
    def shape(self):
        return self.Dxx.shape


def make_operator(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc) -> Operator:
    """Fields are [ny][nx] float64; ax / ay may be scalars (constant)."""
    Dxx = np.asarray(Dxx, dtype=np.float64)
    shape = Dxx.shape
    f = lambda a: np.broadcast_to(np.asarray(a, dtype=np.float64), shape).copy()
    return Operator(f(Dxx), f(Dxy), f(Dyy), f(ax), f(ay), float(hx), float(hy), int(bc))


def _pad(a, bc, dirichlet_mode):
    if bc == PERIODIC:
        return np.pad(a, 1, mode="wrap")
    return np.pad(a, 1, mode=dirichlet_mode)


def apply(op: Operator, u: np.ndarray) -> np.ndarray:
    """y = A u for one grid function u[ny][nx] (see module docstring)."""
    hx, hy = op.hx, op.hy
    U = _pad(u, op.bc, "constant")          # ghost u = 0 for Dirichlet
    Dxx = _pad(op.Dxx, op.bc, "edge")       # boundary face -> interior value
    Dyy = _pad(op.Dyy, op.bc, "edge")
    Dxy = _pad(op.Dxy, op.bc, "constant")   # only multiplies zero ghosts
    ax = _pad(op.ax, op.bc, "constant")
    ay = _pad(op.ay, op.bc, "constant")

    # padded index [j+1, i+1] holds node (i, j); C = centre, E = i+1, ...
    C = (slice(1, -1), slice(1, -1))
    E = (slice(1, -1), slice(2, None))
    W = (slice(1, -1), slice(0, -2))
    N = (slice(2, None), slice(1, -1))
    S = (slice(0, -2), slice(1, -1))
    NE = (slice(2, None), slice(2, None))
    NW = (slice(2, None), slice(0, -2))
    SE = (slice(0, -2), slice(2, None))
    SW = (slice(0, -2), slice(0, -2))

    Fe = 0.5 * (Dxx[C] + Dxx[E])
    Fw = 0.5 * (Dxx[C] + Dxx[W])
    Fn = 0.5 * (Dyy[C] + Dyy[N])
    Fs = 0.5 * (Dyy[C] + Dyy[S])

    diff_x = (Fe * (U[E] - U[C]) - Fw * (U[C] - U[W])) / (hx * hx)
    diff_y = (Fn * (U[N] - U[C]) - Fs * (U[C] - U[S])) / (hy * hy)
    mixed_x = (Dxy[E] * (U[NE] - U[SE]) - Dxy[W] * (U[NW] - U[SW])) / (4.0 * hx * hy)
    mixed_y = (Dxy[N] * (U[NE] - U[NW]) - Dxy[S] * (U[SE] - U[SW])) / (4.0 * hx * hy)
    adv_x = (ax[E] * U[E] - ax[W] * U[W]) / (2.0 * hx)
    adv_y = (ay[N] * U[N] - ay[S] * U[S]) / (2.0 * hy)
    return diff_x + diff_y + mixed_x + mixed_y + adv_x + adv_y


def stencil_rows(op: Operator):
    """The nine matrix entries of every row of A, as arrays [ny][nx]:
    (centre, E, W, N, S, NE, NW, SE, SW); entries that would couple to a
    Dirichlet ghost node are returned as 0 (they are not matrix entries).
    Read off the formula in the module docstring."""
    hx, hy = op.hx, op.hy
    Dxx = _pad(op.Dxx, op.bc, "edge")
    Dyy = _pad(op.Dyy, op.bc, "edge")
    Dxy = _pad(op.Dxy, op.bc, "constant")
    ax = _pad(op.ax, op.bc, "constant")
    ay = _pad(op.ay, op.bc, "constant")
    C = (slice(1, -1), slice(1, -1))
    E = (slice(1, -1), slice(2, None))
    W = (slice(1, -1), slice(0, -2))
    N = (slice(2, None), slice(1, -1))
    S = (slice(0, -2), slice(1, -1))
    Fe = 0.5 * (Dxx[C] + Dxx[E]) / (hx * hx)
    Fw = 0.5 * (Dxx[C] + Dxx[W]) / (hx * hx)
    Fn = 0.5 * (Dyy[C] + Dyy[N]) / (hy * hy)
    Fs = 0.5 * (Dyy[C] + Dyy[S]) / (hy * hy)
    q = 1.0 / (4.0 * hx * hy)
    cen = -(Fe + Fw + Fn + Fs)
    e = Fe + ax[E] / (2.0 * hx)
    w = Fw - ax[W] / (2.0 * hx)
    n = Fn + ay[N] / (2.0 * hy)
    s = Fs - ay[S] / (2.0 * hy)
    ne = (Dxy[E] + Dxy[N]) * q
    nw = -(Dxy[W] + Dxy[N]) * q
    se = -(Dxy[E] + Dxy[S]) * q
    sw = (Dxy[W] + Dxy[S]) * q
    ent = [cen, e, w, n, s, ne, nw, se, sw]
    if op.bc == DIRICHLET:
        ny, nx = op.shape
        ii = np.arange(nx)[None, :]
        jj = np.arange(ny)[:, None]
        east = ii < nx - 1
        west = ii > 0
        north = jj < ny - 1
        south = jj > 0
        masks = [None, east, west, north, south, east & north, west & north,
                 east & south, west & south]
        ent = [x if m is None else np.where(m, x, 0.0) for x, m in zip(ent, masks)]
    return ent
