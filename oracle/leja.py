"""Polynomial interpolation of phi-functions at Leja points (Sec. 2).

The paper's recipe (Sec. 2, "Leja method" paragraph):
  * alpha < 0 approximates the eigenvalue of A of largest magnitude; the
    smallest is taken to be 0, so the spectrum is assumed to lie in [alpha, 0];
  * c = alpha / 2 and gamma = -alpha / 4 map Leja points xi in [-2, 2] onto
    that interval: z = c + gamma xi  (xi = -2 -> alpha, xi = 2 -> 0);
  * the function phi_l((c + gamma xi) dt) is interpolated at the Leja points
    in Newton form, its coefficients d_k being divided differences;
  * the interpolant applied to A is built up term by term:
        p_{m+1} = p_m + d_{m+1} y_{m+1},
        y_{m+1} = ((A - c I)/gamma - xi_m I) y_m,       y_0 = v, p_0 = d_0 v.

Readings of what the paper leaves open (all listed in the design notes):
  * Leja points: xi_0 = 2, then xi_k maximises prod_{j<k} |xi - xi_j| over
    [-2, 2]; ties (the first is at k = 3, +-2/sqrt 3) go to the smaller xi.
  * Stopping (tol is the accuracy asked of the result, as Sec. 3 uses it): the error
    of the degree-m interpolant is estimated by the norms of the last
    STOP_WINDOW Newton terms, and the sweep stops at the first m >= STOP_WINDOW
    with
        sum_{j = m - STOP_WINDOW + 1}^{m} || d_j y_j ||_2 <= tol * || p_m ||_2
    (FP64 Euclidean norms over the grid, summed oldest first).  The terms of
    a sweep over a wide interval rise and fall by orders of magnitude from one
    Leja point to the next, so a single small term says little about the
    truncation error; over a window of five the estimate bounds it on the
    paper's test problems.  v = 0 gives 0 with degree 0.
  * phi_0 over K > 1 substeps is the K-fold product of sweeps whose relative
    errors add up, so each of those sweeps uses tol / K.  (The phi_1 / phi_2
    substep recursion sums h p_j, whose errors are already relative to that
    sum, and keeps tol.)
  * Substepping: a sweep covers at most rho*h <= RHO_MAX (rho = |alpha|);
    a step dt is split into K = ceil(rho dt / RHO_MAX) equal substeps, and K
    is doubled if a sweep reaches the degree cap without converging.
  * phi_1 + phi_2 sums use the augmented matrix [[A, w2/h], [0, 0]] acting on
    [w1; 1] (the "exponential of an augmented matrix" of Sec. 2): its extra
    scalar component obeys s_{k+1} = (2 - xi_k) s_k, s_0 = 1.
"""
from __future__ import annotations

import math
import os
from functools import lru_cache

import numpy as np

from .phi import phi

MAX_DEGREE = 500          # most Newton terms in one sweep
STOP_WINDOW = 5           # Newton terms in the stopping estimate
RHO_MAX = 1600.0          # largest rho*h covered by one sweep
MAX_SUBSTEP_DOUBLINGS = 6
TIE_TOL = 1e-12


class NoConvergence(RuntimeError):
    pass


# --------------------------------------------------------------------------
# Leja points on [-2, 2]
# --------------------------------------------------------------------------
def _gap_maximisers(P: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Maximiser of f(x) = sum_j log|x - P_j| inside each open gap (lo, hi)
    between consecutive sorted points.  f is strictly concave on such a gap
    and f'(x) = sum_j 1/(x - P_j) falls from +inf to -inf, so the maximiser
    is the unique zero of f'; it is found by bisection to full precision."""
    lo = lo.copy()
    hi = hi.copy()
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        done = (mid <= lo) | (mid >= hi)
        if np.all(done):
            break
        fp = np.sum(1.0 / (mid[:, None] - P[None, :]), axis=1)
        up = fp > 0.0
        lo = np.where(done, lo, np.where(up, mid, lo))
        hi = np.where(done, hi, np.where(up, hi, mid))
    return 0.5 * (lo + hi)


TABLE_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "leja_points.txt")


def generate_leja_points(M: int, start=()) -> np.ndarray:
    """First M Leja points on [-2, 2] (greedy max-product sequence), continuing
    from an already generated prefix `start` if given."""
    pts = list(start) if len(start) else [2.0, -2.0, 0.0][:M]
    while len(pts) < M:
        P = np.array(pts)
        s = np.sort(P)
        x = _gap_maximisers(P, s[:-1], s[1:])
        f = np.sum(np.log(np.abs(x[:, None] - P[None, :])), axis=1)
        fmax = f.max()
        ties = f >= fmax - TIE_TOL * max(1.0, abs(fmax))
        pts.append(float(np.min(x[ties])))
    return np.array(pts[:M])


@lru_cache(maxsize=4)
def leja_points(M: int = MAX_DEGREE + 1) -> np.ndarray:
    """First M Leja points.  The sequence is read from the table that
    make_leja_table.py writes with generate_leja_points (exact hex floats);
    points beyond the table are generated."""
    pts = np.zeros(0)
    if os.path.exists(TABLE_FILE):
        with open(TABLE_FILE) as fh:
            vals = [float.fromhex(s.split()[0]) for s in fh
                    if s.strip() and not s.startswith("#")]
        pts = np.array(vals[:M])
    if len(pts) < M:
        pts = generate_leja_points(M, pts)
    pts.setflags(write=False)
    return pts


# --------------------------------------------------------------------------
# divided differences
# --------------------------------------------------------------------------
def divided_differences(x: np.ndarray, f: np.ndarray) -> np.ndarray:
    """Newton coefficients d_k = f[x_0, ..., x_k] by the triangular recurrence
    d_k <- (d_k - d_{k-1}) / (x_k - x_{k-j}), j = 1..n-1, in FP64 (Sec. 2:
    "determined using divided differences")."""
    d = np.array(f, dtype=np.float64)
    n = len(d)
    for j in range(1, n):
        d[j:] = (d[j:] - d[j - 1:-1]) / (x[j:] - x[:n - j])
    return d


def interval_map(alpha: float):
    """c = alpha/2, gamma = -alpha/4 (Sec. 2)."""
    return alpha / 2.0, -alpha / 4.0


def newton_coefficients(l: int, alpha: float, h: float, M: int = MAX_DEGREE + 1):
    """d_k for g(xi) = phi_l((c + gamma xi) h) on the first M Leja points."""
    xi = leja_points(M)
    c, gamma = interval_map(alpha)
    return divided_differences(xi, phi(l, (c + gamma * xi) * h))


def augmented_scalars(M: int = MAX_DEGREE + 1) -> np.ndarray:
    """s_0 = 1, s_{k+1} = (2 - xi_k) s_k: the extra component of the Newton
    vectors of the augmented matrix (its eigenvalue 0 sits at xi = 2)."""
    xi = leja_points(M)
    s = np.empty(M)
    s[0] = 1.0
    for k in range(M - 1):
        s[k + 1] = (2.0 - xi[k]) * s[k]
    return s


# --------------------------------------------------------------------------
# Newton sweep
# --------------------------------------------------------------------------
def newton_sweep(A, v, alpha, h, d, tol, max_degree=MAX_DEGREE, w2=None):
    """One interpolation sweep: returns (p, m, converged).

    p approximates g(A) v where g was interpolated with coefficients d (Sec. 2
    recurrence).  With w2 given, the matrix is the augmented
    [[A, w2/h], [0, 0]] acting on [v; 1] and p is the top block.
    m = number of applications of A (the polynomial degree); the sweep stops
    when the norms of the last STOP_WINDOW terms sum to at most tol ||p||."""
    xi = leja_points(max(len(d), max_degree + 1))
    s = augmented_scalars(max(len(d), max_degree + 1)) if w2 is not None else None
    c, gamma = interval_map(alpha)
    y = np.array(v, dtype=np.float64)
    p = d[0] * y
    if not np.any(y) and (w2 is None or not np.any(w2)):
        return np.zeros_like(y), 0, True
    recent = []  # norms of the last STOP_WINDOW terms, oldest first
    for k in range(max_degree):
        Ay = A(y)
        if s is not None and s[k] != 0.0:
            Ay = Ay + (s[k] / h) * w2
        y = (Ay - (c + gamma * xi[k]) * y) / gamma
        term = d[k + 1] * y
        p = p + term
        tn = np.linalg.norm(term)
        pn = np.linalg.norm(p)
        if not (np.isfinite(tn) and np.isfinite(pn)):
            return p, k + 1, False
        recent.append(tn)
        if len(recent) > STOP_WINDOW:
            recent.pop(0)
        if len(recent) == STOP_WINDOW:
            est = 0.0
            for t in recent:
                est += t
            if est <= tol * pn:
                return p, k + 1, True
    return p, max_degree, False


# --------------------------------------------------------------------------
# substep plan and phi drivers
# --------------------------------------------------------------------------
def substeps(alpha: float, dt: float, rho_max: float = RHO_MAX) -> int:
    """K = ceil(|alpha| dt / rho_max), at least 1."""
    return max(1, int(math.ceil(abs(alpha) * dt / rho_max)))


def _combo_fixed(A, w1, w2, dt, alpha, tol, max_degree, K, st):
    """K substeps of the recursion below; returns (y, all sweeps converged)."""
    h = dt / K
    d = newton_coefficients(1, alpha, h, max_degree + 1)
    y = np.zeros_like(w1)
    for j in range(K):
        f = w1 if w2 is None else w1 + (j * h / dt) * w2
        if j > 0:
            f = A(y) + f
            st["matvecs"] += 1
        w2h = None if w2 is None else (h / dt) * w2
        p, m, conv = newton_sweep(A, f, alpha, h, d, tol, max_degree, w2h)
        st["matvecs"] += m
        st["degrees"].append(m)
        if not conv:
            return y, False
        y = y + h * p
    return y, True


def phi_combo(A, w1, w2, dt, alpha, tol, max_degree=MAX_DEGREE, rho_max=RHO_MAX, stats=None):
    """y = dt [phi_1(A dt) w1 + phi_2(A dt) w2]  (w2 may be None).

    K substeps of h = dt/K integrate y' = A y + w1 + (tau/dt) w2, y(0) = 0,
    exactly (the forcing is linear in tau):
        y_{j+1} = y_j + h [phi_1(A h)(A y_j + w1 + (j h/dt) w2) + phi_2(A h)(h/dt) w2],
    each bracket being one augmented phi_1 sweep; y_K equals the target.
    alpha = 0 (zero operator) gives dt (w1 + w2/2) exactly."""
    st = stats if stats is not None else {}
    st.setdefault("matvecs", 0)
    st.setdefault("degrees", [])
    w1 = np.asarray(w1, dtype=np.float64)
    if alpha == 0.0:
        st["substeps"] = 0
        return dt * (w1 + 0.5 * w2) if w2 is not None else dt * w1
    K = substeps(alpha, dt, rho_max)
    for _ in range(MAX_SUBSTEP_DOUBLINGS + 1):
        y, ok = _combo_fixed(A, w1, w2, dt, alpha, tol, max_degree, K, st)
        if ok:
            st["substeps"] = K
            return y
        K *= 2
    raise NoConvergence("Leja sweep did not converge")


def phi_apply(A, l, dt, v, alpha, tol, max_degree=MAX_DEGREE, rho_max=RHO_MAX, stats=None):
    """phi_l(A dt) v for l in {0, 1, 2} (Sec. 2).

    One substep: the Newton interpolant of phi_l((c + gamma xi) dt).
    K > 1 substeps: phi_0 is applied K times with h = dt/K, each sweep with
    tol / K (their relative errors add); phi_1 and phi_2 come from the exact
    substep recursion of phi_combo, divided by dt (phi_1: w1 = v;  phi_2:
    w1 = 0, w2 = v)."""
    st = stats if stats is not None else {}
    st.setdefault("matvecs", 0)
    st.setdefault("degrees", [])
    v = np.asarray(v, dtype=np.float64)
    if alpha == 0.0:
        st["substeps"] = 0
        return v / math.factorial(l)
    K = substeps(alpha, dt, rho_max)
    for _ in range(MAX_SUBSTEP_DOUBLINGS + 1):
        if K == 1:
            d = newton_coefficients(l, alpha, dt, max_degree + 1)
            p, m, conv = newton_sweep(A, v, alpha, dt, d, tol, max_degree)
            st["matvecs"] += m
            st["degrees"].append(m)
            if conv:
                st["substeps"] = 1
                return p
        elif l == 0:
            h = dt / K
            d = newton_coefficients(0, alpha, h, max_degree + 1)
            y = v.copy()
            conv = True
            for _j in range(K):
                y, m, conv = newton_sweep(A, y, alpha, h, d, tol / K, max_degree)
                st["matvecs"] += m
                st["degrees"].append(m)
                if not conv:
                    break
            if conv:
                st["substeps"] = K
                return y
        else:
            w1, w2 = (v, None) if l == 1 else (np.zeros_like(v), v)
            y, conv = _combo_fixed(A, w1, w2, dt, alpha, tol, max_degree, K, st)
            if conv:
                st["substeps"] = K
                return y / dt
        K *= 2
    raise NoConvergence("Leja sweep did not converge")
