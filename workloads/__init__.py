"""Seeded synthetic inputs for the anisotropic diffusion workloads.

This module only *builds inputs*: grids, coefficient fields, initial data,
sources and step sizes.  It holds none of the integrator's arithmetic (no
operator, no phi-functions, no Leja interpolation) and is shared by the CPU
oracle tests and the GPU path as a plain input generator.

Problem statement (Sec. 1, eq. 2): u_t = div(D grad u) + div(a u) + S(x, y, t)
with a symmetric diffusion tensor D = [[Dxx, Dxy], [Dxy, Dyy]].

Field recipe used by every workload: a unit (or sub-unit) direction field b
and parallel / perpendicular diffusivities give
    D = k_par * b b^T + k_perp * (I - b b^T),
which is the form of the paper's ring and spiral tensors (eq. 6-7: there
D = v v^T, i.e. k_par = |v|^2 along v and k_perp = 0).

Grids (no grid is given in the paper):
  periodic  : cell-centred nodes x_i = x0 + (i + 1/2) h, h = L / n
  dirichlet : interior nodes     x_i = x0 + (i + 1) h,   h = L / (n + 1)
Arrays are row-major [ny][nx]; i runs along x and is contiguous.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

PERIODIC = 0
DIRICHLET = 1


# --------------------------------------------------------------------------
# grids
# --------------------------------------------------------------------------
def grid_1d(n: int, bc: int, lo: float = 0.0, hi: float = 1.0):
    """Node coordinates and spacing of one axis."""
    L = hi - lo
    if bc == PERIODIC:
        h = L / n
        x = lo + (np.arange(n) + 0.5) * h
    else:
        h = L / (n + 1)
        x = lo + (np.arange(n) + 1.0) * h
    return x, h


def grid_2d(nx: int, ny: int, bc: int, box=(0.0, 1.0, 0.0, 1.0)):
    x, hx = grid_1d(nx, bc, box[0], box[1])
    y, hy = grid_1d(ny, bc, box[2], box[3])
    X, Y = np.meshgrid(x, y, indexing="xy")  # [ny][nx]
    return X, Y, hx, hy


# --------------------------------------------------------------------------
# diffusion tensors
# --------------------------------------------------------------------------
def tensor_from_direction(bx, by, k_par, k_perp):
    """D = k_par b b^T + k_perp (I - b b^T); returns (Dxx, Dxy, Dyy)."""
    bx = np.asarray(bx, dtype=np.float64)
    by = np.asarray(by, dtype=np.float64)
    dk = k_par - k_perp
    Dxx = k_perp + dk * bx * bx
    Dyy = k_perp + dk * by * by
    Dxy = dk * bx * by
    return (np.ascontiguousarray(Dxx), np.ascontiguousarray(Dxy),
            np.ascontiguousarray(Dyy))


def circular_direction(X, Y, cx=0.5, cy=0.5):
    """b = (-(y - cy), x - cx) / r: field lines are circles about (cx, cy)."""
    dx = X - cx
    dy = Y - cy
    r = np.hypot(dx, dy)
    r = np.where(r == 0.0, 1.0, r)
    return -dy / r, dx / r


def stream_function_direction(X, Y, seed: int, n_modes: int = 32,
                              kmax: int = 8, eps_frac: float = 1e-3):
    """Direction field b = (d_y psi, -d_x psi)/sqrt(|grad psi|^2 + eps^2) of a
    seeded smooth periodic stream function
        psi = sum_m A_m sin(2 pi (kx_m x + ky_m y) + phi_m),
    integer wave vectors 1 <= |k| <= kmax drawn uniformly from that set,
    A_m ~ N(0,1)/|k|, phi_m ~ U(0, 2 pi).  eps = eps_frac * max |grad psi|
    regularises stagnation points (|b| < 1 there)."""
    rng = np.random.default_rng(seed)
    ks = [(kx, ky) for kx in range(-kmax, kmax + 1) for ky in range(-kmax, kmax + 1)
          if 1 <= math.hypot(kx, ky) <= kmax]
    idx = rng.integers(0, len(ks), size=n_modes)
    amp = rng.standard_normal(n_modes)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=n_modes)
    # X, Y are tensor-product grids: cos(a + b) = cos a cos b - sin a sin b
    # with a = 2 pi kx x + phi (along x) and b = 2 pi ky y (along y)
    x = X[0, :]
    y = Y[:, 0]
    gx = np.zeros_like(X)
    gy = np.zeros_like(X)
    for m in range(n_modes):
        kx, ky = ks[idx[m]]
        kn = math.hypot(kx, ky)
        A = amp[m] / kn
        a = 2.0 * math.pi * kx * x + phase[m]
        b = 2.0 * math.pi * ky * y
        c = (np.outer(np.cos(b), np.cos(a)) - np.outer(np.sin(b), np.sin(a))) * (2.0 * math.pi * A)
        gx += c * kx
        gy += c * ky
    gnorm = np.hypot(gx, gy)
    eps = eps_frac * float(gnorm.max())
    den = np.sqrt(gnorm * gnorm + eps * eps)
    return gy / den, -gx / den


def ring_tensor(X, Y):
    """Ring tensor of eq. 6: D = [[y^2, -xy], [-xy, x^2]]."""
    return (Y * Y, -X * Y, X * X)


def spiral_tensor(X, Y, which: int):
    """Spiral tensors of eq. 7: v = (x + s y, -x), D = v v^T with s = 1 (S1)
    or s = 4 (S2)."""
    s = 1.0 if which == 1 else 4.0
    vx = X + s * Y
    vy = -X
    return (vx * vx, vx * vy, vy * vy)


# --------------------------------------------------------------------------
# initial data and sources
# --------------------------------------------------------------------------
def gaussian(X, Y, cx, cy, sigma, periodic_box: Optional[float] = None):
    """exp(-|x - x0|^2 / (2 sigma^2)); minimum-image distance when periodic."""
    dx = X - cx
    dy = Y - cy
    if periodic_box is not None:
        L = periodic_box
        dx = dx - L * np.round(dx / L)
        dy = dy - L * np.round(dy / L)
    return np.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))


def seeded_centre(seed: int):
    """Centre x0 = 0.25 + 0.5 U(0,1)^2 from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    c = 0.25 + 0.5 * rng.uniform(0.0, 1.0, size=2)
    return float(c[0]), float(c[1])


def source_tis(X, Y):
    """Time-independent sources of eq. 8 (Case II)."""
    return (0.1 + 30.0 * np.exp(-((X + 0.6) ** 2 + (Y - 0.75) ** 2) / 2.5e-2)
            + 40.0 * np.exp(-((X - 0.75) ** 2 + (Y + 0.8) ** 2) / 3e-2))


def source_tds(X, Y, t):
    """Time-dependent sources S_A + S_B + S_C of eq. 9 (Cases III/IV)."""
    sa = 100.0 * np.exp(-((X - 0.25) ** 2 + (Y - 0.25) ** 2) / 1.5e-2) * math.exp(-10.0 * abs(t - 0.1))
    sb = 70.0 * np.exp(-((X - 0.4) ** 2 + (Y + 0.4) ** 2) / 2.5e-2) * math.exp(-5.0 * abs(t - 0.3))
    sc = 50.0 * np.exp(-((X + 0.6) ** 2 + (Y - 0.6) ** 2) / 1.5e-2) * math.exp(-7.5 * abs(t - 0.6))
    return sa + sb + sc


# --------------------------------------------------------------------------
# explicit step size
# --------------------------------------------------------------------------
def cfl_dt(Dxx, Dyy, hx, hy):
    """Explicit (forward Euler) step limit used to express step sizes:
    dt_CFL = 1 / max_nodes(2 Dxx / hx^2 + 2 Dyy / hy^2).
    The paper uses dt_CFL without defining it (Sec. 3); this reading is the
    forward-Euler limit of the constant-coefficient 5-point part."""
    return 1.0 / float(np.max(2.0 * Dxx / hx ** 2 + 2.0 * Dyy / hy ** 2))


# --------------------------------------------------------------------------
# workload container
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    hx: float
    hy: float
    bc: int
    Dxx: np.ndarray
    Dxy: np.ndarray
    Dyy: np.ndarray
    ax: Optional[np.ndarray]      # None -> constant ax_c
    ay: Optional[np.ndarray]
    ax_c: float
    ay_c: float
    u0: np.ndarray
    dt: float
    steps: int
    tol: float
    scheme: str                   # "midpoint" | "quad2" | "exp" (u <- phi_0(dt A) u, no source)
    c1: float = 0.5
    c2: float = 0.5
    source: Optional[Callable[[float], np.ndarray]] = None
    storage: int = 0
    extra: dict = field(default_factory=dict)

    def S(self, t: float) -> Optional[np.ndarray]:
        return None if self.source is None else self.source(t)

    def stage_sources(self, n: int):
        """Source arrays at the quadrature nodes of step n (t^n + c_i dt)."""
        t = n * self.dt
        if self.source is None:
            return (None, None)
        if self.scheme == "midpoint":
            return (self.source(t + self.c1 * self.dt), None)
        return (self.source(t + self.c1 * self.dt), self.source(t + self.c2 * self.dt))

    def ax_field(self):
        return self.ax if self.ax is not None else np.full((self.ny, self.nx), self.ax_c)

    def ay_field(self):
        return self.ay if self.ay is not None else np.full((self.ny, self.nx), self.ay_c)


def c1_periodic_constant(n: int = 64, seed: int = 0, steps: int = 10, cfl_mult: float = 50.0,
                         tol: float = 1e-10) -> Workload:
    """Constant anisotropic tensor on a periodic grid: b = (cos 30deg, sin 30deg),
    k_par = 1, k_perp = 0.01, a = (0.1, 0.05), Gaussian u0 (sigma 0.05), no
    source, exponential midpoint, dt = 50 dt_CFL."""
    X, Y, hx, hy = grid_2d(n, n, PERIODIC)
    th = math.radians(30.0)
    bx = np.full_like(X, math.cos(th))
    by = np.full_like(X, math.sin(th))
    Dxx, Dxy, Dyy = tensor_from_direction(bx, by, 1.0, 0.01)
    cx, cy = seeded_centre(seed)
    u0 = gaussian(X, Y, cx, cy, 0.05, periodic_box=1.0)
    dt = cfl_mult * cfl_dt(Dxx, Dyy, hx, hy)
    return Workload("periodic-constant-%d" % n, n, n, hx, hy, PERIODIC, Dxx, Dxy, Dyy,
                    None, None, 0.1, 0.05, u0, dt, steps, tol, "midpoint", 0.5, 0.5, None)


def c2_dirichlet_circular(n: int = 512, seed: int = 0, steps: int = 50, cfl_mult: float = 200.0,
                          tol: float = 1e-10, k_ratio: float = 1e3) -> Workload:
    """Circular field about the domain centre on a Dirichlet grid, k_par = 1,
    k_par/k_perp = 1e3, a = (0.2, 0), centred time-independent Gaussian
    source (amplitude 1, sigma 0.02), two-stage quadrature c = (1/3, 2/3),
    dt = 200 dt_CFL."""
    X, Y, hx, hy = grid_2d(n, n, DIRICHLET)
    bx, by = circular_direction(X, Y)
    Dxx, Dxy, Dyy = tensor_from_direction(bx, by, 1.0, 1.0 / k_ratio)
    cx, cy = seeded_centre(seed)
    u0 = gaussian(X, Y, cx, cy, 0.05)
    S = gaussian(X, Y, 0.5, 0.5, 0.02)
    dt = cfl_mult * cfl_dt(Dxx, Dyy, hx, hy)
    return Workload("dirichlet-circular-%d" % n, n, n, hx, hy, DIRICHLET, Dxx, Dxy, Dyy,
                    None, None, 0.2, 0.0, u0, dt, steps, tol, "quad2", 1.0 / 3.0, 2.0 / 3.0,
                    lambda t, S=S: S)


def c3_stream_function(n: int = 2048, seed: int = 0, steps: int = 20, cfl_mult: float = 100.0,
                       tol: float = 1e-10, k_ratio: float = 1e4, storage: int = 2,
                       scheme: str = "quad2") -> Workload:
    """Seeded stream-function field on a periodic grid, k_par = 1,
    k_par/k_perp = 1e4, a = (0.2, 0), pulsed Gaussian source
    S = (1 + sin(2 pi t / T_s)) G (sigma 0.02, seeded centre), T_s = 20 dt,
    two-stage quadrature (1/3, 2/3), dt = 100 dt_CFL."""
    X, Y, hx, hy = grid_2d(n, n, PERIODIC)
    bx, by = stream_function_direction(X, Y, seed)
    Dxx, Dxy, Dyy = tensor_from_direction(bx, by, 1.0, 1.0 / k_ratio)
    cx, cy = seeded_centre(seed)
    u0 = gaussian(X, Y, cx, cy, 0.05, periodic_box=1.0)
    G = gaussian(X, Y, 1.0 - cx, 1.0 - cy, 0.02, periodic_box=1.0)
    dt = cfl_mult * cfl_dt(Dxx, Dyy, hx, hy)
    Ts = 20.0 * dt
    src = lambda t, G=G, Ts=Ts: (1.0 + math.sin(2.0 * math.pi * t / Ts)) * G
    c1, c2 = (1.0 / 3.0, 2.0 / 3.0) if scheme == "quad2" else (0.5, 0.5)
    return Workload("periodic-stream-%d" % n, n, n, hx, hy, PERIODIC, Dxx, Dxy, Dyy,
                    None, None, 0.2, 0.0, u0, dt, steps, tol, scheme, c1, c2, src, storage)


def roofline_shape(n: int = 4096, seed: int = 0, steps: int = 1, tol: float = 1e-10) -> Workload:
    """The stream-function field at a size whose working set far exceeds the
    on-chip caches, FP64, exponential midpoint with the pulsed source."""
    w = c3_stream_function(n=n, seed=seed, steps=steps, tol=tol, storage=0, scheme="midpoint")
    w.name = "roofline-stream-%d" % n
    return w


# stream-function seeds of the learned predictor's training samples are the
# sample indices (learned_sample), 0 .. 9999 for the 10 000-sample set; the
# evaluation field takes a seed outside that range
C5_EVAL_SEED = 1_000_001


def c5_learned_eval(n: int = 4096, steps: int = 5, tol: float = 1e-8, seed: int = C5_EVAL_SEED) -> Workload:
    """Evaluation workload of the learned interval: the stream-function
    recipe (k_par = 1, k_par/k_perp = 1e4, a = (0.2, 0), pulsed source,
    dt = 100 dt_CFL) on an n x n periodic grid with a stream function no
    training sample used, FP32 fields, exponential midpoint, tol 1e-8."""
    w = c3_stream_function(n=n, seed=seed, steps=steps, tol=tol, storage=1, scheme="midpoint")
    w.name = "learned-eval-stream-%d" % n
    return w


# --------------------------------------------------------------------------
# the paper's own test problems (Sec. 3)
# --------------------------------------------------------------------------
PAPER_BOX = (-1.0, 1.0, -1.0, 1.0)
PAPER_CASES = ("I", "II", "III", "IV")
PAPER_END_TIMES = {"I": (0.75,), "II": (0.85,), "III": (0.10, 0.30), "IV": (0.10, 0.30)}


def paper_case(case: str, n: int = 256, dt_mult: Optional[float] = None, T: Optional[float] = None,
               scheme: Optional[str] = None, tol: float = 1e-10) -> Workload:
    """Cases I-IV of Sec. 3 on an n x n grid.

    I   ring tensor (eq. 6), no advection, no source: u(T) = exp(T A) u0,
        taken as one step over the whole interval (scheme "exp", phi_0);
    II  spiral 2 (eq. 7, s = 4), a = (1, 1), time-independent sources
        (eq. 8): the exponential midpoint rule is exact in time here;
    III spiral 1 (s = 1), a = (1, 1), time-dependent sources (eq. 9);
    IV  spiral 2, a = (1, 2), time-dependent sources (eq. 9).
    End times: I 0.75, II 0.85, III/IV 0.10 or 0.30.

    The paper gives no domain, grid, boundary or initial data.  Readings:
    [-1, 1]^2 (every source centre of eq. 8-9 lies inside it), zero
    Dirichlet boundary on interior nodes, the tensors exactly as printed
    (k_perp = 0), and one initial Gaussian of width 0.1 centred at
    (0.5, 0) for every case.  The step is dt_mult * dt_CFL, shortened so
    that a whole number of steps ends at T (default: one step for I,
    10^4 dt_CFL for II, 100 dt_CFL for III/IV); scheme "quad2" uses the
    Gauss nodes 1/2 -+ sqrt(3)/6 (eq. 5)."""
    if case not in PAPER_CASES:
        raise ValueError("case must be one of %s" % (PAPER_CASES,))
    X, Y, hx, hy = grid_2d(n, n, DIRICHLET, box=PAPER_BOX)
    if case == "I":
        Dxx, Dxy, Dyy = ring_tensor(X, Y)
        ax_c, ay_c, src = 0.0, 0.0, None
    elif case == "II":
        Dxx, Dxy, Dyy = spiral_tensor(X, Y, 2)
        ax_c, ay_c = 1.0, 1.0
        S = source_tis(X, Y)
        src = lambda t, S=S: S
    else:
        Dxx, Dxy, Dyy = spiral_tensor(X, Y, 1 if case == "III" else 2)
        ax_c, ay_c = (1.0, 1.0) if case == "III" else (1.0, 2.0)
        src = lambda t, X=X, Y=Y: source_tds(X, Y, t)
    if T is None:
        T = PAPER_END_TIMES[case][0]
    dcfl = cfl_dt(Dxx, Dyy, hx, hy)
    if dt_mult is None:
        steps = 1 if case == "I" else max(1, math.ceil(T / ((1e4 if case == "II" else 100.0) * dcfl)))
    else:
        steps = max(1, math.ceil(T / (dt_mult * dcfl)))
    dt = T / steps
    if scheme is None:
        scheme = "exp" if case == "I" else ("midpoint" if case == "II" else "quad2")
    if scheme == "quad2":
        c1, c2 = 0.5 - math.sqrt(3.0) / 6.0, 0.5 + math.sqrt(3.0) / 6.0
    else:
        c1 = c2 = 0.5
    u0 = gaussian(X, Y, 0.5, 0.0, 0.1)
    w = Workload("paper-case-%s-%d" % (case, n), n, n, hx, hy, DIRICHLET, Dxx, Dxy, Dyy,
                 None, None, ax_c, ay_c, u0, dt, steps, tol, scheme, c1, c2, src)
    w.extra.update(T=T, dt_cfl=dcfl, case=case)
    return w


BIN_SIZES = (128, 192, 256, 384, 512)


def c4_bins(nbins: int = 256, seed: int = 0, steps: int = 10, cfl_mult: float = 50.0,
            tol: float = 1e-10, sizes=BIN_SIZES, k_ratio: float = 1e3):
    """Momentum bins b = 0..nbins-1 with p_b = 10^(4 b/(nbins-1)),
    k_par = p_b^0.5, k_perp = k_par / k_ratio; grid sizes drawn independently
    per axis from `sizes` (numpy default_rng(seed)); Dirichlet; shared
    circular field; a = (0.2, 0); centred Gaussian source (sigma 0.02);
    FP64 exponential midpoint with a shared dt = 50 min_b dt_CFL,b."""
    rng = np.random.default_rng(seed)
    dims = rng.choice(np.array(sizes), size=(nbins, 2))
    bins = []
    for b in range(nbins):
        p = 10.0 ** (4.0 * b / max(nbins - 1, 1))
        kpar = p ** 0.5
        nx, ny = int(dims[b, 0]), int(dims[b, 1])
        X, Y, hx, hy = grid_2d(nx, ny, DIRICHLET)
        bx, by = circular_direction(X, Y)
        Dxx, Dxy, Dyy = tensor_from_direction(bx, by, kpar, kpar / k_ratio)
        cx, cy = seeded_centre(seed + 1 + b)
        u0 = gaussian(X, Y, cx, cy, 0.05)
        S = gaussian(X, Y, 0.5, 0.5, 0.02)
        bins.append(Workload("bin%03d-%dx%d" % (b, nx, ny), nx, ny, hx, hy, DIRICHLET,
                             Dxx, Dxy, Dyy, None, None, 0.2, 0.0, u0, 0.0, steps, tol,
                             "midpoint", 0.5, 0.5, lambda t, S=S: S,
                             extra={"p": p, "k_par": kpar}))
    dt = cfl_mult * min(cfl_dt(w.Dxx, w.Dyy, w.hx, w.hy) for w in bins)
    for w in bins:
        w.dt = dt
    return bins


def learned_sample(seed: int, sizes=BIN_SIZES):
    """One training sample for the bound predictor: stream-function field on a
    periodic grid with k_par ~ logU[0.1, 100], k_par/k_perp ~ logU[10, 1e4],
    |a| ~ U[0, 1] (random direction), dt ~ logU[10, 1000] dt_CFL."""
    rng = np.random.default_rng(10_000 + seed)
    nx = int(rng.choice(np.array(sizes)))
    ny = int(rng.choice(np.array(sizes)))
    kpar = 10.0 ** rng.uniform(-1.0, 2.0)
    ratio = 10.0 ** rng.uniform(1.0, 4.0)
    amag = rng.uniform(0.0, 1.0)
    ath = rng.uniform(0.0, 2.0 * math.pi)
    mult = 10.0 ** rng.uniform(1.0, 3.0)
    X, Y, hx, hy = grid_2d(nx, ny, PERIODIC)
    bx, by = stream_function_direction(X, Y, seed)
    Dxx, Dxy, Dyy = tensor_from_direction(bx, by, kpar, kpar / ratio)
    dt = mult * cfl_dt(Dxx, Dyy, hx, hy)
    return dict(nx=nx, ny=ny, hx=hx, hy=hy, bc=PERIODIC, Dxx=Dxx, Dxy=Dxy, Dyy=Dyy,
                ax_c=amag * math.cos(ath), ay_c=amag * math.sin(ath), dt=dt,
                k_par=kpar, k_perp=kpar / ratio)


def random_vector(shape, seed: int):
    """Seeded standard-normal vector (test input)."""
    return np.random.default_rng(seed).standard_normal(shape)


def random_fields(nx: int, ny: int, seed: int, advect: bool = True, field_advection: bool = False):
    """Smooth random positive-definite coefficient fields for operator tests."""
    rng = np.random.default_rng(seed)
    X, Y, hx, hy = grid_2d(nx, ny, PERIODIC)
    th = 2 * math.pi * (X + 0.3 * np.sin(2 * math.pi * Y)) + rng.uniform(0, 6.28)
    kpar = 1.0 + 0.5 * np.sin(2 * math.pi * X) * np.cos(2 * math.pi * Y) + rng.uniform(0, 0.2)
    kperp = 0.05 + 0.02 * np.cos(2 * math.pi * (X + Y))
    Dxx, Dxy, Dyy = tensor_from_direction(np.cos(th), np.sin(th), kpar, kperp)
    if field_advection:
        ax = 0.3 * np.cos(2 * math.pi * Y)
        ay = 0.2 * np.sin(2 * math.pi * X)
        return Dxx, Dxy, Dyy, ax, ay
    c = (0.3, -0.2) if advect else (0.0, 0.0)
    return Dxx, Dxy, Dyy, c[0], c[1]
