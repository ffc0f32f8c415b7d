"""Oracle runs at the full sizes of the GPU tests, for worker processes.

Each function builds its seeded workload, runs the FP64 oracle
single-threaded (plain NumPy, no GPU) and returns plain arrays and numbers.
The GPU tests submit them to a process pool (spawned processes: nothing here
touches the GPU) so that the runs at 1024^2 .. 4096^2 proceed side by side;
test infrastructure only."""
import os
import sys
import time

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import bounds, integrators, leja  # noqa: E402
from oracle import operator as O  # noqa: E402


def _round32(a, s):
    """The field as FP32 storage holds it: the scaled value rounded to FP32,
    scaled back (the oracle then applies the same scale)."""
    return (np.asarray(a, dtype=np.float64) * s).astype(np.float32).astype(np.float64) / s


def counted(op, name, every=16):
    """x -> A x through the oracle's operator, printing a progress line every
    `every` applications (long runs report as they go)."""
    t0, n = time.time(), [0]

    def A(x):
        n[0] += 1
        if n[0] % every == 0:
            print("oracle %s: %d matvecs, %.0fs" % (name, n[0], time.time() - t0), flush=True)
            sys.stdout.flush()
        return O.apply(op, x)
    return A


def operator_of(w, fp32_fields=False):
    Dxx, Dxy, Dyy = w.Dxx, w.Dxy, w.Dyy
    if fp32_fields:
        Dxx = _round32(Dxx, 1.0 / (w.hx * w.hx))
        Dyy = _round32(Dyy, 1.0 / (w.hy * w.hy))
        Dxy = _round32(Dxy, 1.0 / (4.0 * w.hx * w.hy))
    return O.make_operator(Dxx, Dxy, Dyy, w.ax_field(), w.ay_field(), w.hx, w.hy, w.bc)


def midpoint_steps(name, n, steps, tol=None, fp32_fields=False):
    """u after `steps` exponential midpoint steps of workload `name` at n x n
    (Gershgorin interval of the oracle's operator), with the interval and
    the matvecs of each step."""
    w = {"roofline": W.roofline_shape, "c5": W.c5_learned_eval}[name](n=n, steps=steps)
    tol = w.tol if tol is None else tol
    op = operator_of(w, fp32_fields)
    A = counted(op, "%s-%d" % (name, n))
    alpha = bounds.gershgorin(op)
    u, mvs = w.u0.copy(), []
    for k in range(steps):
        st = {}
        u = integrators.exp_midpoint_step(A, u, w.stage_sources(k)[0], w.dt, alpha, tol, stats=st)
        mvs.append(st["matvecs"])
    return u, alpha, mvs


def quad2_steps(n, steps, tol=1e-10, fp32_fields=False):
    """u after `steps` two-stage steps of the stream-function quadrature
    workload (pulsed source, c = (1/3, 2/3)) at n x n, FP64 vectors."""
    w = W.c3_stream_function(n=n, steps=steps, tol=tol, storage=0)
    op = operator_of(w, fp32_fields)
    A = counted(op, "quad2-%d%s" % (n, "-fp32" if fp32_fields else ""))
    alpha = bounds.gershgorin(op)
    u, mvs = w.u0.copy(), []
    for k in range(steps):
        S1, S2 = w.stage_sources(k)
        st = {}
        u = integrators.exp_quad2_step(A, u, S1, S2, w.c1, w.c2, w.dt, alpha, tol, stats=st)
        mvs.append(st["matvecs"])
    return u, alpha, mvs


def phi1_sweep(n, tol=1e-10, fp32_fields=False):
    """phi_1(A dt) v of the stream-function quadrature workload's operator at
    n x n (v = its initial Gaussian plus a seeded perturbation), with the
    sweep's statistics."""
    w = W.c3_stream_function(n=n, steps=1, tol=tol, storage=0)
    op = operator_of(w, fp32_fields)
    alpha = bounds.gershgorin(op)
    v = w.u0 + 1e-3 * W.random_vector(w.u0.shape, 21)
    st = {}
    p = leja.phi_apply(counted(op, "phi1-%d%s" % (n, "-fp32" if fp32_fields else "")), 1, w.dt, v, alpha, tol,
                       stats=st)
    return p, alpha, st["matvecs"], st["substeps"]
