#!/usr/bin/env python3
"""Benchmark of the Leja exponential integrator on one MI355X.

Headline workload (one "step" = one pass of the hot path: the stage vector
w = A u + S, the Newton-Leja sweep of phi_1 with its fused norm reductions
and stopping decisions, and the update u += dt p): the 4096 x 4096 periodic
stream-function field (32 seeded Fourier modes, wavenumber <= 8), k_par = 1,
k_par/k_perp = 1e4, a = (0.2, 0), pulsed Gaussian source
S = (1 + sin(2 pi t / T_s)) G, exponential midpoint rule, dt = 100 dt_CFL,
tol 1e-10, FP64 -- the grid whose working set (~1 GB per Newton term) is far
beyond L2 and the 256 MB Infinity Cache.  Operator setup, the Gershgorin
bound and the source arrays of every step are on the device before timing.

Prints one JSON line.  `value` = time steps per second on one GPU.
`roofline` = the dominant kernel, the three-term Newton-Leja launch
(leja3s_kernel: input rows staged in LDS): 56 B per point and Newton term
(read y, three tensor fields and p, write y and p, FP64) times the terms of
a launch, over the launch's average duration from HIP events on its own
dispatches, against 8 TB/s; `traffic` = the HBM bytes per launch measured by
rocprofv3 counters (profiles/).  `cpu_baseline` = the FP64 NumPy oracle,
single-threaded, on a bounded sample of the same workload.  Extra legs: the
512^2 two-stage quadrature workload, one-, two- and three-term kernels at
4096^2, four terms per launch at 640^2, the 256-bin momentum workload
(chosen vs plain), the paper's Cases I-IV.
"""
import os

for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import argparse  # noqa: E402
import json  # noqa: E402
import math  # noqa: E402
import sys  # noqa: E402
import time  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "stencil GB/s (%HBM peak), Leja steps/s; chosen vs plain at fixed rel. error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dev_tensor(a):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def make_op(w, storage=None):
    import paper_2307_12276_amd as A
    st = w.storage if storage is None else storage
    return A.Op(dev_tensor(w.Dxx), dev_tensor(w.Dxy), dev_tensor(w.Dyy), w.hx, w.hy, w.bc, st,
                ax_c=w.ax_c, ay_c=w.ay_c)


def gpu_step(op, w, u, n, srcs):
    S1, S2 = srcs(n)
    if w.scheme == "midpoint":
        return op.midpoint_step(u, S1, w.dt, w.tol)
    return op.quad2_step(u, S1, S2, w.c1, w.c2, w.dt, w.tol)


def device_sources(w):
    """Source arrays at the quadrature nodes, moved to the device once per
    distinct array (the time-independent source is one array)."""
    cache = {}

    def get(a):
        if a is None:
            return None
        k = id(a)
        if k not in cache:
            cache[k] = (a, dev_tensor(a))
        return cache[k][1]

    def srcs(n):
        S1, S2 = w.stage_sources(n)
        return get(S1), get(S2)
    return srcs


KERNEL_SOURCES = ("device.h", "internal.h", "stencil.hip", "tile.h", "staged.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "leja3s_kernel_stream4096_traffic.txt")
TRAFFIC_KEY = "traffic_bytes_per_launch_stream4096"
BYTES_PER_TERM_FP64 = 56.0  # read y, Dxx, Dxy, Dyy, p; write y, p (FP64, constant advection)


def sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2307_12276_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record():
    """key: value lines of the committed counter summary, or None."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        return kv
    except OSError:
        return None


def measured_traffic():
    """HBM bytes per three-term Newton-Leja launch of the 4096^2 workload from
    the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None when the
    kernel sources have changed since those counters were taken."""
    kv = traffic_record()
    try:
        if kv is None or sources_sha256() != kv.get("kernel_sources_sha256"):
            return None
        return float(kv[TRAFFIC_KEY])
    except (OSError, KeyError, ValueError):
        return None


def kernel_roofline(op_ms, launches, nbytes):
    avg_ms = op_ms / max(launches, 1)
    per_launch = nbytes / max(launches, 1)
    achieved = per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    return avg_ms, per_launch, achieved


KIND_KERNELS = {"two": "leja2s_kernel (two Newton terms per launch, input rows staged in LDS, non-temporal "
                        "hints on the vectors read or written once)",
                "three": "leja3s_kernel (three Newton terms per launch, input rows staged in LDS, non-temporal "
                         "hints on the vectors read or written once)",
                "four": "leja4_kernel (four Newton terms per launch)"}

LEG_KERNELS = {0: ("one-term", "leja_kernel"),
               1: ("three-term (the default)", "leja3s_kernel (input rows staged in LDS) + leja_kernel (first term)"),
               2: ("two-term", "leja2s_kernel (input rows staged in LDS) + leja_kernel (first term)"),
               3: ("two-term, register frames", "leja2_kernel + leja_kernel (first term)"),
}


def run_roofline_leg(w, storage, mode=1):
    """Midpoint steps of the stream-function field at n x n (two warm-up
    steps, three timed): the Newton-Leja kernels' dispatch-timed bandwidth on
    a working set far beyond the caches, with one term per launch (mode 0),
    the library's choice at this size (mode 1: three terms per launch, input
    rows staged in LDS), two with staged rows (mode 2) or two with register
    frames (mode 3)."""
    import torch
    import paper_2307_12276_amd as A
    n = w.nx
    op = make_op(w, storage)
    op.set_term_fusion(mode)
    op.spectral_bound(A.BOUND_GERSHGORIN)
    u = dev_tensor(w.u0)
    srcs = device_sources(w)
    for k in range(2):  # warm-up (plan, predicted degree, first touch of every sweep buffer)
        gpu_step(op, w, u, k, srcs)
    torch.cuda.synchronize()
    op.profile(True)
    t0 = time.perf_counter()
    timed = 3
    for k in range(2, 2 + timed):
        st = gpu_step(op, w, u, k, srcs)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / timed
    ms, launches, nbytes = op.profile_read()
    op.profile(False)
    avg_ms, per_launch, achieved = kernel_roofline(ms, launches, nbytes)
    terms = st["matvecs"] - 1  # the stage vector's matrix application is not a Newton term
    res = {"workload": w.name, "storage": ["fp64", "fp32-fields", "fp32-fields+y"][storage],
           "launches_of": LEG_KERNELS[mode][0],
           "nx": n, "ny": n, "kernel": LEG_KERNELS[mode][1],
           "launches": launches, "bytes_per_launch": per_launch, "avg_kernel_us": avg_ms * 1e3,
           "us_per_term": ms * 1e3 / (timed * max(terms + 1, 1)),
           "achieved_GBs": achieved, "frac_of_8TBs": achieved / HBM_PEAK_GBS,
           "matvecs_per_step": st["matvecs"], "step_ms": wall * 1e3}
    del op
    torch.cuda.empty_cache()
    return res


def four_term_leg(n=640, steps=30):
    """The C2-type two-stage quadrature on an n x n Dirichlet circular-field
    grid (within the four-term default range), with two Newton terms per
    launch (register frames) and with four: steps/s and the average
    Newton-Leja launch from HIP events on a second, event-timed pass."""
    import torch
    import paper_2307_12276_amd as A
    import workloads as W
    w = W.c2_dirichlet_circular(n=n, steps=steps + 3)
    res = {"workload": "dirichlet-circular-%d: the 512^2 workload's recipe on a %dx%d grid" % (n, n, n),
           "steps": steps}
    for mode, key in ((3, "two_terms"), (4, "four_terms")):
        op = make_op(w, A.STORAGE_FP64)
        op.spectral_bound(A.BOUND_GERSHGORIN)
        op.set_term_fusion(mode)
        srcs = device_sources(w)
        u = dev_tensor(w.u0)
        for k in range(3):
            gpu_step(op, w, u, k, srcs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mv = 0
        for k in range(3, 3 + steps):
            mv += gpu_step(op, w, u, k, srcs)["matvecs"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        u = dev_tensor(w.u0)
        op.profile(True)
        for k in range(3, 3 + steps):
            gpu_step(op, w, u, k, srcs)
        torch.cuda.synchronize()
        ms, nl, _ = op.profile_read()
        op.profile(False)
        res[key] = {"steps_per_s": steps / el, "matvecs_per_step": mv / steps, "avg_launch_us": 1e3 * ms / nl,
                    "launches": nl}
        del op
    res["speedup_four_vs_two"] = res["four_terms"]["steps_per_s"] / res["two_terms"]["steps_per_s"]
    log("four-term leg %d^2: two terms %.0f steps/s (%.1f us/launch), four terms %.0f steps/s (%.1f us/launch), "
        "%.2fx" % (n, res["two_terms"]["steps_per_s"], res["two_terms"]["avg_launch_us"],
                   res["four_terms"]["steps_per_s"], res["four_terms"]["avg_launch_us"], res["speedup_four_vs_two"]))
    return res


def paper_cases_leg(n=256, tol=1e-10):
    """The paper's test problems (Sec. 3, Cases I-IV; workloads.paper_case)
    at n x n, FP64, each with its default step (I: one phi_0 step over the
    whole interval; II: steps of 1e4 dt_CFL; III/IV: exponential Gauss
    quadrature, steps of 100 dt_CFL, T = 0.1), the GPU's own Gershgorin
    bound: GPU time to T with the source arrays already on the device.
    Accuracy on these problems is checked in tests/test_gpu_paper_cases.py."""
    import torch
    import paper_2307_12276_amd as A
    import workloads as W
    res = []
    for case in W.PAPER_CASES:
        w = W.paper_case(case, n, tol=tol)
        op = make_op(w, A.STORAGE_FP64)
        op.spectral_bound(A.BOUND_GERSHGORIN)
        u = dev_tensor(w.u0)
        out = torch.empty_like(u)
        S = [] if w.scheme == "exp" else [[None if a is None else dev_tensor(a) for a in w.stage_sources(k)]
                                          for k in range(w.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mv = 0
        for k in range(w.steps):
            if w.scheme == "exp":
                st = op.leja_phi(0, w.dt, u, out, tol)
                u, out = out, u
            elif w.scheme == "midpoint":
                st = op.midpoint_step(u, S[k][0], w.dt, tol)
            else:
                st = op.quad2_step(u, S[k][0], S[k][1], w.c1, w.c2, w.dt, tol)
            mv += st["matvecs"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res.append({"case": case, "n": n, "scheme": {"exp": "phi_0 (one step)", "midpoint": "exp. midpoint",
                                                     "quad2": "exp. Gauss"}[w.scheme],
                    "T": w.extra["T"], "steps": w.steps, "dt_over_dt_cfl": w.dt / w.extra["dt_cfl"],
                    "tol": tol, "matvecs": mv, "seconds": el, "matvecs_per_s": mv / el,
                    "us_per_matvec": 1e6 * el / max(mv, 1)})
        log("paper case %s (%d^2, %s): %d steps, %d matvecs in %.3fs (%.2f us per matvec)" % (
            case, n, res[-1]["scheme"], w.steps, mv, el, res[-1]["us_per_matvec"]))
        del op, S
        torch.cuda.empty_cache()
    return res


def chosen_vs_plain(steps=10, tol=1e-9):
    """Momentum-bin workload (256 bins, grids from {128,...,512}^2, k_par =
    p^0.5, shared circular field, midpoint, shared dt).
    plain  = per-bin FP64 operators, power-iteration interval per bin,
             per-bin exponential midpoint steps;
    chosen = FP32 fields, learned interval per bin (field statistics + MLP
             + Gershgorin cap, power-iteration fallback), all bins advanced by
             the batched kernels, every launch covering all bins (eager;
             the captured-hipGraph replay of the same step is timed too).
    Both at the same tolerance; reported: steps/s of the steps, time to
    solution including the interval estimation, and the relative difference
    of the chosen result from the plain FP64 result (max over bins)."""
    import numpy as np
    import torch
    import paper_2307_12276_amd as A
    from paper_2307_12276_amd import learned
    import workloads as W
    t0 = time.time()
    bins = W.c4_bins(steps=steps)
    log("chosen-vs-plain: 256 bins built in %.1fs (sum N = %.1fM)" % (time.time() - t0, sum(b.nx * b.ny for b in bins) / 1e6))
    dt = bins[0].dt
    S = [dev_tensor(b.S(0)) for b in bins]
    res = {"workload": "256 momentum bins, grids {128..512}^2, k_par=p^0.5, p=10^(4b/255), midpoint, "
                       "dt=50 min dt_CFL, %d steps" % steps, "tol": tol}
    # plain
    ops_p = [make_op(b, A.STORAGE_FP64) for b in bins]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pits = 0
    for op in ops_p:
        _, it = op.spectral_bound(A.BOUND_POWER, max_iter=2000, rtol=1e-3, seed=1)
        pits += it
    torch.cuda.synchronize()
    t_bound_p = time.perf_counter() - t0
    up = [dev_tensor(b.u0) for b in bins]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mv_p = 0
    for n in range(steps):
        for op, u, s in zip(ops_p, up, S):
            mv_p += op.midpoint_step(u, s, dt, tol)["matvecs"]
    torch.cuda.synchronize()
    t_steps_p = time.perf_counter() - t0
    # chosen
    ops_c = [make_op(b, A.STORAGE_FP32_FIELDS) for b in bins]
    Wd = torch.from_numpy(learned.load()).cuda()
    batch = A.Batch(ops_c)
    scratch = torch.empty(72 * len(ops_c), dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.learned_bound(dt, Wd, scratch)
    torch.cuda.synchronize()
    t_bound_c = time.perf_counter() - t0
    uc = [dev_tensor(b.u0) for b in bins]
    best_rows, _ = batch.autotune(uc, S, dt, tol, candidates=(8, 16, 32, 64))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mv_c = 0
    fb = 0
    batch.bind(uc, S)
    for n in range(steps):
        st = batch.midpoint_step(None, None, dt, tol, use_graph=False).array
        mv_c += int(st["matvecs"].sum())
        fb += int(st["fallback"].sum())
    torch.cuda.synchronize()
    t_steps_c = time.perf_counter() - t0
    # the same steps replayed as a captured hipGraph (same results; slower
    # to launch on this runtime), from a copy of the state
    ug = [dev_tensor(b.u0) for b in bins]
    batch.bind(ug, S)
    batch.midpoint_step(None, None, dt, tol, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n in range(steps):
        batch.midpoint_step(None, None, dt, tol, use_graph=True)
    torch.cuda.synchronize()
    t_steps_g = time.perf_counter() - t0
    diff = max(float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)) for a, b in zip(uc, up))
    res.update({
        "plain": {"steps_per_s": steps / t_steps_p, "bound_s": t_bound_p, "power_iterations": pits,
                  "time_to_solution_s": t_bound_p + t_steps_p, "matvecs": mv_p},
        "chosen": {"steps_per_s": steps / t_steps_c, "bound_s": t_bound_c, "tile_rows": best_rows,
                   "time_to_solution_s": t_bound_c + t_steps_c, "matvecs": mv_c, "fallbacks": fb,
                   "launch": "eager (the step's launches enqueued one by one)",
                   "graph_steps_per_s": steps / t_steps_g},
        "speedup_steps": t_steps_p / t_steps_c,
        "speedup_time_to_solution": (t_bound_p + t_steps_p) / (t_bound_c + t_steps_c),
        "max_rel_diff_chosen_vs_plain_fp64": diff})
    log("chosen-vs-plain: plain %.2f steps/s (bound %.2fs), chosen %.2f steps/s (bound %.3fs), "
        "speedup %.1fx steps, %.1fx time-to-solution, max rel diff %.2e"
        % (res["plain"]["steps_per_s"], t_bound_p, res["chosen"]["steps_per_s"], t_bound_c,
           res["speedup_steps"], res["speedup_time_to_solution"], diff))
    del batch, ops_c, ops_p
    torch.cuda.empty_cache()
    return res


def profile_leja(n, mode=1, fp32=False):
    """One phi_1 sweep on the n x n stream-function field (profiler driver);
    mode as for adl_op_set_term_fusion; fp32: fields stored in FP32."""
    import torch
    import paper_2307_12276_amd as A
    import workloads as W
    w = W.roofline_shape(n=n)
    op = make_op(w, A.STORAGE_FP32_FIELDS if fp32 else A.STORAGE_FP64)
    op.set_term_fusion(mode)
    op.spectral_bound(A.BOUND_GERSHGORIN)
    v = dev_tensor(w.u0)
    out = torch.empty_like(v)
    st = op.leja_phi(1, w.dt, v, out, w.tol)
    torch.cuda.synchronize()
    print(json.dumps({"profile_leja": n, "terms": st["matvecs"]}), flush=True)


def profile_c2(steps=5):
    """A few steps of the 512^2 Dirichlet two-stage quadrature workload
    alone (four Newton terms per launch), for rocprofv3."""
    import torch
    import paper_2307_12276_amd as A
    import workloads as W
    w = W.c2_dirichlet_circular(n=512, steps=steps)
    op = make_op(w, A.STORAGE_FP64)
    op.spectral_bound(A.BOUND_GERSHGORIN)
    u = dev_tensor(w.u0)
    srcs = device_sources(w)
    mv = 0
    for n in range(steps):
        mv += gpu_step(op, w, u, n, srcs)["matvecs"]
    torch.cuda.synchronize()
    print(json.dumps({"profile_c2": steps, "matvecs": mv}), flush=True)


def profile_bins(steps=4, tile_rows=16, tol=1e-9):
    """The chosen form of the 256-bin momentum workload alone (FP32 fields,
    learned interval, eager launches of each batched midpoint step) for a
    few steps, for rocprofv3."""
    import torch
    import paper_2307_12276_amd as A
    from paper_2307_12276_amd import learned
    import workloads as W
    bins = W.c4_bins(steps=steps)
    dt = bins[0].dt
    S = [dev_tensor(b.S(0)) for b in bins]
    ops = [make_op(b, A.STORAGE_FP32_FIELDS) for b in bins]
    Wd = torch.from_numpy(learned.load()).cuda()
    batch = A.Batch(ops, tile_rows=tile_rows)
    batch.learned_bound(dt, Wd, torch.empty(72 * len(ops), dtype=torch.float32, device="cuda"))
    u = [dev_tensor(b.u0) for b in bins]
    batch.bind(u, S)
    mv = 0
    for _ in range(steps):
        mv += int(batch.midpoint_step(None, None, dt, tol).array["matvecs"].sum())
    torch.cuda.synchronize()
    log("bins: %d steps, %d matvecs, tile rows %d" % (steps, mv, tile_rows))


def calibrate_copy():
    """A plain 1 GiB device copy (read 1 GiB, write 1 GiB): the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    a = torch.zeros(128 << 20, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": a.numel() * 8}), flush=True)


def copy_bandwidth(nbytes=1 << 30, reps=5):
    """Device-to-device copy of nbytes (read nbytes, write nbytes), timed with
    HIP events on the current stream: the practical HBM rate next to the 8 TB/s
    peak.  Returns GB/s of moved bytes (2 * nbytes per copy), best of reps."""
    import torch
    a = torch.zeros(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = max(best, 2.0 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def host_cpu():
    """Model name of the host CPU and the number of logical CPUs."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline_c2(w, budget_s):
    """The FP64 oracle, single-threaded, on the first steps of the 512^2
    workload until budget_s seconds of CPU work have been spent."""
    from threadpoolctl import threadpool_limits
    from oracle import bounds, integrators
    from oracle import operator as O
    oop = O.make_operator(w.Dxx, w.Dxy, w.Dyy, w.ax_c, w.ay_c, w.hx, w.hy, w.bc)
    A_ = lambda x: O.apply(oop, x)
    alpha = bounds.gershgorin(oop)
    u = w.u0.copy()
    steps = 0
    t0 = time.perf_counter()
    with threadpool_limits(1):
        while True:
            S1, S2 = w.stage_sources(steps)
            u = integrators.exp_quad2_step(A_, u, S1, S2, w.c1, w.c2, w.dt, alpha, w.tol)
            steps += 1
            if time.perf_counter() - t0 >= budget_s:
                break
    el = time.perf_counter() - t0
    return steps / el, steps, el, u


def cpu_baseline_sample(w, budget_s, matvecs_per_step):
    """The FP64 oracle, single-threaded, on a bounded sample of the headline
    workload: the stage vector w = A u0 + S of step 1 (one matvec, with the
    step's Newton coefficients) and then as many Newton terms of its phi_1
    sweep as fit the budget.  The oracle's steps/s is 1 / (seconds per matvec
    x the matvecs of a step)."""
    from threadpoolctl import threadpool_limits
    from oracle import bounds, leja
    from oracle import operator as O
    oop = O.make_operator(w.Dxx, w.Dxy, w.Dyy, w.ax_c, w.ay_c, w.hx, w.hy, w.bc)
    A_ = lambda x: O.apply(oop, x)
    alpha = bounds.gershgorin(oop)  # once per operator (setup), as on the GPU
    with threadpool_limits(1):
        t0 = time.perf_counter()
        S1 = w.stage_sources(0)[0]
        v = A_(w.u0) + S1
        d = leja.newton_coefficients(1, alpha, w.dt)
        t_stage = time.perf_counter() - t0
        n = max(2, min(matvecs_per_step, int(budget_s / max(t_stage, 1e-3)) - 1))
        t1 = time.perf_counter()
        leja.newton_sweep(A_, v, alpha, w.dt, d, w.tol, max_degree=n)
        t_sweep = time.perf_counter() - t1
    s_per_mv = (t_stage + t_sweep) / (1 + n)
    return 1.0 / (s_per_mv * matvecs_per_step), n, t_stage + t_sweep, s_per_mv


def c2_leg(steps=50, warmup=2, cpu_budget=0.0):
    """The 512^2 Dirichlet two-stage quadrature workload (working set in
    L2/MALL, four Newton terms per launch): steps/s, the Newton-Leja launches
    from HIP events on a second pass, and the GPU's error against the
    oracle on the first steps (with the oracle's steps/s) when cpu_budget > 0."""
    import numpy as np
    import torch
    import paper_2307_12276_amd as A
    import workloads as W
    w = W.c2_dirichlet_circular(n=512, steps=warmup + 2 * steps)
    op = make_op(w, A.STORAGE_FP64)
    alpha, _ = op.spectral_bound(A.BOUND_GERSHGORIN)
    u = dev_tensor(w.u0)
    srcs = device_sources(w)
    for n in range(warmup):
        gpu_step(op, w, u, n, srcs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mv = 0
    for n in range(warmup, warmup + steps):
        mv += gpu_step(op, w, u, n, srcs)["matvecs"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    op.profile(True)
    for n in range(warmup + steps, warmup + 2 * steps):
        gpu_step(op, w, u, n, srcs)
    torch.cuda.synchronize()
    ms4, n4, b4, t4 = op.profile_read_kind(A.LAUNCH_FOUR)
    ms, launches, nbytes = op.profile_read()
    op.profile(False)
    res = {"workload": "dirichlet-circular-512: Dirichlet 512x512, circular b, k_par/k_perp=1e3, a=(0.2,0), "
                       "time-independent Gaussian source, two-stage exp. quadrature c=(1/3,2/3), "
                       "dt=200 dt_CFL, tol=1e-10, FP64",
           "steps": steps, "steps_per_s": steps / el, "matvecs_per_step": mv / steps,
           "leja_launches": launches, "avg_leja_launch_us": 1e3 * ms / max(launches, 1),
           "four_term_launches": n4, "avg_four_term_launch_us": 1e3 * ms4 / max(n4, 1),
           "four_term_GBs_8d": (BYTES_PER_TERM_FP64 * w.nx * w.ny * t4 / max(n4, 1))
           / (ms4 / max(n4, 1) * 1e-3) / 1e9 if n4 else None,
           "note": "~15 MB per Newton term: L2/MALL-resident, launch-latency bound"}
    log("512^2 leg: %.1f steps/s, %.1f matvecs/step, four-term launches %.2f us avg"
        % (res["steps_per_s"], res["matvecs_per_step"], res["avg_four_term_launch_us"]))
    if cpu_budget > 0:
        cw = W.c2_dirichlet_circular(n=512, steps=steps)
        rate, nst, el_cpu, u_cpu = cpu_baseline_c2(cw, cpu_budget)
        op2 = make_op(cw, A.STORAGE_FP64)
        op2.set_bound(alpha)
        ug = dev_tensor(cw.u0)
        s2 = device_sources(cw)
        for n in range(nst):
            gpu_step(op2, cw, ug, n, s2)
        torch.cuda.synchronize()
        err = float(np.linalg.norm(ug.cpu().numpy() - u_cpu) / np.linalg.norm(u_cpu))
        res["oracle_steps_per_s"] = rate
        res["parity"] = {"steps": nst, "rel_l2_vs_oracle": err, "oracle_seconds": el_cpu}
        log("512^2 leg: oracle %.3f steps/s over %d steps; GPU rel err on those steps %.2e" % (rate, nst, err))
        del op2
    del op
    torch.cuda.empty_cache()
    return res


def _c4_worker_init():
    global _C4_BINS
    import workloads as W
    _C4_BINS = W.c4_bins(steps=1)


def _c4_worker_step(b, tol):
    """One oracle midpoint step of bin b (single-threaded, Gershgorin bound)."""
    from threadpoolctl import threadpool_limits
    from oracle import bounds, integrators
    from oracle import operator as O
    w = _C4_BINS[b]
    with threadpool_limits(1):
        oop = O.make_operator(w.Dxx, w.Dxy, w.Dyy, w.ax_c, w.ay_c, w.hx, w.hy, w.bc)
        alpha = bounds.gershgorin(oop)
        t0 = time.perf_counter()
        st = {}
        integrators.exp_midpoint_step(lambda x: O.apply(oop, x), w.u0, w.S(0.0), w.dt, alpha, tol, stats=st)
        return time.perf_counter() - t0, st["matvecs"]


def oracle_c4_all_cores(tol=1e-9, workers=None):
    """The oracle on every host core: one midpoint step of all 256 momentum
    bins, each bin in a single-threaded worker process (a process pool of one
    worker per logical CPU, at most 16), with each bin's Gershgorin interval.
    Returns steps/s of the whole 256-bin system (1 / wall time of the step)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    n = workers or min(16, os.cpu_count() or 1)
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(max_workers=n, mp_context=ctx, initializer=_c4_worker_init) as ex:
        list(ex.map(_c4_worker_step, [0] * n, [tol] * n))  # start the workers, build the bins
        t0 = time.perf_counter()
        res = list(ex.map(_c4_worker_step, range(256), [tol] * 256))
        wall = time.perf_counter() - t0
    cpu = sum(r[0] for r in res)
    return {"steps_per_s": 1.0 / wall, "wall_s": wall, "cpu_s": cpu, "workers": n,
            "matvecs": sum(r[1] for r in res),
            "sample": "one exponential midpoint step of all 256 bins (tol %g, Gershgorin interval per bin), "
                      "one single-threaded NumPy process per logical CPU" % tol}


def headline(args):
    """The 4096^2 FP64 stream-function workload (module docstring)."""
    import torch
    import paper_2307_12276_amd as A
    import workloads as W
    total = args.warmup + 2 * args.steps
    t0 = time.perf_counter()
    w = W.roofline_shape(n=4096, steps=total)
    log("headline: 4096^2 fields built in %.1fs" % (time.perf_counter() - t0))
    t0 = time.perf_counter()
    op = make_op(w, A.STORAGE_FP64)
    alpha, _ = op.spectral_bound(A.BOUND_GERSHGORIN)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    # the pulsed source at each step's midpoint, resident in HBM before timing
    S = [dev_tensor(w.stage_sources(n)[0]) for n in range(total)]
    u = dev_tensor(w.u0)
    for n in range(args.warmup):
        op.midpoint_step(u, S[n], w.dt, w.tol)
    torch.cuda.synchronize()
    # timed region: K steps, no per-launch instrumentation
    t0 = time.perf_counter()
    mv = 0
    for n in range(args.warmup, args.warmup + args.steps):
        mv += op.midpoint_step(u, S[n], w.dt, w.tol)["matvecs"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # kernel timing pass: the next K steps again, every Newton-Leja launch timed
    # by HIP events attached to its dispatch on the op's stream (per-launch
    # events slow the host loop, so they stay out of the timed region)
    op.profile(True)
    t1 = time.perf_counter()
    for n in range(args.warmup + args.steps, total):
        op.midpoint_step(u, S[n], w.dt, w.tol)
    torch.cuda.synchronize()
    el_prof = time.perf_counter() - t1
    kinds = {k: op.profile_read_kind(getattr(A, "LAUNCH_" + k.upper()))
             for k in ("first", "one", "two", "three", "four")}
    op.profile_read()
    op.profile(False)
    # the dominant launch kind (the most kernel time): three terms per launch
    dom = max(("two", "three", "four"), key=lambda k: kinds[k][0])
    ms2, n2, fused2, terms2 = kinds[dom]
    N = w.nx * w.ny
    avg_s = ms2 / max(n2, 1) * 1e-3
    alg = BYTES_PER_TERM_FP64 * N * terms2 / max(n2, 1)
    achieved = alg / avg_s / 1e9 if n2 else 0.0
    traffic = measured_traffic()
    value = args.steps / el
    log("headline: %d steps in %.3fs: %.2f steps/s, %.1f matvecs/step; %s-term launches %.1f us avg over %d "
        "(%.2f terms each): %.0f GB/s by 56 B/pt/term (%.1f%% of 8 TB/s)"
        % (args.steps, el, value, mv / args.steps, dom, avg_s * 1e6, n2, terms2 / max(n2, 1), achieved,
           100 * achieved / HBM_PEAK_GBS))
    out = {
        "metric": METRIC, "value": value, "unit": "steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded analytic fields)",
        "config": {"workload": "periodic-stream-4096: periodic 4096x4096, b from a seeded 32-mode stream "
                               "function, k_par=1, k_par/k_perp=1e4, a=(0.2,0), pulsed Gaussian source, "
                               "exp. midpoint, dt=100 dt_CFL, tol=1e-10, FP64",
                   "nx": w.nx, "ny": w.ny, "dt": w.dt, "tol": w.tol, "alpha": alpha,
                   "matvecs_per_step": mv / args.steps, "matvecs_per_s": mv / el, "setup_s": setup_s},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": KIND_KERNELS[dom],
                     "bytes_per_launch": alg, "bytes_rule": "56 B per point and Newton term (FP64) x %d points "
                                                           "x %.2f terms per launch" % (N, terms2 / max(n2, 1)),
                     "avg_kernel_us": avg_s * 1e6, "launches": n2,
                     "fused_bytes_per_launch": fused2 / max(n2, 1),
                     "timing": "HIP events on each %s-term dispatch, second pass of %d steps (%.3fs)"
                               % (dom, args.steps, el_prof),
                     "traffic_source": "profiles/%s (rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, "
                                       "scaled by a 1 GiB copy), bytes per launch" % os.path.basename(TRAFFIC_FILE)},
        "launch_kinds": {k: {"launches": v[1], "avg_us": 1e3 * v[0] / v[1] if v[1] else None, "terms": v[3]}
                         for k, v in kinds.items()},
    }
    if traffic:
        out["roofline"]["traffic_GBs"] = traffic / avg_s / 1e9
    del op, S, u
    torch.cuda.empty_cache()
    return out, w


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the 512^2, roofline, bins and paper-case legs")
    ap.add_argument("--profile-leja", type=int, default=0, help="run one sweep at this size and exit")
    ap.add_argument("--profile-c2", type=int, default=0,
                    help="run this many steps of the 512^2 Dirichlet quadrature workload and exit")
    ap.add_argument("--calibrate-copy", action="store_true", help="run a 1 GiB copy and exit")
    ap.add_argument("--fp32", action="store_true", help="with --profile-leja: fields stored in FP32")
    ap.add_argument("--profile-bins", action="store_true",
                    help="run the chosen 256-bin batched form for a few steps and exit")
    ap.add_argument("--one-term", action="store_true", help="with --profile-leja: one Newton term per launch")
    ap.add_argument("--frames", action="store_true",
                    help="with --profile-leja: two terms per launch with the register-frame kernel")
    args = ap.parse_args()
    if args.profile_leja:
        profile_leja(args.profile_leja, 0 if args.one_term else (3 if args.frames else 1), args.fp32)
        return
    if args.profile_c2:
        profile_c2(args.profile_c2)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.profile_bins:
        profile_bins()
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(bins and row slabs would shard across GPUs; see the design notes). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2307_12276_amd as A
    import workloads as W

    torch.cuda.init()
    out, w = headline(args)

    if not args.no_cpu:
        mvs = out["config"]["matvecs_per_step"]
        rate, nterms, el_cpu, s_mv = cpu_baseline_sample(w, args.cpu_budget, int(round(mvs)))
        model, ncpu = host_cpu()
        out["cpu_baseline"] = {"value": rate, "unit": "steps/s", "cores": 1, "kind": "oracle",
                               "sample": "step 1 of the same 4096^2 workload: the stage vector and the first %d "
                                         "Newton terms of its phi_1 sweep (%d matvecs, %.1fs, %.2fs per matvec); "
                                         "steps/s = 1 / (s per matvec x %.1f matvecs per step), NumPy FP64, "
                                         "single-threaded" % (nterms, nterms + 1, el_cpu, s_mv, mvs),
                               "host_cpu": model, "host_logical_cpus": ncpu}
        log("cpu oracle: %.2f s per matvec at 4096^2 -> %.4f steps/s" % (s_mv, rate))
    del w

    if not args.no_extra:
        torch.cuda.empty_cache()
        out["c2_512"] = c2_leg(cpu_budget=0.0 if args.no_cpu else 5.0)
        legs = []
        t0 = time.time()
        rw = W.roofline_shape(n=4096)
        log("roofline leg: 4096^2 fields built in %.1fs" % (time.time() - t0))
        for storage, mode in ((A.STORAGE_FP64, 0), (A.STORAGE_FP64, 2), (A.STORAGE_FP64, 3),
                              (A.STORAGE_FP64, 1), (A.STORAGE_FP32_FIELDS, 2), (A.STORAGE_FP32_FIELDS, 1)):
            legs.append(run_roofline_leg(rw, storage, mode))
            log("roofline leg %s %s: %.1f us/launch, %.1f us/term, %.0f GB/s (%.1f%% of 8 TB/s)" % (
                legs[-1]["storage"], legs[-1]["launches_of"], legs[-1]["avg_kernel_us"],
                legs[-1]["us_per_term"], legs[-1]["achieved_GBs"], 100 * legs[-1]["frac_of_8TBs"]))
        copy_gbs = copy_bandwidth()
        log("device copy of 1 GiB: %.0f GB/s (read + write)" % copy_gbs)
        for leg in legs:
            leg["frac_of_copy"] = leg["achieved_GBs"] / copy_gbs
        out["roofline_4096"] = legs
        out["copy_GBs"] = copy_gbs
        out["four_term_640"] = four_term_leg()
        out["chosen_vs_plain"] = chosen_vs_plain()
        if not args.no_cpu:
            c4 = oracle_c4_all_cores()
            out["chosen_vs_plain"]["oracle_all_cores"] = c4
            log("oracle, all cores (%d workers): one step of 256 bins in %.1fs (%.1f s of CPU)"
                % (c4["workers"], c4["wall_s"], c4["cpu_s"]))
        out["paper_cases"] = paper_cases_leg()

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
