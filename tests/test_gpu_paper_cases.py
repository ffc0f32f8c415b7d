"""The paper's test problems (Sec. 3, Cases I-IV) through the C-ABI on the
GPU: parity with the oracle on every case and scheme, and the Leja half of
the work-precision study against exact-in-time references (paper_refs.py):
error and matvec count per tolerance for Cases I/II, the orders of the
exponential midpoint and Gauss rules for Cases III/IV.  The tables are
printed (pytest -s)."""
import pytest

import paper_refs as R
import workloads as W
from oracle import bounds

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12276_amd as A  # noqa: E402
from gpu_util import rel, to_dev, to_np  # noqa: E402


def make_op(w):
    return A.Op(to_dev(w.Dxx), to_dev(w.Dxy), to_dev(w.Dyy), w.hx, w.hy, w.bc, A.STORAGE_FP64,
                ax_c=w.ax_c, ay_c=w.ay_c)


def gpu_run(w, op, tol):
    """u after w.steps steps of the workload's scheme, and the matvec count."""
    u = to_dev(w.u0)
    mv = 0
    if w.scheme == "exp":
        out = torch.empty_like(u)
        for _ in range(w.steps):
            mv += op.leja_phi(0, w.dt, u, out, tol)["matvecs"]
            u, out = out, u
        return to_np(u), mv
    for k in range(w.steps):
        S1, S2 = w.stage_sources(k)
        if w.scheme == "midpoint":
            st = op.midpoint_step(u, to_dev(S1), w.dt, tol)
        else:
            st = op.quad2_step(u, to_dev(S1), to_dev(S2), w.c1, w.c2, w.dt, tol)
        mv += st["matvecs"]
    return to_np(u), mv


@pytest.mark.parametrize("case,scheme", [("I", "exp"), ("II", "midpoint"), ("III", "midpoint"),
                                         ("III", "quad2"), ("IV", "midpoint"), ("IV", "quad2")])
def test_paper_case_parity(case, scheme):
    """Each case at 40 x 40 with its default step (Case I: one phi_0 step over
    the whole interval, in substeps): same matvec count as the oracle and
    the same result to 1e-10."""
    w = W.paper_case(case, 40, scheme=scheme)
    alpha = bounds.gershgorin(R.op_of(w))
    op = make_op(w)
    op.set_bound(alpha)
    g, mg = gpu_run(w, op, w.tol)
    o, mo = R.oracle_run(w, w.tol, alpha)
    print("case %s %s: %d steps, %d matvecs, rel diff %.2e" % (case, scheme, w.steps, mg, rel(g, o)))
    assert mg == mo
    assert rel(g, o) < 1e-10


@pytest.mark.parametrize("case", ["I", "II"])
def test_work_precision_exact_in_time(case):
    """Cases I (ring, T = 0.75, one step) and II (spiral 2 with advection and
    the sources of eq. 8, T = 0.85, steps of 1e4 dt_CFL) at 64 x 64, tol 1e-2
    .. 1e-10, the GPU's own Gershgorin bound: tol is the accuracy asked of
    the solution (as Sec. 3 uses it), so for tol <= 1e-4 the error against the exact
    solution stays within 10 tol -- the bound the oracle's stopping rule is
    pinned to on these problems (tests/test_paper_cases.py, measured up to
    5 tol) -- the error falls with the tolerance from 1e-3 on (to 5 % at
    saturation) and the matvec count never falls."""
    w = W.paper_case(case, 64)
    ref = R.exact_solution(w)
    op = make_op(w)
    op.spectral_bound(A.BOUND_GERSHGORIN)
    rows = []
    for e in range(2, 11):
        tol = 10.0 ** -e
        u, mv = gpu_run(w, op, tol)
        rows.append((tol, mv, rel(u, ref)))
    print("\ncase %s, 64^2, %d step(s) of %.3g dt_CFL:" % (case, w.steps, w.dt / w.extra["dt_cfl"]))
    for tol, mv, err in rows:
        print("  tol %.0e  matvecs %6d  rel. error %.2e  error / tol %.2f" % (tol, mv, err, err / tol))
    errs = [r[2] for r in rows[1:]]
    assert all(b <= 1.05 * a for a, b in zip(errs, errs[1:])), errs
    assert all(a[1] <= b[1] for a, b in zip(rows, rows[1:]))
    assert all(err <= 10 * tol for tol, _, err in rows if tol <= 1e-4), rows


@pytest.mark.parametrize("case", ["III", "IV"])
def test_midpoint_and_gauss_orders(case):
    """Cases III/IV (time-dependent sources of eq. 9) at 64 x 64 to T = 0.1,
    tol 1e-12, steps of 80, 40, 20 and 10 dt_CFL: exponential midpoint
    converges with order 2, exponential Gauss with order 4, and Gauss is the
    more accurate at every step size for a similar matvec count."""
    w0 = W.paper_case(case, 64)
    ref = R.exact_solution(w0)
    res = {}
    print("\ncase %s, 64^2, T = 0.1:" % case)
    for scheme in ("midpoint", "quad2"):
        steps, errs, mvs = [], [], []
        for mult in (80.0, 40.0, 20.0, 10.0):
            w = W.paper_case(case, 64, dt_mult=mult, scheme=scheme)
            op = make_op(w)
            op.spectral_bound(A.BOUND_GERSHGORIN)
            u, mv = gpu_run(w, op, 1e-12)
            steps.append(w.steps)
            errs.append(rel(u, ref))
            mvs.append(mv)
            print("  %-8s dt %3.0f dt_CFL  steps %4d  matvecs %6d  rel. error %.2e"
                  % (scheme, mult, w.steps, mv, errs[-1]))
        res[scheme] = (steps, errs, mvs)
    om = R.observed_order(*res["midpoint"][:2])
    og = R.observed_order(*res["quad2"][:2])
    print("  observed orders: midpoint %s, Gauss %s" % (["%.2f" % p for p in om], ["%.2f" % p for p in og]))
    assert all(1.5 <= p <= 2.5 for p in om), om
    assert all(p >= 3.2 for p in og), og
    assert all(g < m for g, m in zip(res["quad2"][1], res["midpoint"][1]))
    assert all(g <= 1.2 * m for g, m in zip(res["quad2"][2], res["midpoint"][2]))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("case,T", [("III", 0.10), ("III", 0.30), ("IV", 0.10), ("IV", 0.30)])
def test_work_precision_time_dependent_sources(case, T):
    """The Leja half of Figs. 4-5 (Sec. 3): spirals 1 and 2 with advection and
    the time-dependent sources of eq. 9 at 64 x 64, T = 0.10 and 0.30, steps
    of 10, 100 and 500 dt_CFL, tol 1e-2 .. 1e-10, exponential midpoint and
    exponential Gauss quadrature, error against the exact solution and
    matvec count (the table is printed).  What the paper reports for these
    figures, checked here:
    - Gauss, fourth order, is more accurate than the second-order midpoint
      rule in every configuration once tol no longer dominates (tol <= 1e-6);
    - at 100 and 500 dt_CFL the midpoint error saturates: the step's
      discretisation error sets it whatever the tolerance (tol 1e-6 .. 1e-10
      within a factor of 1.5 of each other);
    - at large steps Gauss is at least 3x more accurate than midpoint for a
      similar number of matvecs (within 1.5x)."""
    ref = R.exact_solution(W.paper_case(case, 64, T=T))
    res = {}
    print("\ncase %s, 64^2, T = %.2f:" % (case, T))
    for mult in (10.0, 100.0, 500.0):
        for scheme in ("midpoint", "quad2"):
            w = W.paper_case(case, 64, dt_mult=mult, T=T, scheme=scheme)
            op = make_op(w)
            op.spectral_bound(A.BOUND_GERSHGORIN)
            rows = []
            for e in range(2, 11):
                u, mv = gpu_run(w, op, 10.0 ** -e)
                rows.append((10.0 ** -e, mv, rel(u, ref)))
            res[(mult, scheme)] = rows
            print("  dt %3.0f dt_CFL (%4d steps) %-8s " % (mult, w.steps, "midpoint" if scheme == "midpoint"
                                                            else "Gauss")
                  + " ".join("%.0e:%d/%.1e" % (t, m, err) for t, m, err in rows))
            del op
    for mult in (10.0, 100.0, 500.0):
        mid, gau = res[(mult, "midpoint")], res[(mult, "quad2")]
        for (t, _, em), (_, _, eg) in zip(mid, gau):
            if t <= 1e-6:
                assert eg < em, (mult, t, eg, em)
        if mult >= 100.0:
            tight = [r[2] for r in mid if r[0] <= 1e-6]
            assert max(tight) <= 1.5 * min(tight), (mult, tight)
            em, mm = mid[-1][2], mid[-1][1]
            eg, mg = gau[-1][2], gau[-1][1]
            assert eg * 3.0 <= em and mg <= 1.5 * mm, (mult, em, mm, eg, mg)
