"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  FP64 results must agree to 1e-10 relative L2 with the
same Leja degrees."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import bounds, integrators, leja
from oracle import operator as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12276_amd as A  # noqa: E402
from gpu_util import make_pair, rel, to_dev, to_np, workload_pair  # noqa: E402

SHAPES = [(3, 3), (5, 7), (64, 64), (130, 70), (257, 33), (256, 9), (300, 129), (128, 128)]


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
@pytest.mark.parametrize("adv", ["const", "field"])
def test_apply_matches_oracle(nx, ny, bc, adv):
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=nx * 31 + ny, field_advection=(adv == "field"))
    hx, hy = 1.0 / nx, 0.7 / ny
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc)
    x = W.random_vector((ny, nx), 5)
    y = torch.empty_like(to_dev(x))
    gop.apply(to_dev(x), y)
    ref = O.apply(oop, x)
    assert rel(to_np(y), ref) < 1e-13


@pytest.mark.parametrize("storage", [1, 2])
def test_apply_fp32_fields(storage):
    nx, ny = 300, 77
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=3, field_advection=True)
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, 1 / nx, 1 / ny, O.PERIODIC, storage)
    x = W.random_vector((ny, nx), 1)
    y = torch.empty_like(to_dev(x))
    gop.apply(to_dev(x), y)
    assert rel(to_np(y), O.apply(oop, x)) < 1e-13


@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
def test_tile_corner_impulses(bc):
    """Unit impulses at tile corners and strip / band edges."""
    nx, ny = 520, 200
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=8, field_advection=True)
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, 1 / nx, 1 / ny, bc)
    t = gop_tiling_guess = None  # noqa: F841
    x = np.zeros((ny, nx))
    for j in (0, 1, 3, 4, 15, 16, 31, 32, 63, 64, ny - 2, ny - 1):
        for i in (0, 1, 63, 64, 127, 128, 255, 256, 511, 512, nx - 1):
            x[j, i] += 1.0 + 0.001 * (i + j)
    y = torch.empty_like(to_dev(x))
    gop.apply(to_dev(x), y)
    ref = O.apply(oop, x)
    assert np.max(np.abs(to_np(y) - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
def test_gershgorin(bc):
    nx, ny = 131, 66
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=2, field_advection=True)
    oop, gop = make_pair(Dxx, Dxy, Dyy, 5 * ax, 5 * ay, 1 / nx, 1 / ny, bc)
    a, _ = gop.spectral_bound(A.BOUND_GERSHGORIN)
    assert a == pytest.approx(bounds.gershgorin(oop), rel=1e-13)


def test_power_iteration():
    w = W.c2_dirichlet_circular(n=48)
    oop, gop = workload_pair(w)
    a, its = gop.spectral_bound(A.BOUND_POWER, max_iter=3000, rtol=1e-6, seed=7)
    ao, itso = bounds.spectral_bound(oop, 1, max_iter=3000, rtol=1e-6, seed=7)
    assert its == itso
    assert a == pytest.approx(ao, rel=1e-10)


@pytest.mark.parametrize("l", [0, 1, 2])
@pytest.mark.parametrize("rho_max", [1600.0, 30.0])
def test_leja_phi(l, rho_max):
    w = W.c2_dirichlet_circular(n=40)
    oop, gop = workload_pair(w)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    gop.set_limits(500, rho_max)
    v = W.random_vector(oop.shape, 4)
    out = torch.empty_like(to_dev(v))
    st = gop.leja_phi(l, w.dt, to_dev(v), out, 1e-10)
    ost = {}
    ref = leja.phi_apply(lambda x: O.apply(oop, x), l, w.dt, v, alpha, 1e-10, rho_max=rho_max, stats=ost)
    assert st["substeps"] == ost["substeps"]
    assert st["matvecs"] == ost["matvecs"]
    assert rel(to_np(out), ref) < 1e-12


def run_workload(w, steps, storage=None, quad2_mode=A.QUAD2_AUGMENTED):
    oop, gop = workload_pair(w, storage)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    gop.set_quad2_mode(quad2_mode)
    u = w.u0.copy()
    ug = to_dev(w.u0)
    A_ = lambda x: O.apply(oop, x)
    for n in range(steps):
        S1, S2 = w.stage_sources(n)
        ost = {}
        if w.scheme == "midpoint":
            u = integrators.exp_midpoint_step(A_, u, S1, w.dt, alpha, w.tol, stats=ost)
            st = gop.midpoint_step(ug, to_dev(S1) if S1 is not None else None, w.dt, w.tol)
        else:
            mode = "augmented" if quad2_mode == A.QUAD2_AUGMENTED else "two_sweep"
            u = integrators.exp_quad2_step(A_, u, S1, S2, w.c1, w.c2, w.dt, alpha, w.tol, stats=ost, mode=mode)
            st = gop.quad2_step(ug, to_dev(S1) if S1 is not None else None,
                                to_dev(S2) if S2 is not None else None, w.c1, w.c2, w.dt, w.tol)
        assert st["matvecs"] == ost["matvecs"], (n, st, ost)
    return to_np(ug), u


def test_periodic_constant_midpoint_full_config():
    """64x64 periodic constant tensor, exponential midpoint, 10 steps."""
    w = W.c1_periodic_constant(n=64, steps=10)
    g, o = run_workload(w, w.steps)
    assert rel(g, o) < 1e-10


@pytest.mark.parametrize("mode", [A.QUAD2_AUGMENTED, A.QUAD2_TWO_SWEEP])
def test_dirichlet_circular_quad2_small(mode):
    w = W.c2_dirichlet_circular(n=96, steps=4)
    g, o = run_workload(w, w.steps, quad2_mode=mode)
    assert rel(g, o) < 1e-10


def test_dirichlet_circular_quad2_full_size_two_steps():
    """512x512 Dirichlet circular field, two-stage quadrature (1/3, 2/3),
    dt = 200 dt_CFL: the first two of its steps against the oracle."""
    w = W.c2_dirichlet_circular(n=512)
    g, o = run_workload(w, 2)
    assert rel(g, o) < 1e-10


def test_stream_function_fp32_storage_parity():
    """Stream-function field with FP32 fields (mode 1) and FP32 Newton vectors
    (mode 2): mode 1 equals the oracle run on the FP32-rounded fields to
    1e-10; mode 2 is within 1e-5 of it."""
    w = W.c3_stream_function(n=128, steps=3, storage=1)
    g1, o1 = run_workload(w, 3, storage=1)
    assert rel(g1, o1) < 1e-10
    g2, _ = run_workload(w, 3, storage=2)
    assert rel(g2, o1) < 1e-5


def test_gauss_quad2_and_time_dependent_source():
    """Exponential Gauss nodes with the time-dependent sources of eq. 9."""
    X, Y, hx, hy = W.grid_2d(70, 60, W.DIRICHLET, box=(-1, 1, -1, 1))
    Dxx, Dxy, Dyy = W.spiral_tensor(X, Y, 2)
    oop, gop = make_pair(Dxx + 1e-4, Dxy, Dyy + 1e-4, 1.0, 2.0, hx, hy, W.DIRICHLET)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    c1, c2 = 0.5 - math.sqrt(3) / 6, 0.5 + math.sqrt(3) / 6
    u = W.gaussian(X, Y, 0.2, 0.1, 0.2)
    ug = to_dev(u)
    dt = 2e-3
    A_ = lambda x: O.apply(oop, x)
    for n in range(3):
        t = 0.08 + n * dt
        S1, S2 = W.source_tds(X, Y, t + c1 * dt), W.source_tds(X, Y, t + c2 * dt)
        u = integrators.exp_quad2_step(A_, u, S1, S2, c1, c2, dt, alpha, 1e-10)
        gop.quad2_step(ug, to_dev(S1), to_dev(S2), c1, c2, dt, 1e-10)
    assert rel(to_np(ug), u) < 1e-10


@pytest.mark.parametrize("n,mode", [(64, 1), (128, 5), (128, 6)])
def test_zero_vector_degree_zero(n, mode):
    """v = 0 gives 0 with degree 0 (no matvec), whichever launch holds the
    first term: a one-term launch (mode 1 at 64^2), or the first launch of
    three (mode 5, which also runs terms 2 and 3 there) or of one then four
    (mode 6)."""
    w = W.c1_periodic_constant(n=n)
    oop, gop = workload_pair(w)
    gop.set_bound(-1000.0)
    gop.set_term_fusion(mode)
    z = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    out = torch.full_like(z, 7.0)
    st = gop.leja_phi(1, 1e-3, z, out, 1e-10)
    assert st["matvecs"] == 0 and float(out.abs().max()) == 0.0


def test_nan_input_is_reported_and_u_untouched():
    w = W.c1_periodic_constant(n=64)
    oop, gop = workload_pair(w)
    gop.spectral_bound(A.BOUND_GERSHGORIN)
    u = to_dev(w.u0)
    S = torch.zeros_like(u)
    S[3, 5] = float("nan")
    before = u.clone()
    with pytest.raises(A.AdlError) as e:
        gop.midpoint_step(u, S, w.dt, 1e-10)
    assert e.value.code == A.ENAN
    assert torch.equal(u, before)


def test_degree_cap_triggers_substeps_then_enoconv():
    w = W.c1_periodic_constant(n=64)
    oop, gop = workload_pair(w)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    gop.set_limits(20, 1600.0)
    v = W.random_vector(oop.shape, 2)
    out = torch.empty_like(to_dev(v))
    st = gop.leja_phi(1, w.dt, to_dev(v), out, 1e-10)
    ost = {}
    ref = leja.phi_apply(lambda x: O.apply(oop, x), 1, w.dt, v, alpha, 1e-10, max_degree=20, stats=ost)
    assert st["substeps"] == ost["substeps"] > 1
    assert rel(to_np(out), ref) < 1e-12
    gop.set_limits(2, 1600.0)
    with pytest.raises(A.AdlError) as e:
        gop.leja_phi(1, 100 * w.dt, to_dev(v), out, 1e-10)
    assert e.value.code == A.ENOCONV


def test_invalid_arguments():
    w = W.c1_periodic_constant(n=64)
    oop, gop = workload_pair(w)
    u = to_dev(w.u0)
    with pytest.raises(A.AdlError) as e:
        gop.midpoint_step(u, None, w.dt, 1e-10)  # no bound yet
    assert e.value.code == A.EBOUND
    gop.set_bound(-100.0)
    for dt, tol in [(0.0, 1e-10), (-1.0, 1e-10), (1e-3, 0.0), (1e-3, 1.0)]:
        with pytest.raises(A.AdlError) as e:
            gop.midpoint_step(u, None, dt, tol)
        assert e.value.code == A.EINVAL
    with pytest.raises(A.AdlError):
        gop.quad2_step(u, None, None, 0.5, 0.5, 1e-3, 1e-10)
    with pytest.raises(A.AdlError) as e:
        gop.set_bound(1.0)
    assert e.value.code == A.EBOUND


def test_deterministic_bitwise():
    w = W.c2_dirichlet_circular(n=200, steps=2)
    oop, gop = workload_pair(w)
    gop.spectral_bound(A.BOUND_GERSHGORIN)
    outs = []
    for _ in range(2):
        u = to_dev(w.u0)
        S = to_dev(w.S(0))
        for n in range(2):
            gop.quad2_step(u, S, S, w.c1, w.c2, w.dt, w.tol)
        outs.append(to_np(u))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("nx,ny", [(33, 45), (64, 64), (130, 70), (257, 33), (300, 129), (128, 128), (250, 7)])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
@pytest.mark.parametrize("storage", [0, 1, 2])
def test_two_term_launches_match_one_term_launches(nx, ny, bc, storage):
    """Two Newton terms per launch (y_{k+1} kept on chip, one-column frames
    recomputed), with the input rows staged in LDS or read into registers,
    give the one-term result: same degree, same polynomial up to the
    grouping of the norm partial sums; and every mode equals the oracle
    (FP64 and FP32 fields: 1e-10 with the oracle's degree; FP32 Newton
    vectors: within the 1e-5 bound of the FP32-storage path -- each y_k is
    rounded to 2^-24 and the Newton sum's terms exceed |p| by the hump of
    the interpolant, observed 1.8e-6)."""
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=nx + 7 * ny, field_advection=(storage == 0))
    hx, hy = 1.0 / nx, 0.8 / ny
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc, storage)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    v = to_dev(W.random_vector((ny, nx), 11))
    dt = 300.0 / abs(alpha)
    outs, degs = [], []
    # one term per launch; two with LDS-staged rows; two with register frames
    for mode in (0, 2, 3):
        gop.set_term_fusion(mode)
        out = torch.empty_like(v)
        st = gop.leja_phi(1, dt, v, out, 1e-10)
        outs.append(to_np(out))
        degs.append(st["max_degree"])
    assert degs[0] == degs[1] == degs[2], degs
    assert rel(outs[1], outs[0]) < 1e-13
    assert rel(outs[2], outs[0]) < 1e-13
    ost = {}
    ref = leja.phi_apply(lambda x: O.apply(oop, x), 1, dt, to_np(v), alpha, 1e-10, stats=ost)
    for mode, o, d in zip((0, 2, 3), outs, degs):
        if storage == 2:
            assert rel(o, ref) < 1e-5, mode
        else:
            assert d == max(ost["degrees"]), (mode, d, ost)
            assert rel(o, ref) < 1e-10, mode


@pytest.mark.parametrize("nx,ny", [(33, 45), (64, 64), (130, 70), (257, 33), (300, 129), (250, 7), (70, 200)])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
@pytest.mark.parametrize("storage", [0, 1, 2])
def test_four_term_launches_match_one_term_launches(nx, ny, bc, storage):
    """Four Newton terms per launch (y_{k+1} .. y_{k+3} kept in LDS, three-row
    and three-lane frames recomputed) give the one-term result: same degree
    wherever the sweep stops inside a launch, same polynomial up to the
    grouping of the norm partial sums; the phi_1 + phi_2 sweep of the
    augmented form (the first term alone, then four per launch) too."""
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=5 * nx + ny, field_advection=(storage == 0))
    hx, hy = 1.0 / nx, 0.8 / ny
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc, storage)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    v = to_dev(W.random_vector((ny, nx), 13))
    outs, degs, quads = [], [], []
    for mode in (0, 4):
        gop.set_term_fusion(mode)
        o, d = [], []
        for mult in (40.0, 300.0, 2000.0):
            out = torch.empty_like(v)
            st = gop.leja_phi(1, mult / abs(alpha), v, out, 1e-10)
            o.append(to_np(out))
            d.append(st["max_degree"])
        outs.append(o)
        degs.append(d)
        u = v.clone()
        S = torch.full_like(v, 0.5)
        qs = gop.quad2_step(u, S, 2.0 * S, 1.0 / 3.0, 2.0 / 3.0, 300.0 / abs(alpha), 1e-10)
        quads.append((to_np(u), qs["matvecs"]))
    assert degs[0] == degs[1], degs
    # each kernel rounds (and fuses) the m terms' updates on its own: the
    # difference grows with the degree, ~m ulp of the largest partial sum
    errs = [rel(b, a) for a, b in zip(outs[0], outs[1])]
    print("degrees %s, four-term vs one-term %s" % (degs[0], ["%.1e" % e for e in errs]))
    for e, m in zip(errs, degs[0]):
        assert e < max(1e-13, 4e-15 * m), (e, m)
    # the quadrature step, with the same rounding bound over its matvecs; a
    # stage sweep whose stopping estimate lands within rounding of the
    # tolerance may stop one term apart in the two modes, a difference of the
    # order of tol |p|
    eq = rel(quads[1][0], quads[0][0])
    mq = quads[0][1]
    print("quad2 step: matvecs %d / %d, four-term vs one-term %.1e" % (mq, quads[1][1], eq))
    assert eq < (max(1e-13, 4e-15 * mq) if mq == quads[1][1] else 1e-10), eq


@pytest.mark.parametrize("mode,terms", [(5, 3), (6, 4)])
@pytest.mark.parametrize("nx,ny", [(128, 128), (130, 70), (300, 129), (250, 7), (200, 200), (256, 9), (512, 33)])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
@pytest.mark.parametrize("storage", [0, 1, 2])
def test_staged_multi_term_launches_match_one_term_launches(mode, terms, nx, ny, bc, storage):
    """Three (mode 5) or four (mode 6) Newton terms per launch with LDS-staged
    rows (the intermediate y kept in LDS rings) give the one-term result: the
    same degree wherever the sweep stops inside a launch (a replay of the
    launch stores p of that term), the same polynomial up to the grouping of
    the norm partial sums; the phi_1 + phi_2 sweep of the augmented form too;
    and the oracle's result (1e-10, same degree; FP32 Newton vectors within
    the 1e-5 of the FP32-storage path)."""
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=9 * nx + ny, field_advection=(storage == 0))
    hx, hy = 1.0 / nx, 0.8 / ny
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc, storage)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    v0 = W.random_vector((ny, nx), 17)
    v = to_dev(v0)
    outs, degs, quads, n3s = [], [], [], []
    mults = (40.0, 300.0, 2000.0)
    kind = A.LAUNCH_THREE if terms == 3 else A.LAUNCH_FOUR
    for m in (0, mode):
        gop.set_term_fusion(m)
        o, d = [], []
        gop.profile(True)
        for mult in mults:
            out = torch.empty_like(v)
            st = gop.leja_phi(1, mult / abs(alpha), v, out, 1e-10)
            o.append(to_np(out))
            d.append(st["max_degree"])
        _, n3, _, t3 = gop.profile_read_kind(kind)
        gop.profile(False)
        n3s.append((n3, t3))
        outs.append(o)
        degs.append(d)
        u = v.clone()
        S = torch.full_like(v, 0.5)
        qs = gop.quad2_step(u, S, 2.0 * S, 1.0 / 3.0, 2.0 / 3.0, 300.0 / abs(alpha), 1e-10)
        quads.append((to_np(u), qs["matvecs"]))
    assert n3s[0][0] == 0 and n3s[1][0] > 0 and n3s[1][1] == terms * n3s[1][0], n3s
    assert degs[0] == degs[1], degs
    errs = [rel(b, a) for a, b in zip(outs[0], outs[1])]
    print("degrees %s, %d-term vs one-term %s" % (degs[0], terms, ["%.1e" % e for e in errs]))
    for e, m in zip(errs, degs[0]):
        assert e < max(1e-13, 4e-15 * m), (e, m)
    eq = rel(quads[1][0], quads[0][0])
    mq = quads[0][1]
    print("quad2 step: matvecs %d / %d, %d-term vs one-term %.1e" % (mq, quads[1][1], terms, eq))
    assert eq < (max(1e-13, 4e-15 * mq) if mq == quads[1][1] else 1e-10), eq
    for mult, o, d in zip(mults, outs[1], degs[1]):
        ost = {}
        ref = leja.phi_apply(lambda x: O.apply(oop, x), 1, mult / abs(alpha), v0, alpha, 1e-10, stats=ost)
        if storage == 2:
            assert rel(o, ref) < 1e-5, mult
        else:
            assert d == max(ost["degrees"]), (mult, d, ost)
            assert rel(o, ref) < 1e-10, mult


@pytest.mark.parametrize("nx,ny", [(128, 128), (130, 70), (256, 9), (300, 129), (512, 33)])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
@pytest.mark.parametrize("storage", [0, 1])
def test_staged_midpoint_steps_match_oracle(nx, ny, bc, storage):
    """Midpoint steps with three terms per launch (mode 5): with FP64 Newton
    vectors the sweep's first launch forms the stage vector w = A u + S
    itself (the four-stage LDS march) instead of a separate stage launch.
    Two steps equal the oracle's (1e-10, the same matvec counts; FP32 fields:
    the oracle on the rounded fields) and the one-term-per-launch steps
    (1e-12), with a source and without one."""
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=5 * nx + ny, field_advection=(storage == 0))
    hx, hy = 1.0 / nx, 0.8 / ny
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc, storage)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    u0 = W.random_vector((ny, nx), 23)
    S0 = 0.3 * W.random_vector((ny, nx), 29)
    dt = 250.0 / abs(alpha)
    A_ = lambda x: O.apply(oop, x)  # noqa: E731
    for with_src in (True, False):
        res = {}
        for mode in (0, 5):
            gop.set_term_fusion(mode)
            u = to_dev(u0)
            S = to_dev(S0) if with_src else None
            mv = []
            for _ in range(2):
                mv.append(gop.midpoint_step(u, S, dt, 1e-10)["matvecs"])
            res[mode] = (to_np(u), mv)
        uo, mvo = u0.copy(), []
        for _ in range(2):
            ost = {}
            uo = integrators.exp_midpoint_step(A_, uo, S0 if with_src else None, dt, alpha, 1e-10, stats=ost)
            mvo.append(ost["matvecs"])
        e5, e0 = rel(res[5][0], uo), rel(res[5][0], res[0][0])
        print("source %s: matvecs %s / %s / oracle %s; mode 5 vs oracle %.1e, vs one-term %.1e"
              % (with_src, res[5][1], res[0][1], mvo, e5, e0))
        assert res[5][1] == res[0][1] == mvo
        assert e5 < 1e-10 and e0 < 1e-12


@pytest.mark.parametrize("nx,ny", [(33, 45), (64, 64), (257, 33)])
def test_staged_multi_term_modes_need_two_columns_per_lane(nx, ny):
    """Modes 5 and 6 need tilings with two columns per lane (nx even and at
    least 128): other widths are refused with ADL_EINVAL."""
    z = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    op = A.Op(z + 1.0, z, z + 1.0, 1.0 / nx, 1.0 / ny, A.BC_PERIODIC, A.STORAGE_FP64)
    for mode in (5, 6):
        with pytest.raises(A.AdlError) as e:
            op.set_term_fusion(mode)
        assert e.value.code == A.EINVAL


def test_default_mode_runs_four_terms_on_mid_grids():
    """Below 2^20 points the default mode launches four terms
    at a time (a quarter of the launches of a one-term sweep, give or take
    the first term and the tail), with the one-term result to rounding."""
    nx, ny = 704, 600
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=17, field_advection=False)
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, 1.0 / nx, 1.0 / ny, O.DIRICHLET, 0)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    v = to_dev(W.random_vector((ny, nx), 3))
    res = {}
    for mode in (0, 1):
        gop.set_term_fusion(mode)
        gop.profile(True)
        out = torch.empty_like(v)
        st = gop.leja_phi(1, 500.0 / abs(alpha), v, out, 1e-10)
        _, launches, _ = gop.profile_read()
        gop.profile(False)
        res[mode] = (to_np(out), st["max_degree"], launches)
    m = res[0][1]
    assert res[1][1] == m
    assert res[0][2] >= m and res[1][2] <= (m + 2) // 4 + 3, (res[0][2], res[1][2], m)
    assert rel(res[1][0], res[0][0]) < max(1e-13, 4e-15 * m)


def test_four_term_mode_needs_a_sweep_without_hints():
    """Mode 4 is refused while the op's sweeps carry non-temporal hints (the
    four-term kernel has no hinted form) and accepted without them, also at
    2^20 points (a fused launch stores only its last term's y and p, so the
    workspace needs no extra buffers for it)."""
    nx = ny = 1024
    z = torch.zeros((ny, nx), dtype=torch.float64, device="cuda")
    op = A.Op(z + 1.0, z, z + 1.0, 1.0 / nx, 1.0 / ny, A.BC_PERIODIC, A.STORAGE_FP64)
    op.set_streaming(1)
    with pytest.raises(A.AdlError, match="non-temporal"):
        op.set_term_fusion(4)
    op.set_streaming(0)
    op.set_term_fusion(4)
    op.set_term_fusion(1)


@pytest.mark.parametrize("nx,ny", [(64, 64), (130, 70), (257, 33)])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.DIRICHLET])
@pytest.mark.parametrize("storage", [0, 2])
def test_streaming_hints_do_not_change_results(nx, ny, bc, storage):
    """Non-temporal hints on the Newton vectors change cache policy only:
    bitwise the same result in every mode, one term per launch and two with
    either two-term kernel (the four-term kernel, the default on these grids,
    has no hinted form: with hints on, a sweep runs two terms per launch)."""
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=3 * nx + ny, field_advection=(storage == 0))
    hx, hy = 1.0 / nx, 1.0 / ny
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc, storage)
    gop.set_bound(bounds.gershgorin(oop))
    v = to_dev(W.random_vector((ny, nx), 5))
    dt = 200.0 / abs(bounds.gershgorin(oop))
    for fuse in (0, 2, 3):
        gop.set_term_fusion(fuse)
        outs = []
        for mode in (0, 1, -1):
            gop.set_streaming(mode)
            out = torch.empty_like(v)
            gop.leja_phi(1, dt, v, out, 1e-10)
            outs.append(to_np(out))
        assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    with pytest.raises(A.AdlError):
        gop.set_streaming(2)


def _wait_case(spin, v, dt, alpha, fields):
    """A fresh op (so that its first sweep guesses the chunk length), one
    phi_1 sweep and one quad2 step with the given host wait mode."""
    oop, gop = make_pair(*fields)
    gop.set_bound(alpha)
    gop.set_host_wait(spin)
    assert gop.host_wait() == spin
    out = torch.empty_like(v)
    s1 = gop.leja_phi(1, dt, v, out, 1e-10)
    u = v.clone()
    S = torch.full_like(v, 0.5)
    s2 = gop.quad2_step(u, S, 2.0 * S, 1.0 / 3.0, 2.0 / 3.0, dt, 1e-10)
    return to_np(out), s1, to_np(u), s2


def test_host_wait_modes_agree():
    """The sweep outcome awaited by spinning on the op's pinned host mirror
    (the default) or by copying the control block back: bitwise the same
    phi_1 result and quad2 step and the same statistics, over sweeps of
    several chunks (dt = 2000 / |alpha|: two substeps of degree 138 and 123,
    the first sweep of the plan guesses 114 terms and needs a second chunk);
    the phi_1 result matches the oracle."""
    nx, ny = 130, 70
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=11)
    fields = (Dxx, Dxy, Dyy, ax, ay, 1.0 / nx, 1.0 / ny, O.DIRICHLET)
    oop = O.make_operator(*fields)
    alpha = bounds.gershgorin(oop)
    v0 = W.random_vector((ny, nx), 5)
    v = to_dev(v0)
    dt = 2000.0 / abs(alpha)
    spin = _wait_case(True, v, dt, alpha, fields)
    copy = _wait_case(False, v, dt, alpha, fields)
    assert np.array_equal(spin[0], copy[0]) and np.array_equal(spin[2], copy[2])
    assert spin[1] == copy[1] and spin[3] == copy[3]
    st = {}
    ref = leja.phi_apply(lambda x: O.apply(oop, x), 1, dt, v0, alpha, 1e-10, stats=st)
    assert spin[1]["matvecs"] == st["matvecs"] and spin[1]["matvecs"] > 40
    assert rel(spin[0], ref) < 1e-10
    _, gop = make_pair(*fields)
    assert gop.host_wait()  # the default where pinned memory is available
    with pytest.raises(A.AdlError):
        A._check(A.lib().adl_op_set_host_wait(gop.handle, 2))


def test_host_mirror_slots_are_recycled():
    """More ops alive at once than one page of mirror slots (64), then all
    destroyed and as many created again (slots reused): every op's sweep
    gives the same result as the first op's, spinning on its mirror
    (76 terms in two chunks)."""
    n = 24
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(n, n, seed=5)
    fields = (Dxx, Dxy, Dyy, ax, ay, 1.0 / n, 1.0 / n, O.PERIODIC)
    alpha = bounds.gershgorin(O.make_operator(*fields))
    v = to_dev(W.random_vector((n, n), 2))
    dt = 300.0 / abs(alpha)

    def run(op):
        op.set_bound(alpha)
        out = torch.empty_like(v)
        st = op.leja_phi(1, dt, v, out, 1e-10)
        return to_np(out), st

    first = None
    for _ in range(2):
        ops = [make_pair(*fields)[1] for _ in range(80)]
        for op in ops:
            assert op.host_wait()
            out, st = run(op)
            if first is None:
                first = (out, st)
            assert np.array_equal(out, first[0]) and st == first[1]
        for op in ops:
            op.close()


@pytest.mark.parametrize("nx,ny", [(40, 3), (40, 4), (33, 5), (70, 6), (70, 7), (64, 8), (130, 9), (64, 10),
                                   (96, 11)])
def test_periodic_few_rows_sweeps_match_oracle(nx, ny):
    """Periodic grids with few rows: the four-term kernel's row rule wraps a
    row index once, so ny = 3, 4, 5 and 9 refuse four terms per launch (the
    default mode runs two); on the others mode 4 runs.  Every mode's phi_1
    sweep and quadrature step equal the oracle (same degree)."""
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=3 * nx + ny, field_advection=True)
    hx, hy = 1.0 / nx, 1.0 / ny
    oop, gop = make_pair(Dxx, Dxy, Dyy, ax, ay, hx, hy, O.PERIODIC)
    alpha = bounds.gershgorin(oop)
    gop.set_bound(alpha)
    v0 = W.random_vector((ny, nx), 9)
    v = to_dev(v0)
    dt = 400.0 / abs(alpha)
    four = ny not in (3, 4, 5, 9)
    if not four:
        with pytest.raises(A.AdlError) as e:
            gop.set_term_fusion(4)
        assert e.value.code == A.EINVAL
    st = {}
    ref = leja.phi_apply(lambda x: O.apply(oop, x), 1, dt, v0, alpha, 1e-10, stats=st)
    modes = (1, 0, 2, 3) + ((4,) if four else ()) + ((5, 6) if nx % 2 == 0 and nx >= 128 else ())
    for mode in modes:
        gop.set_term_fusion(mode)
        out = torch.empty_like(v)
        s = gop.leja_phi(1, dt, v, out, 1e-10)
        assert s["matvecs"] == st["matvecs"], (mode, s, st)
        assert rel(to_np(out), ref) < 1e-10, mode
    S1, S2 = W.random_vector((ny, nx), 4), W.random_vector((ny, nx), 6)
    A_ = lambda x: O.apply(oop, x)
    ost = {}
    uo = integrators.exp_quad2_step(A_, v0, S1, S2, 1.0 / 3.0, 2.0 / 3.0, dt, alpha, 1e-10, stats=ost)
    gop.set_term_fusion(1)
    ug = v.clone()
    s = gop.quad2_step(ug, to_dev(S1), to_dev(S2), 1.0 / 3.0, 2.0 / 3.0, dt, 1e-10)
    assert s["matvecs"] == ost["matvecs"]
    assert rel(to_np(ug), uo) < 1e-10
