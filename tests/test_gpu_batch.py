"""GPU parity of the batched bins path against the oracle, bin by bin."""
import numpy as np
import pytest

import workloads as W
from oracle import bounds, integrators
from oracle import operator as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12276_amd as A  # noqa: E402
from gpu_util import rel, to_dev, to_np, workload_pair  # noqa: E402


def make_batch(bins, tile_rows=0):
    pairs = [workload_pair(w) for w in bins]
    for (oop, gop) in pairs:
        gop.set_bound(bounds.gershgorin(oop))
    b = A.Batch([g for _, g in pairs], tile_rows=tile_rows)
    return pairs, b


def oracle_steps(w, oop, nsteps):
    alpha = bounds.gershgorin(oop)
    u = w.u0.copy()
    degs = []
    for n in range(nsteps):
        st = {}
        u = integrators.exp_midpoint_step(lambda x: O.apply(oop, x), u, w.S(0), w.dt, alpha, w.tol, stats=st)
        degs.append(st["matvecs"])
    return u, degs


# term fusion modes of the batched sweep: two terms per launch (True, the
# default), one (False), three with LDS-staged blocks (3)
MODES = [True, False, 3]


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("mode", MODES)
def test_batch_matches_oracle_per_bin(use_graph, mode):
    bins = W.c4_bins(nbins=10, sizes=(128, 130, 192, 256))
    pairs, b = make_batch(bins)
    b.set_term_fusion(mode)
    us = [to_dev(w.u0) for w in bins]
    Ss = [to_dev(w.S(0)) for w in bins]
    for step in range(2):
        stats = b.midpoint_step(us, Ss, bins[0].dt, bins[0].tol, use_graph=use_graph)
    for w, (oop, _), u, st in zip(bins, pairs, us, stats):
        ref, degs = oracle_steps(w, oop, 2)
        assert st["matvecs"] == degs[-1], (w.name, st, degs)
        assert rel(to_np(u), ref) < 1e-10, w.name


@pytest.mark.parametrize("mode", MODES)
def test_batch_zero_stage_vector_bin(mode):
    """A bin with u = 0 and no source has w = A u + S = 0: its sweep stops at
    degree 0 (the three-term first launch detects y_0 = 0 from its vanishing
    first term and p_1) and u stays 0, while the other bins match the
    oracle; same matvec counts as the oracle."""
    bins = W.c4_bins(nbins=4, sizes=(128, 192))
    bins[1].u0 = np.zeros_like(bins[1].u0)
    pairs, b = make_batch(bins)
    b.set_term_fusion(mode)
    us = [to_dev(w.u0) for w in bins]
    Ss = [to_dev(w.S(0)) for w in bins]
    Ss[1] = None
    stats = b.midpoint_step(us, Ss, bins[0].dt, bins[0].tol)
    for i, (w, (oop, _), u, st) in enumerate(zip(bins, pairs, us, stats)):
        ost = {}
        ref = integrators.exp_midpoint_step(lambda x: O.apply(oop, x), w.u0, None if i == 1 else w.S(0), w.dt,
                                            bounds.gershgorin(oop), w.tol, stats=ost)
        assert st["matvecs"] == ost["matvecs"], (i, st, ost)
        if i == 1:
            assert not torch.any(u) and st["max_degree"] == 0, st
        else:
            assert rel(to_np(u), ref) < 1e-10, i


@pytest.mark.parametrize("mode", MODES)
def test_batch_graph_replays_equal_eager(mode):
    bins = W.c4_bins(nbins=6, sizes=(128, 256))
    _, b1 = make_batch(bins)
    _, b2 = make_batch(bins)
    b1.set_term_fusion(mode)
    b2.set_term_fusion(mode)
    ua = [to_dev(w.u0) for w in bins]
    ub = [to_dev(w.u0) for w in bins]
    S = [to_dev(w.S(0)) for w in bins]
    for _ in range(4):
        b1.midpoint_step(ua, S, bins[0].dt, bins[0].tol, use_graph=True)
        torch.cuda.synchronize()
        b2.midpoint_step(ub, S, bins[0].dt, bins[0].tol, use_graph=False)
        torch.cuda.synchronize()
        for x, y in zip(ua, ub):
            assert torch.equal(x, y)


def test_batch_bound_state_steps_like_passed_state():
    """bind() once and step with us=None: the same results as passing the
    tensors every step; stepping without bound state is refused."""
    bins = W.c4_bins(nbins=5, sizes=(128, 192))
    _, b1 = make_batch(bins)
    _, b2 = make_batch(bins)
    ua = [to_dev(w.u0) for w in bins]
    ub = [to_dev(w.u0) for w in bins]
    S = [to_dev(w.S(0)) for w in bins]
    with pytest.raises(ValueError):
        b1.midpoint_step(None, None, bins[0].dt, bins[0].tol)
    b1.bind(ua, S)
    for _ in range(3):
        s1 = b1.midpoint_step(None, None, bins[0].dt, bins[0].tol)
        s2 = b2.midpoint_step(ub, S, bins[0].dt, bins[0].tol)
        assert [x["matvecs"] for x in s1] == [x["matvecs"] for x in s2]
    torch.cuda.synchronize()
    for x, y in zip(ua, ub):
        assert torch.equal(x, y)
    b1.bind(None, None)
    with pytest.raises(ValueError):
        b1.midpoint_step(None, None, bins[0].dt, bins[0].tol)


def varied_bins(shapes, bcs, field_adv, seed):
    """Bins with smooth random coefficient fields, random u0 and source, the
    given shapes and boundary conditions, field or constant advection, and a
    shared dt = 50 min dt_CFL."""
    bins = []
    for i, ((nx, ny), bc) in enumerate(zip(shapes, bcs)):
        Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed + i, field_advection=field_adv)
        _, _, hx, hy = W.grid_2d(nx, ny, bc)
        u0 = W.random_vector((ny, nx), seed + 100 + i)
        S = 0.1 * W.random_vector((ny, nx), seed + 200 + i)
        bins.append(W.Workload("varied%d-%dx%d" % (i, nx, ny), nx, ny, hx, hy, bc, Dxx, Dxy, Dyy,
                               ax if field_adv else None, ay if field_adv else None,
                               0.0 if field_adv else ax, 0.0 if field_adv else ay, u0, 0.0, 2, 1e-10,
                               "midpoint", 0.5, 0.5, lambda t, S=S: S))
    dt = 50.0 * min(W.cfl_dt(w.Dxx, w.Dyy, w.hx, w.hy) for w in bins)
    for w in bins:
        w.dt = dt
    return bins


# (shapes, boundary conditions, field advection, storage, tile rows): odd
# widths take one column per lane; odd tile heights and ragged last tiles
# take the marching tiles' single-row tail step
VARIED = {
    "periodic-field-adv-fp64-vec1": ([(97, 64), (64, 33), (33, 20)], [O.PERIODIC] * 3, True, 0, 5),
    "dirichlet-field-adv-fp32-vec2": ([(128, 45), (130, 70), (256, 19)], [O.DIRICHLET] * 3, True, 1, 7),
    "mixed-bc-const-adv-fp32-vec2": ([(128, 37), (256, 20), (192, 9)], [O.PERIODIC, O.DIRICHLET, O.PERIODIC],
                                     False, 1, 3),
    "periodic-field-adv-fp64-vec2": ([(128, 40), (256, 33), (192, 17)], [O.PERIODIC] * 3, True, 0, 5),
    "dirichlet-whole-strip-fp64-vec2": ([(128, 64), (128, 23), (384, 30)], [O.DIRICHLET] * 3, False, 0, 4),
}


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("case", sorted(VARIED))
def test_batch_varied_bins_match_oracle(case, mode):
    """Batched bins beyond the C4 layout (periodic and mixed boundaries,
    field advection, FP32 fields, odd widths, odd tile heights) against the
    oracle bin by bin over two midpoint steps: same matvec count, 1e-10.
    Three terms per launch need every bin at two columns per lane: a batch
    with an odd or narrow bin refuses them (ADL_EINVAL)."""
    shapes, bcs, field_adv, storage, rows = VARIED[case]
    bins = varied_bins(shapes, bcs, field_adv, seed=len(case))
    pairs = [workload_pair(w, storage) for w in bins]
    alphas = [bounds.gershgorin(oop) for oop, _ in pairs]
    for (oop, gop), a in zip(pairs, alphas):
        gop.set_bound(a)
    b = A.Batch([g for _, g in pairs], tile_rows=rows)
    if mode == 3 and any(w.nx % 2 or w.nx < 128 for w in bins):
        with pytest.raises(A.AdlError) as e:
            b.set_term_fusion(mode)
        assert e.value.code == A.EINVAL
        return
    b.set_term_fusion(mode)
    us = [to_dev(w.u0) for w in bins]
    Ss = [to_dev(w.S(0)) for w in bins]
    for _ in range(2):
        stats = b.midpoint_step(us, Ss, bins[0].dt, bins[0].tol)
    for w, (oop, _), a, u, st in zip(bins, pairs, alphas, us, stats):
        ref = w.u0.copy()
        for _ in range(2):
            ost = {}
            ref = integrators.exp_midpoint_step(lambda x: O.apply(oop, x), ref, w.S(0), w.dt, a, w.tol, stats=ost)
        assert st["substeps"] == 1, (w.name, st)  # advanced by the batched kernels
        assert st["fallback"] == 0 and st["matvecs"] == ost["matvecs"], (w.name, st, ost)
        assert rel(to_np(u), ref) < 1e-10, (w.name, rel(to_np(u), ref))


def test_batch_fallback_bins_and_autotune():
    """A bin whose step needs substeps, a source-free bin and a zero operator
    are advanced by the single-op path inside the same call."""
    bins = W.c4_bins(nbins=4, sizes=(128, 192))
    z = bins[3]
    z.Dxx = np.zeros_like(z.Dxx); z.Dxy = np.zeros_like(z.Dxy); z.Dyy = np.zeros_like(z.Dyy); z.ax_c = 0.0
    pairs = [workload_pair(w) for w in bins]
    for (oop, gop) in pairs:
        gop.set_bound(bounds.gershgorin(oop))
    pairs[0][1].set_limits(500, 0.1)  # bin 0: rho dt > 0.1 -> substeps
    b = A.Batch([g for _, g in pairs])
    us = [to_dev(w.u0) for w in bins]
    Ss = [to_dev(w.S(0)) for w in bins]
    Ss[1] = None
    best, ms = b.autotune(us, Ss, bins[0].dt, bins[0].tol, candidates=(2, 8, 16))
    assert best in (2, 8, 16) and ms > 0
    assert all(torch.equal(u, to_dev(w.u0)) for u, w in zip(us, bins))  # autotune leaves u alone
    # the result is cached by (architecture, storage, advection, shapes,
    # candidates): the same key again, on this batch or another one, installs
    # the cached height and time without timing
    b.set_tile_rows(4)
    assert b.autotune(us, Ss, bins[0].dt, bins[0].tol, candidates=(2, 8, 16)) == (best, ms)
    assert b.get_tile_rows() == best
    b2 = A.Batch([g for _, g in pairs])
    assert b2.autotune(us, Ss, bins[0].dt, bins[0].tol, candidates=(2, 8, 16)) == (best, ms)
    b2.close()
    _, ms3 = b.autotune(us, Ss, bins[0].dt, bins[0].tol, candidates=(8, 2, 16))  # another key: timed
    assert ms3 != ms
    stats = b.midpoint_step(us, Ss, bins[0].dt, bins[0].tol)
    assert stats[0]["substeps"] > 1
    for i, (w, (oop, _), u) in enumerate(zip(bins, pairs, us)):
        alpha = bounds.gershgorin(oop)
        S = None if i == 1 else w.S(0)
        rho_max = 0.1 if i == 0 else 1600.0
        ref = integrators.exp_midpoint_step(lambda x: O.apply(oop, x), w.u0, S, w.dt, alpha, w.tol, rho_max=rho_max)
        assert rel(to_np(u), ref) < 1e-10, i


def test_batch_full_config_sampled_bins():
    """256 bins (grid sizes from {128,...,512}^2, k_par = p^0.5): one batched
    step; bins 0 (softest), 255 (stiffest) and the largest are checked
    against the oracle one by one."""
    bins = W.c4_bins()
    pairs = [workload_pair(w) for w in bins]
    alphas = [bounds.gershgorin(oop) for oop, _ in pairs]
    for (oop, gop), a in zip(pairs, alphas):
        gop.set_bound(a)
    b = A.Batch([g for _, g in pairs])
    us = [to_dev(w.u0) for w in bins]
    Ss = [to_dev(w.S(0)) for w in bins]
    stats = b.midpoint_step(us, Ss, bins[0].dt, bins[0].tol)
    largest = max(range(256), key=lambda i: bins[i].nx * bins[i].ny)
    for i in (0, 255, largest):
        w, (oop, _) = bins[i], pairs[i]
        st = {}
        ref = integrators.exp_midpoint_step(lambda x: O.apply(oop, x), w.u0, w.S(0), w.dt, alphas[i], w.tol, stats=st)
        assert stats[i]["matvecs"] == st["matvecs"]
        assert rel(to_np(us[i]), ref) < 1e-10, i
    assert all(s["status"] == 0 for s in stats)


@pytest.mark.parametrize("mode", [True, 3])
def test_batch_all_bins_equal_single_op_steps(mode):
    """The chosen form on the 256-bin workload (FP32 fields, learned
    intervals, two or three terms per launch, eager launches): three batched
    steps equal, bin by bin, the same steps taken by each bin's own operator
    (same fields, same intervals; the single-op path equals the oracle).
    Every bin is advanced exactly once per step, whichever launch its update
    falls in (a bin is advanced by its tiles in the launch after the one
    whose decision stopped it, or by the step's last launch), and with
    whichever term of its last launch it stopped at (with three terms per
    launch the degrees cover all three positions)."""
    from paper_2307_12276_amd import learned
    bins = W.c4_bins()
    dt = bins[0].dt
    tol = 1e-9
    Ss = [to_dev(w.S(0)) for w in bins]
    ops = [A.Op(to_dev(w.Dxx), to_dev(w.Dxy), to_dev(w.Dyy), w.hx, w.hy, w.bc, A.STORAGE_FP32_FIELDS,
                ax_c=w.ax_c, ay_c=w.ay_c) for w in bins]
    b = A.Batch(ops)
    b.set_term_fusion(mode)
    b.learned_bound(dt, torch.from_numpy(learned.load()).cuda(),
                    torch.empty(72 * len(ops), dtype=torch.float32, device="cuda"))
    ub = [to_dev(w.u0) for w in bins]
    us = [to_dev(w.u0) for w in bins]
    b.bind(ub, Ss)
    positions = set()
    for step in range(3):
        st = b.midpoint_step(None, None, dt, tol, use_graph=False).array
        for op, u, S in zip(ops, us, Ss):
            op.midpoint_step(u, S, dt, tol)
        d = [float(torch.linalg.vector_norm(x - y) / torch.linalg.vector_norm(y)) for x, y in zip(ub, us)]
        worst = int(np.argmax(d))
        print("step %d: max rel diff %.2e (bin %d, %d matvecs)" % (step, d[worst], worst, int(st["matvecs"][worst])))
        assert max(d) < 1e-12, (step, worst, d[worst])
        # degree m = matvecs - 1; three-term launches hold terms 1-3, 4-6,
        # ...: (m - 1) % 3 is the stopping term's place in its launch
        positions |= {(int(mv) - 1 - 1) % 3 for mv in st["matvecs"] if mv - 1 >= 1}
    if mode == 3:
        assert positions == {0, 1, 2}, positions
