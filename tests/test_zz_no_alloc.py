"""The allocation-free entry point adl_gershgorin_bound_noalloc (through the
C ABI) against adl_spectral_bound(ADL_BOUND_GERSHGORIN) on an FP64 op of the
same fields: the same value, bit for bit (same reduction, same order), on
two calls in a row that share the library's static scratch, the second on
a smaller grid; rejected arguments leave a message."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_12276_amd as A  # noqa: E402
from gpu_util import to_dev  # noqa: E402


def case(nx, ny, bc, field_adv, seed):
    Dxx, Dxy, Dyy, ax, ay = W.random_fields(nx, ny, seed=seed, field_advection=field_adv)
    hx, hy = 1.0 / nx, 0.7 / ny
    if not field_adv:
        ax, ay = 0.3, -0.2
    return Dxx, Dxy, Dyy, ax, ay, hx, hy, bc


def reference(c):
    Dxx, Dxy, Dyy, ax, ay, hx, hy, bc = c
    if np.isscalar(ax):
        op = A.Op(to_dev(Dxx), to_dev(Dxy), to_dev(Dyy), hx, hy, bc, A.STORAGE_FP64, ax_c=ax, ay_c=ay)
    else:
        op = A.Op(to_dev(Dxx), to_dev(Dxy), to_dev(Dyy), hx, hy, bc, A.STORAGE_FP64, ax=to_dev(ax), ay=to_dev(ay))
    a, _ = op.spectral_bound(A.BOUND_GERSHGORIN)
    op.close()
    return a


def noalloc(c, out):
    Dxx, Dxy, Dyy, ax, ay, hx, hy, bc = c
    if np.isscalar(ax):
        A.gershgorin_bound_noalloc(to_dev(Dxx), to_dev(Dxy), to_dev(Dyy), hx, hy, bc, out, ax_c=ax, ay_c=ay)
    else:
        A.gershgorin_bound_noalloc(to_dev(Dxx), to_dev(Dxy), to_dev(Dyy), hx, hy, bc, out, ax=to_dev(ax),
                                   ay=to_dev(ay))


def test_noalloc_gershgorin_matches_spectral_bound():
    cases = [case(700, 450, W.DIRICHLET, True, 3), case(64, 40, W.PERIODIC, False, 4)]
    refs = [reference(c) for c in cases]
    outs = [torch.full((1,), float("nan"), dtype=torch.float64, device="cuda") for _ in cases]
    for c, o in zip(cases, outs):  # two calls in a row, the second on a smaller grid
        noalloc(c, o)
    torch.cuda.synchronize()
    got = [float(o.item()) for o in outs]
    print("Gershgorin: no-alloc %s, op %s" % (got, refs))
    assert got == refs
    # the first call's scratch contents do not leak into a repeat of the second
    o2 = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    noalloc(cases[1], o2)
    assert float(o2.item()) == refs[1]


def test_noalloc_rejects_bad_arguments():
    L = A.lib()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    z = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    p = ctypes.c_void_p(z.data_ptr())
    rc = L.adl_gershgorin_bound_noalloc(2, 4, 0.1, 0.1, 0, p, p, p, None, None, 0.0, 0.0,
                                        ctypes.c_void_p(out.data_ptr()), None)
    assert rc == A.EINVAL and b"nx" in L.adl_last_error()
    rc = L.adl_gershgorin_bound_noalloc(4, 4, 0.1, 0.1, 0, p, p, p, None, None, 0.0, 0.0, None, None)
    assert rc == A.EINVAL and b"alpha_out" in L.adl_last_error()
    rc = L.adl_gershgorin_bound_noalloc(4, 4, 0.1, 0.1, 0, p, p, p, p, None, 0.0, 0.0,
                                        ctypes.c_void_p(out.data_ptr()), None)
    assert rc == A.EINVAL
