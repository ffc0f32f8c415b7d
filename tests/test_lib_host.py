"""CPU-only checks of the C-ABI library: it loads, exports every function the
public header declares, and its host-side logic (Leja points, Newton
coefficients, argument validation) agrees with the oracle.  No kernel is
launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import leja

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
A = pytest.importorskip("paper_2307_12276_amd")


def _lib():
    if not os.path.exists(A.LIB_PATH):
        pytest.skip("libadl.so not built")
    return A.lib()


def declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            src = open(os.path.join(inc, f)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^[A-Za-z_][\w \*]*?\b(adl_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("adl_op_create", "adl_apply", "adl_spectral_bound", "adl_leja_phi",
                 "adl_exp_midpoint_step", "adl_exp_quad2_step", "adl_batch_midpoint_step",
                 "adl_mlp_forward", "adl_mlp_backward", "adl_mlp_adam_step", "adl_field_stats"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(A.LIB_PATH) if os.path.exists(A.LIB_PATH) else pytest.skip("not built")
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # and the binding wraps exactly the declared set
    assert sorted(A.exported_symbols()) == declared_functions()


def test_leja_points_match_oracle():
    _lib()
    got = np.array(A.leja_points(501))
    ref = leja.leja_points(501)
    assert np.max(np.abs(got - ref)) <= 4 * np.finfo(float).eps * 2
    assert got[0] == 2.0 and got[1] == -2.0 and got[2] == 0.0


@pytest.mark.parametrize("l", [0, 1, 2])
@pytest.mark.parametrize("rho_h", [3.0, 100.0, 1600.0])
def test_newton_coefficients_match_oracle(l, rho_h):
    _lib()
    n = 200
    got = np.array(A.newton_coefficients(l, -rho_h, 1.0, n))
    ref = leja.newton_coefficients(l, -rho_h, 1.0, n)
    # the terms that matter: agreement relative to the largest coefficient
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_argument_validation_without_gpu():
    L = _lib()
    assert L.adl_workspace_bytes(2, 10, 0, 0) == 0
    assert L.adl_workspace_bytes(10, 10, 3, 0) == 0
    assert L.adl_workspace_bytes(10, 10, 0, 0) > 10 * 10 * 8 * 12
    h = ctypes.c_void_p()
    rc = L.adl_op_create(2, 10, 0.1, 0.1, 0, 0, None, None, None, None, None, 0.0, 0.0, None, 0, None,
                         ctypes.byref(h))
    assert rc == A.EINVAL and b"nx" in L.adl_last_error()
    rc = L.adl_op_create(10, 10, -0.1, 0.1, 0, 0, None, None, None, None, None, 0.0, 0.0, None, 0, None,
                         ctypes.byref(h))
    assert rc == A.EINVAL
    assert L.adl_leja_points(0, (ctypes.c_double * 1)()) == A.EINVAL
    assert L.adl_newton_coefficients(1, 1.0, 1.0, 5, (ctypes.c_double * 5)()) == A.EINVAL
    assert L.adl_apply(None, None, None, None) == A.EINVAL
    assert L.adl_set_bound(None, -1.0) == A.EINVAL
    assert L.adl_mlp_forward(None, None, None, None, 4, None) == A.EINVAL


def test_product_path_has_no_oracle_dependency():
    """The package and its C++ sources never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2307_12276_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.lower(), f


def test_xcd_block_order_is_a_bijection():
    """The staged two-term kernel's dispatch-to-logical block map (each XCD
    a contiguous range): a permutation of [0, n) that keeps block 0 (the
    decision block) first, restated here from its definition."""
    def f(bid, n):
        q, rem = n // 8, n % 8
        x, l = bid % 8, bid // 8
        return x * (q + 1) + l if x < rem else rem * (q + 1) + (x - rem) * q + l
    for n in (1, 2, 7, 8, 9, 15, 16, 17, 641, 3877, 4097):
        got = [f(b, n) for b in range(n)]
        assert sorted(got) == list(range(n)) and got[0] == 0
        # blocks dealt to one XCD are consecutive logical blocks
        for x in range(min(n, 8)):
            seq = [got[b] for b in range(x, n, 8)]
            assert seq == list(range(seq[0], seq[0] + len(seq)))


def test_four_term_rows_stay_inside_periodic_grids():
    """Row indices of a four-term launch, restated from the kernel: a block
    with output rows J0 .. J0 + 7 (J0 = 8 b <= ny - 1) computes stage 1 on
    rows J0 - 3 .. J0 + 10 and loads their neighbours, J0 - 4 .. J0 + 11; a
    periodic row index is wrapped once (r + ny below 0, r - ny from ny).
    The host's test for four terms per launch on a periodic grid (lowest row
    >= -ny, highest row of the last block <= 2 ny - 1) holds exactly where
    every load stays inside the grid: always from 11 rows up, never at
    ny = 3, 4, 5 and 9 (which run two terms per launch)."""
    def rows_inside(ny):
        for J0 in range(0, ny, 8):
            for r in range(J0 - 4, J0 + 12):
                m = r + ny if r < 0 else (r - ny if r >= ny else r)
                if not 0 <= m < ny:
                    return False
        return True

    def host_rule(ny):
        j0_last = 8 * ((ny - 1) // 8)
        return -4 >= -ny and j0_last + 8 - 1 + 4 <= 2 * ny - 1

    for ny in range(3, 300):
        assert rows_inside(ny) == host_rule(ny), ny
    assert [ny for ny in range(3, 300) if not rows_inside(ny)] == [3, 4, 5, 9]


def test_batch_errors_reach_last_error(capfd):
    """A rejected batch call reports through adl_last_error like every other
    entry point, and the library prints nothing."""
    L = _lib()
    h = ctypes.c_void_p()
    assert L.adl_op_set_limits(None, 10, 1.0) == A.EINVAL  # leaves a message of its own
    rc = L.adl_batch_create(0, None, None, 0, 0, ctypes.byref(h))
    assert rc == A.EINVAL
    assert b"nbins" in L.adl_last_error()
    assert L.adl_batch_set_tile_rows(None, 4) == A.EINVAL
    assert b"tile rows" in L.adl_last_error()
    out, err = capfd.readouterr()
    assert out == "" and err == ""
