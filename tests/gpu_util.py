"""Helpers for GPU parity tests: build the same seeded inputs for the oracle
and the HIP path (through the C-ABI binding)."""
import numpy as np

import workloads as W
from oracle import operator as O


def torch_dev():
    import torch
    return torch.device("cuda", 0)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(torch_dev())


def to_np(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def round32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def make_pair(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc, storage=0):
    """(oracle operator, GPU op).  ax/ay: scalars (constant) or arrays (field).
    For FP32 storage the oracle operator uses the same FP32-rounded scaled
    coefficients (so parity checks the kernels, not the rounding)."""
    import paper_2307_12276_amd as A
    const_adv = np.isscalar(ax)
    if storage == 0:
        oop = O.make_operator(Dxx, Dxy, Dyy, ax, ay, hx, hy, bc)
    else:
        sxx, syy, sxy = 1 / (hx * hx), 1 / (hy * hy), 1 / (4 * hx * hy)
        r = lambda a, s: round32(np.asarray(a) * s) / s
        if const_adv:
            oax, oay = ax, ay
        else:
            oax, oay = r(ax, 1 / (2 * hx)), r(ay, 1 / (2 * hy))
        oop = O.make_operator(r(Dxx, sxx), r(Dxy, sxy), r(Dyy, syy), oax, oay, hx, hy, bc)
    if const_adv:
        gop = A.Op(to_dev(Dxx), to_dev(Dxy), to_dev(Dyy), hx, hy, bc, storage, ax_c=ax, ay_c=ay)
    else:
        gop = A.Op(to_dev(Dxx), to_dev(Dxy), to_dev(Dyy), hx, hy, bc, storage, ax=to_dev(ax), ay=to_dev(ay))
    return oop, gop


def workload_pair(w, storage=None):
    st = w.storage if storage is None else storage
    ax = w.ax if w.ax is not None else w.ax_c
    ay = w.ay if w.ay is not None else w.ay_c
    return make_pair(w.Dxx, w.Dxy, w.Dyy, ax, ay, w.hx, w.hy, w.bc, st)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
