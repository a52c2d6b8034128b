"""dl_observables_noalloc (no plan, no allocation: partial sums in the
library's static device array) against dl_observables of a plan on the same
state, through the raw C ABI: two calls in a row, the second on a smaller
input, for both dtypes and a two-component line; the values must carry the
same bits (same kernels, same partition of the cells)."""
import ctypes

import numpy as np
import pytest

from paper_1107_4650_amd import libdirac as L
from paper_1107_4650_amd.inputs import C_LIGHT, packet, random_spinor
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _with_plan(shape, dx, xmin, psi, x_b, dtype, bispinor=False):
    with L.Plan(shape, dx, dx / C_LIGHT, C_LIGHT, 1.0, dtype=dtype, xmin=xmin,
                bispinor=bispinor) as p:
        return p.observables(psi, x_b)


def _noalloc(lib, shape, dx, xmin, psi, x_b, dtype, bispinor=False):
    import torch
    g = L.make_grid(shape, xmin=xmin)
    out = torch.full((5,), float("nan"), dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.dl_observables_noalloc(ctypes.byref(g), dx, L._dtype_code(dtype),
                                    L.DL_BISPINOR if bispinor else 0,
                                    ctypes.c_void_p(psi.data_ptr()), x_b,
                                    ctypes.c_void_p(out.data_ptr()), st)
    assert rc == L.DL_OK, lib.dl_last_error()
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_observables_match_plan_observables():
    import torch
    lib = L.load()
    cases = [
        # (shape x-first, dtype, bispinor): the second input is smaller than the first
        (((300, 200), "c64", False), ((120,), "c128", False)),
        (((64, 40, 24), "c128", False), ((1000,), "c64", True)),
    ]
    for first, second in cases:
        for shape, dtype, pair in (first, second):
            announce(f"noalloc observables {shape} {dtype} pair={pair}")
            dx = 0.02
            xmin = [-0.5 * n * dx for n in shape]
            tdt = torch.complex64 if dtype == "c64" else torch.complex128
            if pair:
                arr = random_spinor(shape[::-1], seed=len(shape))[..., :2]
            elif len(shape) == 3:
                arr = random_spinor(shape[::-1], seed=3)
            else:
                arr = packet(shape, dx, delta=0.3, p0=[20.0] + [0.0] * (len(shape) - 1),
                             r0=[0.1] + [0.0] * (len(shape) - 1))
            psi = torch.from_numpy(np.ascontiguousarray(arr)).to("cuda").to(tdt)
            for x_b in (0.0, 0.37):
                ref = _with_plan(shape, dx, xmin, psi, x_b, dtype, pair)
                got = _noalloc(lib, shape, dx, xmin, psi, x_b, dtype, pair)
                assert np.array_equal(got, ref), (shape, dtype, x_b, got, ref)


def test_noalloc_observables_refusals():
    import torch
    lib = L.load()
    psi = torch.zeros((8, 4), dtype=torch.complex64, device="cuda")
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    g = L.make_grid((8,), xmin=[0.0])
    P = lambda t, off=0: ctypes.c_void_p(t.data_ptr() + off)  # noqa: E731
    assert lib.dl_observables_noalloc(None, 0.1, 0, 0, P(psi), 0.0, P(out), None) == L.DL_ERR_ARG
    assert lib.dl_observables_noalloc(ctypes.byref(g), -0.1, 0, 0, P(psi), 0.0, P(out),
                                      None) == L.DL_ERR_ARG
    assert lib.dl_observables_noalloc(ctypes.byref(g), 0.1, 5, 0, P(psi), 0.0, P(out),
                                      None) == L.DL_ERR_DTYPE
    assert lib.dl_observables_noalloc(ctypes.byref(g), 0.1, 0, 0, P(psi, 8), 0.0, P(out),
                                      None) == L.DL_ERR_ALIGN
    assert lib.dl_observables_noalloc(ctypes.byref(g), 0.1, 0, 0, P(psi), 0.0, P(out, 4),
                                      None) == L.DL_ERR_ALIGN
    assert lib.dl_observables_noalloc(ctypes.byref(g), 0.1, 0, 0, P(psi), 0.0, None,
                                      None) == L.DL_ERR_ARG
    big = L.make_grid((1 << 21, 1 << 20), xmin=[0.0, 0.0])
    assert lib.dl_observables_noalloc(ctypes.byref(big), 0.1, 0, 0, P(psi), 0.0, P(out),
                                      None) == L.DL_ERR_ARG
    assert b"2^40" in lib.dl_last_error()
    g2 = L.make_grid((8, 8), xmin=[0.0, 0.0])
    assert lib.dl_observables_noalloc(ctypes.byref(g2), 0.1, 0, L.DL_BISPINOR, P(psi), 0.0,
                                      P(out), None) == L.DL_ERR_ARG
