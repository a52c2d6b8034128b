"""A time-dependent vector potential (a laser pulse with a linear turn-on ramp,
A(t, x) = f(t) P(x)) through dl_step_pulse, against the oracle's pulse step
(whose per-step field integrals come from Gauss-Legendre quadrature, the
library's from a closed form): relative L2 1e-12 with FP64 state, 5e-6 with
FP32 state, over runs that cross the envelope's corners; passes of 1, 2 and 3
fused steps give the same bits (and 3-D second-order groups of 1, 2 and 5
steps); refused arguments."""
import ctypes

import numpy as np
import pytest

from oracle import oracle as O
from paper_1107_4650_amd import libdirac as L
from paper_1107_4650_amd.inputs import C_LIGHT, packet, random_spinor
from tests.gpu_util import announce, rel_l2, same_bits

pytestmark = pytest.mark.gpu

C = C_LIGHT
DX = 0.01
TOL = {"c128": 1e-12, "c64": 5e-6}


def _pulse(dt, nsteps):
    # ramp up over the first third of the run, a short plateau, ramp down;
    # a carrier of a few periods over the run
    T = nsteps * dt
    return dict(omega=2 * np.pi * 4.0 / T, phase=0.3, t_on=0.3 * T, t_flat=0.15 * T,
                t_off=0.35 * T)


def _profile(shape, amp=(3000.0, -2000.0, 1500.0)):
    ng = shape[::-1]
    P = np.zeros((3,) + ng)
    X = np.linspace(-1.0, 1.0, shape[0])
    for d in range(3):
        P[d] = amp[d] * (1.0 + 0.3 * np.sin(np.pi * X))  # broadcast along x
    return P


def _gpu(psi, V, P, pulse, *, t0, dt, nsteps, axes, bc="zero", dtype="c128", scheme="lie",
         depth=None, chunks=None):
    import torch
    shape = tuple(reversed(psi.shape[:-1]))
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    t = torch.from_numpy(np.ascontiguousarray(psi)).to("cuda").to(tdt)
    tV = None if V is None else torch.from_numpy(np.ascontiguousarray(V)).to("cuda")
    tP = torch.from_numpy(np.ascontiguousarray(P)).to("cuda")
    with L.Plan(shape, DX, dt, C, 1.0, dtype=dtype, bc=bc, axes=axes, scheme=scheme) as p:
        if depth is not None:
            p.set_depth(depth)
        if chunks:
            done = 0
            for k in chunks:
                p.step_pulse(t, tV, tP, pulse, t0 + done * dt, k)
                done += k
        else:
            p.step_pulse(t, tV, tP, pulse, t0, nsteps)
        torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [((300,), (0,), "zero", "lie"), ((96, 70), (0, 1), "zero", "lie"),
         ((90, 64), (0, 2), "periodic", "lie"), ((80, 66), (1, 2), "zero", "lie"),
         ((96, 70), (0, 1), "zero", "strang"), ((40, 24, 18), (0, 1, 2), "zero", "lie"),
         ((40, 24, 18), (0, 1, 2), "zero", "strang"), ((33, 20, 12), (0, 1, 2), "periodic", "strang")]


@pytest.mark.parametrize("shape,axes,bc,scheme", CASES,
                         ids=[f"{'x'.join(map(str, c[0]))}-{c[2]}-{c[3]}" for c in CASES])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_pulse_vs_oracle(shape, axes, bc, scheme, dtype):
    announce(f"pulse {shape} {axes} {bc} {scheme} {dtype}")
    dt = (1 if scheme == "lie" else (2 if len(shape) < 3 else 4)) * DX / C
    nsteps = 60
    psi = packet(shape, DX, delta=0.15, p0=[25.0] + [5.0] * (len(shape) - 1),
                 r0=[0.0] * len(shape))
    V = np.random.default_rng(5).uniform(-0.5, 0.5, shape[::-1]) * C * C
    P = _profile(shape)
    pulse = _pulse(dt, nsteps)
    t0 = -0.1 * nsteps * dt  # the run starts before the pulse does
    ref = O.step_pulse(psi, V, P, pulse, t0=t0, dt=dt, c=C, m=1.0, nsteps=nsteps, axes=axes,
                       bc=bc, scheme=scheme)
    src = psi if dtype == "c128" else psi.astype(np.complex64)
    got = _gpu(src, V, P, pulse, t0=t0, dt=dt, nsteps=nsteps, axes=axes, bc=bc, dtype=dtype,
               scheme=scheme)
    err = rel_l2(got, ref)
    announce(f"rel-L2 {err:.3e}")
    assert err <= TOL[dtype]
    # the pulse acted: the field-free run is far from it
    free = O.step(psi, V, dt=dt, c=C, m=1.0, nsteps=nsteps, axes=axes, bc=bc) \
        if scheme == "lie" else O.step_strang(psi, V, dt=dt, c=C, m=1.0, nsteps=nsteps, axes=axes,
                                             bc=bc)
    assert rel_l2(free, ref) > 1e-3


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_pulse_fused_passes_keep_the_bits(dtype):
    """Passes of 1, 2 and 3 steps (and a run split over calls at a step
    boundary) give the same bits: each step's time comes from its index."""
    announce(f"pulse fusion {dtype}")
    shape, axes = (130, 45), (0, 1)
    dt = DX / C
    nsteps = 37
    psi = random_spinor(shape[::-1], seed=2)
    if dtype == "c64":
        psi = psi.astype(np.complex64)
    V = np.random.default_rng(1).uniform(-1, 1, shape[::-1]) * C * C
    P = _profile(shape)
    pulse = _pulse(dt, nsteps)
    runs = [_gpu(psi, V, P, pulse, t0=0.0, dt=dt, nsteps=nsteps, axes=axes, dtype=dtype,
                 depth=d) for d in (1, 2, 3)]
    assert same_bits(runs[0], runs[1]) and same_bits(runs[0], runs[2])
    split = _gpu(psi, V, P, pulse, t0=0.0, dt=dt, nsteps=nsteps, axes=axes, dtype=dtype,
                 chunks=[12, 25])
    assert rel_l2(split, runs[0]) <= (1e-14 if dtype == "c128" else 1e-6)


def test_pulse_refusals():
    import torch
    announce("pulse refusals")
    lib = L.load()
    shape = (64, 32)
    psi = torch.zeros((32, 64, 4), dtype=torch.complex64, device="cuda")
    P = torch.zeros((3, 32, 64), dtype=torch.float64, device="cuda")
    ok = L.Pulse(1.0, 0.0, 1.0, 1.0, 1.0)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    with L.Plan(shape, DX, DX / C, C, 1.0, dtype="c64") as p:
        h = p.handle
        assert lib.dl_step_pulse(h, vp(psi), None, vp(P), ctypes.byref(ok), 0.0, 3, None) == L.DL_OK
        for bad in (L.Pulse(1.0, 0.0, -1.0, 1.0, 1.0), L.Pulse(float("nan"), 0.0, 1.0, 1.0, 1.0),
                    L.Pulse(1.0, 0.0, 1.0, float("inf"), 1.0)):
            assert lib.dl_step_pulse(h, vp(psi), None, vp(P), ctypes.byref(bad), 0.0, 3,
                                     None) == L.DL_ERR_ARG
        assert lib.dl_step_pulse(h, vp(psi), None, None, ctypes.byref(ok), 0.0, 3,
                                 None) == L.DL_ERR_ARG
        assert lib.dl_step_pulse(h, vp(psi), None, vp(P), None, 0.0, 3, None) == L.DL_ERR_ARG
        assert lib.dl_step_pulse(h, vp(psi), None, vp(P), ctypes.byref(ok), float("nan"), 3,
                                 None) == L.DL_ERR_ARG
        assert lib.dl_step_pulse(h, vp(psi), None, vp(P), ctypes.byref(ok), 0.0, -1,
                                 None) == L.DL_ERR_ARG


def test_pulse_3d_second_order_groups_keep_the_bits():
    """3-D second-order plans: groups of 1, 2 and 5 steps per call of the
    fused passes give the same bits; a run split over two calls agrees."""
    announce("pulse 3-D second-order grouping")
    shape, axes = (36, 20, 14), (0, 1, 2)
    dt = 4 * DX / C
    nsteps = 11
    psi = random_spinor(shape[::-1], seed=4).astype(np.complex64)
    V = np.random.default_rng(2).uniform(-1, 1, shape[::-1]) * C * C
    P = _profile(shape)
    pulse = _pulse(dt, nsteps)
    kw = dict(t0=-dt, dt=dt, nsteps=nsteps, axes=axes, dtype="c64", scheme="strang")
    runs = [_gpu(psi, V, P, pulse, depth=d, **kw) for d in (1, 2, 5)]
    assert same_bits(runs[0], runs[1]) and same_bits(runs[0], runs[2])
    # the second call starts from t0 + 4 dt, whose rounding can move F_n by an ulp
    split = _gpu(psi, V, P, pulse, chunks=[4, 7], **kw)
    assert rel_l2(split, runs[0]) <= 1e-6
