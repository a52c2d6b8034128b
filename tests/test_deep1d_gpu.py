"""1-D lines run passes of 24 lowest-order steps (each wave writing the middle
16 of its 64 cells) before the plan's shallower passes: the same bits as
single steps on long and short lines, both walls, every axis, both state
types, every phase mode without a vector potential, and two-component lines."""
import numpy as np
import pytest

from paper_1107_4650_amd import libdirac as L
from paper_1107_4650_amd.inputs import random_spinor, C_LIGHT
from tests.gpu_util import announce, gpu_step, same_bits

pytestmark = pytest.mark.gpu

C = C_LIGHT
DX = 0.01
DT = DX / C


@pytest.mark.parametrize("n,axis,bc", [(4096, 0, "zero"), (777, 1, "periodic"), (50, 2, "zero"),
                                       (20, 0, "periodic"), (10000, 2, "periodic")])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_deep_passes_keep_single_step_bits(n, axis, bc, dtype):
    announce(f"deep 1-D n={n} axis={axis} {bc} {dtype}")
    psi = random_spinor((n,), seed=n)
    V = np.random.default_rng(n).uniform(-3, 3, size=(n,)) * C * C
    kw = dict(dx=DX, dt=DT, c=C, axes=(axis,), bc=bc, dtype=dtype)
    with L.Plan((n,), DX, DT, C, 1.0, dtype=dtype, bc=bc, axes=(axis,)) as p:
        assert p.info()["deep_1d_depth"] == 24
    for nsteps in (24, 50, 75):
        single = gpu_step(psi, V, m=1.0, nsteps=nsteps, depth=1,
                          tiling={"allow_resident": False}, **kw)
        assert same_bits(gpu_step(psi, V, m=1.0, nsteps=nsteps, **kw), single), nsteps
    for m, Vm in ((1.0, None), (0.0, None)):  # constant mass phase; pure streaming
        single = gpu_step(psi, Vm, m=m, nsteps=49, depth=1, tiling={"allow_resident": False},
                          **kw)
        assert same_bits(gpu_step(psi, Vm, m=m, nsteps=49, **kw), single), m


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_deep_passes_two_component_line(dtype):
    import torch
    announce(f"deep 1-D bispinor {dtype}")
    n = 3001
    full = random_spinor((n,), seed=3)
    pair = np.ascontiguousarray(full[:, [0, 3]])
    V = np.random.default_rng(4).uniform(-2, 2, size=(n,)) * C * C
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    tV = torch.from_numpy(V).to("cuda")
    out = []
    for depth in (1, None):
        t = torch.from_numpy(pair).to("cuda").to(tdt).contiguous()
        with L.Plan((n,), DX, DT, C, 1.0, dtype=dtype, bispinor=True) as p:
            if depth is not None:
                p.set_depth(depth)
                p.set_tiling(allow_resident=False)
            else:
                assert p.info()["deep_1d_depth"] == 24
            p.step(t, tV, 53)
            torch.cuda.synchronize()
        out.append(t.cpu().numpy())
    assert same_bits(out[1], out[0])


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_deep_passes_in_graph_replays(dtype):
    """Graph replays of 2 x 32 steps (two deep passes and the shallow rest) give
    the bits of single steps."""
    announce(f"deep 1-D graph {dtype}")
    n = 4096
    psi = random_spinor((n,), seed=11)
    V = np.random.default_rng(12).uniform(-3, 3, size=(n,)) * C * C
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, axes=(0,), dtype=dtype)
    single = gpu_step(psi, V, nsteps=200, depth=1, tiling={"allow_resident": False}, **kw)
    assert same_bits(gpu_step(psi, V, nsteps=200, graph=True, **kw), single)
