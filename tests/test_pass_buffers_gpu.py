"""Step calls whose passes end in psi through the plan's third state buffer
(an odd number, three or more, of passes) keep the bits of single steps, in
eager calls, repeated calls on one plan, graph replays and 3-D plans."""
import numpy as np
import pytest

from paper_1107_4650_amd.inputs import random_spinor, C_LIGHT
from tests.gpu_util import announce, gpu_step, same_bits

pytestmark = pytest.mark.gpu

C = C_LIGHT
DX = 0.01
DT = DX / C


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("nsteps,depth", [(11, None), (13, None), (15, None), (3, 1), (9, 3)])
def test_odd_pass_counts_keep_single_step_bits(dtype, nsteps, depth):
    announce(f"odd passes n={nsteps} depth={depth} {dtype}")
    shape = (150, 97)
    psi = random_spinor(shape[::-1], seed=nsteps)
    V = np.random.default_rng(nsteps).uniform(-3, 3, size=shape[::-1]) * C * C
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, axes=(0, 1), dtype=dtype, depth=depth)
    ref = gpu_step(psi, V, nsteps=nsteps, chunks=[1] * nsteps, **kw)
    got = gpu_step(psi, V, nsteps=nsteps, **kw)
    assert same_bits(got, ref)
    # the same plan twice (the buffer is reused), and a mix of pass counts
    got2 = gpu_step(psi, V, nsteps=3 * nsteps, chunks=[nsteps, nsteps + 1, nsteps - 1], **kw)
    ref2 = gpu_step(psi, V, nsteps=3 * nsteps, chunks=[1] * (3 * nsteps), **kw)
    assert same_bits(got2, ref2)


def test_odd_pass_counts_in_graph_replays():
    """2 x 6 steps per graph are three passes at depth 5: every replay ends in psi."""
    announce("odd passes graph")
    shape = (128, 90)
    psi = random_spinor(shape[::-1], seed=5)
    V = np.random.default_rng(6).uniform(-1, 1, size=shape[::-1]) * C * C
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, axes=(0, 1), dtype="c64")
    ref = gpu_step(psi, V, nsteps=29, chunks=[1] * 29, **kw)
    got = gpu_step(psi, V, nsteps=29, graph=True, tiling={"graph_pairs": 6}, **kw)
    assert same_bits(got, ref)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_odd_pass_counts_3d(dtype):
    announce(f"odd passes 3-D {dtype}")
    shape = (70, 13, 11)
    psi = random_spinor(shape[::-1], seed=13)
    V = np.random.default_rng(7).uniform(-1, 1, size=shape[::-1]) * C * C
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, axes=(0, 1, 2), dtype=dtype)
    ref = gpu_step(psi, V, nsteps=5, chunks=[1] * 5, **kw)
    got = gpu_step(psi, V, nsteps=5, **kw)
    assert same_bits(got, ref)
