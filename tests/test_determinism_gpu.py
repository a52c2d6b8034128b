"""Determinism and tiling invariance of the HIP sweep (doubles as a race check):
the same run twice, every tiling, the resident and the tiled 1-D paths, graph
replay and n + n = 2n steps must all give identical bits."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1107_4650_amd.inputs import random_spinor, C_LIGHT
from tests.gpu_util import announce, gpu_step, same_bits, rel_l2

pytestmark = pytest.mark.gpu

C = C_LIGHT
DX = 0.01
DT = DX / C


def _V(shape, seed=5):
    return np.random.default_rng(seed).uniform(-2, 2, size=shape[::-1]) * C * C


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("shape", [(300, 260), (96, 40, 33)])
def test_tiling_invariance_and_repeatability(dtype, shape):
    announce(f"tilings {shape} {dtype}")
    axes = tuple(range(len(shape)))
    psi = random_spinor(shape[::-1], seed=1)
    V = _V(shape)
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, nsteps=25, axes=axes, dtype=dtype)
    base = gpu_step(psi, V, **kw)
    assert same_bits(base, gpu_step(psi, V, **kw))
    for tiling in ({"waves_per_cu": 1}, {"waves_per_cu": 4, "seg_len": 9},
                   {"waves_per_cu": 16, "seg_len": 5}, {"waves_per_cu": 2, "seg_len": 1000}):
        assert same_bits(base, gpu_step(psi, V, tiling=tiling, **kw)), tiling


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("n,bc", [(4096, "zero"), (1000, "zero"), (2048, "periodic"),
                                  (130, "zero")])
def test_resident_1d_equals_tiled(dtype, n, bc):
    announce(f"resident vs tiled n={n} {bc} {dtype}")
    psi = random_spinor((n,), seed=n)
    V = _V((n,))
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, nsteps=333, axes=(0,), bc=bc, dtype=dtype)
    res = gpu_step(psi, V, depth=2, **kw)  # passes of at most 2 steps: resident kernel
    tiled = gpu_step(psi, V, tiling={"allow_resident": False}, **kw)
    assert same_bits(res, tiled)
    if dtype == "c128":
        ref = O.step(psi, V, dt=DT, c=C, m=1.0, nsteps=333, axes=(0,), bc=bc)
        assert rel_l2(res, ref) <= 1e-12


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_graph_replay_and_resume(dtype):
    announce(f"graph and resume {dtype}")
    shape = (200, 150)
    psi = random_spinor(shape[::-1], seed=2)
    V = _V(shape)
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, axes=(0, 1), dtype=dtype)
    eager = gpu_step(psi, V, nsteps=150, **kw)
    graph = gpu_step(psi, V, nsteps=150, graph=True, tiling={"graph_pairs": 8}, **kw)
    assert same_bits(eager, graph)
    # replay the same captured graph on several calls, with eager work between them
    chunked = gpu_step(psi, V, nsteps=0, graph=True, tiling={"graph_pairs": 8},
                       chunks=[40, 16, 33, 16, 45], **kw)
    assert same_bits(eager, chunked)
    split = gpu_step(psi, V, nsteps=0, chunks=[75, 75], **kw)
    assert same_bits(eager, split)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("shape,axes,bc", [((300, 260), (0, 1), "zero"), ((130, 45), (0, 2), "periodic"),
                                           ((5000,), (1,), "zero"), ((4099,), (0,), "periodic"),
                                           ((63, 70), (1, 2), "periodic"), ((62, 9), (0, 1), "zero"),
                                           ((57, 8), (0, 1), "periodic"), ((200, 7), (0, 1), "periodic")])
def test_fused_passes_same_bits(dtype, shape, axes, bc):
    """Passes of 2 to 5 fused steps give the bits of single steps (counts
    that are and are not multiples of the depth, tilings, walls, wrap-around,
    periodic boxes too thin for the deepest pass)."""
    announce(f"fused passes {shape} {axes} {bc} {dtype}")
    psi = random_spinor(shape[::-1], seed=21)
    V = _V(shape, seed=22)
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, axes=axes, bc=bc, dtype=dtype,
              tiling={"allow_resident": False})
    depths = (2, 3, 4, 5)
    for n in (1, 2, 3, 7, 20):
        single = gpu_step(psi, V, nsteps=n, depth=1, **kw)
        for d in depths:
            assert same_bits(single, gpu_step(psi, V, nsteps=n, depth=d, **kw)), (n, d)
    massless = gpu_step(psi, None, nsteps=9, depth=1, **{**kw, "m": 0.0})
    for d in depths:
        assert same_bits(massless, gpu_step(psi, None, nsteps=9, depth=d, **{**kw, "m": 0.0}))


@pytest.mark.parametrize("pairs", [2, 7, 32])
def test_graph_replay_with_odd_pass_counts(pairs):
    """A captured group of 2 * pairs steps that takes an odd number of passes
    (4 steps: one pass of 4; 14: 5 + 5 + 4) ends in the plan's buffer; every
    replay must still leave the state where the next one starts."""
    announce(f"graph odd passes pairs={pairs}")
    shape = (130, 70)
    psi = random_spinor(shape[::-1], seed=14)
    V = _V(shape, seed=15)
    kw = dict(dx=DX, dt=DT, c=C, m=1.0, axes=(0, 1), dtype="c64")
    n = 4 * pairs + 3
    eager = gpu_step(psi, V, nsteps=n, **kw)
    graph = gpu_step(psi, V, nsteps=n, graph=True, tiling={"graph_pairs": pairs}, **kw)
    assert same_bits(eager, graph)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("shape,axes,scheme", [((64, 48, 40), (0, 1, 2), "lie"),
                                               ((200, 150), (0, 2), "strang")])
def test_graph_replay_of_3d_and_second_order_passes(dtype, shape, axes, scheme):
    """Graph capture and replay of fused 3-D passes and of second-order
    passes give the bits of the same steps run eagerly, over several calls
    with eager work between the replays."""
    announce(f"graph 3-D / strang {shape} {scheme} {dtype}")
    psi = random_spinor(shape[::-1], seed=12)
    V = _V(shape, seed=13)
    dt = (2 if scheme == "strang" else 1) * DT
    kw = dict(dx=DX, dt=dt, c=C, m=1.0, axes=axes, dtype=dtype, scheme=scheme)
    eager = gpu_step(psi, V, nsteps=101, **kw)
    graph = gpu_step(psi, V, nsteps=0, graph=True, tiling={"graph_pairs": 6},
                     chunks=[30, 24, 47], **kw)
    assert same_bits(eager, graph)


@pytest.mark.parametrize("shape,bc,seg", [((70, 13, 11), "zero", 0), ((130, 6, 21), "periodic", 4),
                                          ((61, 9, 5), "zero", 2), ((64, 64, 40), "zero", 7),
                                          ((3, 2, 2), "periodic", 0), ((2, 5, 3), "zero", 0),
                                          ((121, 4, 9), "periodic", 3), ((2, 2, 7), "periodic", 2)])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_fused_3d_passes_same_bits(shape, bc, seg, dtype):
    """3-D passes of two fused steps give the bits of single steps: ragged
    strips and row blocks, segments marching up and down, walls,
    wrap-around, boxes of two cells per axis; every phase mode."""
    announce(f"fused 3-D passes {shape} {bc} seg={seg} {dtype}")
    psi = random_spinor(shape[::-1], seed=31)
    V = _V(shape, seed=32)
    kw = dict(dx=DX, dt=DT, c=C, axes=(0, 1, 2), bc=bc, dtype=dtype,
              tiling={"seg_len": seg} if seg else None)
    for n in (1, 2, 3, 8):
        single = gpu_step(psi, V, m=1.0, nsteps=n, depth=1, **kw)
        assert same_bits(single, gpu_step(psi, V, m=1.0, nsteps=n, depth=2, **kw)), n
    for m in (0.0, 1.0):
        single = gpu_step(psi, None, m=m, nsteps=5, depth=1, **kw)
        assert same_bits(single, gpu_step(psi, None, m=m, nsteps=5, depth=2, **kw)), m


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_step_fused_out_matches_single_steps(dtype):
    import torch
    from paper_1107_4650_amd import libdirac as L
    announce(f"step_fused_out {dtype}")
    shape = (257, 130)
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    psi = torch.from_numpy(random_spinor(shape[::-1], seed=5)).to(tdt)
    V = torch.from_numpy(_V(shape)).to("cuda")
    with L.Plan(shape, DX, DT, C, 1.0, dtype=dtype) as p:
        a = psi.to("cuda")
        ref = [a]
        for _ in range(11):
            nxt = torch.empty_like(a)
            p.step_out(ref[-1], nxt, V)
            ref.append(nxt)
        for k in range(1, 12):
            d = torch.empty_like(a)
            p.step_fused_out(a, d, V, k)
            torch.cuda.synchronize()
            assert same_bits(ref[k].cpu().numpy(), d.cpu().numpy()), k
        assert same_bits(a.cpu().numpy(), psi.numpy())  # src untouched
