"""Batched launches: every instance of a mixed 1-D / 2-D batch matches the FP64
oracle's run of that instance (relative L2 1e-12 for complex128 state, 5e-6 for
complex64) and ends bit-identical to the same instance advanced alone with
dl_step, for uneven step counts (odd, even, zero), both dtypes, with and
without graphs, whether an instance runs whole in the lines kernel or pass by
pass over tiles, at every pass depth, and after autotuning (which must leave
the caller's states untouched and records its choice in the cache file)."""
import numpy as np
import pytest

from paper_1107_4650_amd import libdirac as L
from paper_1107_4650_amd.inputs import config_batch, C_LIGHT
from tests.gpu_util import announce, rel_l2, same_bits

pytestmark = pytest.mark.gpu

# relative L2 bars against the FP64 oracle: complex128 state differs from it by
# sine / cosine roundings only; complex64 state by about one FP32 rounding per
# component per step, over at most 150 steps here
ORACLE_TOL = {"c128": 1e-12, "c64": 5e-6}


def check_oracle(psi0, V, nsteps, got, *, dt, c, m, axes, bc, dtype, what):
    """The batched result `got` of one instance against the oracle's run of
    the same instance from the same (already rounded) initial state."""
    from oracle import oracle as O
    start = np.asarray(psi0).astype(np.complex128)
    if nsteps == 0:
        assert same_bits(got, np.asarray(psi0)), what
        return 0.0
    ref = O.step(start, V, dt=dt, c=c, m=m, nsteps=nsteps, axes=axes, bc=bc)
    err = rel_l2(got, ref)
    assert err <= ORACLE_TOL[dtype], (what, err)
    return err


def _instances(count, seed, max_side=256):
    ws = config_batch(count=count, nsteps=1, seed=seed, sides=(64, 96, 160), n1d=(200, 5000),
                      max_side=max_side)
    return ws


def _alone(w, nsteps, dtype, with_V=True):
    import torch
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    psi = torch.from_numpy(w.psi0).to("cuda").to(tdt)
    V = torch.from_numpy(w.V).to("cuda") if with_V else None
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype=dtype, axes=w.axes) as p:
        p.step(psi, V, nsteps)
        torch.cuda.synchronize()
    return psi.cpu().numpy()


def _start(w, dtype):
    return w.psi0.astype(np.complex64 if dtype == "c64" else np.complex128)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_matches_oracle_and_single_runs(dtype, graph):
    import torch
    announce(f"batch dtype={dtype} graph={graph}")
    ws = _instances(12, seed=3)
    rng = np.random.default_rng(4)
    nsteps = [int(v) for v in rng.integers(0, 90, size=len(ws))]
    nsteps[0] = 0
    nsteps[1] = 77
    nsteps[2] = 64
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    psis = [torch.from_numpy(w.psi0).to("cuda").to(tdt) for w in ws]
    Vs = [torch.from_numpy(w.V).to("cuda") for w in ws]
    with L.Batch([w.shape for w in ws], [w.dx for w in ws], [w.dt for w in ws],
                 [w.c for w in ws], [w.m for w in ws], dtype=dtype, graph=graph) as b:
        b.set(seg_len=24)
        b.step(psis, Vs, nsteps)
        torch.cuda.synchronize()
    for w, n, t in zip(ws, nsteps, psis):
        got = t.cpu().numpy()
        check_oracle(_start(w, dtype), w.V, n, got, dt=w.dt, c=w.c, m=w.m, axes=w.axes,
                     bc="zero", dtype=dtype, what=(w.name, w.shape, n))
        assert same_bits(got, _alone(w, n, dtype)), (w.name, w.shape, n)


def test_autotune_leaves_inputs_and_keeps_bits():
    import torch
    announce("batch autotune")
    ws = _instances(6, seed=8)
    psis = [torch.from_numpy(w.psi0).to("cuda").to(torch.complex64) for w in ws]
    Vs = [torch.from_numpy(w.V).to("cuda") for w in ws]
    before = [t.cpu().numpy() for t in psis]
    with L.Batch([w.shape for w in ws], [w.dx for w in ws], [w.dt for w in ws],
                 [w.c for w in ws], [w.m for w in ws], dtype="c64") as b:
        ch = b.autotune(psis, Vs, trials=2)
        torch.cuda.synchronize()
        assert ch["depth"] in (3, 4, 5) and ch["seg_len"] in (16, 32, 64, 128, 256, 512)
        assert ch["line_threads"] in (256, 512, 1024)
        assert b.depth() == ch["depth"]
        for t, ref in zip(psis, before):
            assert same_bits(t.cpu().numpy(), ref)
        b.step(psis, Vs, [40] * len(ws))
        torch.cuda.synchronize()
    for w, t in zip(ws, psis):
        got = t.cpu().numpy()
        check_oracle(_start(w, "c64"), w.V, 40, got, dt=w.dt, c=w.c, m=w.m, axes=w.axes,
                     bc="zero", dtype="c64", what=(w.name, w.shape))
        assert same_bits(got, _alone(w, 40, "c64"))


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_batch_graph_replay_of_fused_passes(dtype):
    """Every instance long enough for graph replay of whole passes, counts
    that are and are not multiples of the pass depth, some instances
    without a potential."""
    import torch
    announce(f"batch graph replay {dtype}")
    ws = _instances(9, seed=11)
    nsteps = [70, 71, 72, 73, 150, 99, 64, 65, 131]
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    psis = [torch.from_numpy(w.psi0).to("cuda").to(tdt) for w in ws]
    Vs = [None if k % 3 == 2 else torch.from_numpy(w.V).to("cuda") for k, w in enumerate(ws)]
    with L.Batch([w.shape for w in ws], [w.dx for w in ws], [w.dt for w in ws],
                 [w.c for w in ws], [w.m for w in ws], dtype=dtype, graph=True) as b:
        b.set(seg_len=32)
        b.step(psis, Vs, nsteps)
        torch.cuda.synchronize()
    for k, (w, n, t) in enumerate(zip(ws, nsteps, psis)):
        got = t.cpu().numpy()
        with_V = Vs[k] is not None
        check_oracle(_start(w, dtype), w.V if with_V else None, n, got, dt=w.dt, c=w.c, m=w.m,
                     axes=w.axes, bc="zero", dtype=dtype, what=(w.name, w.shape, n))
        assert same_bits(got, _alone(w, n, dtype, with_V)), (w.name, w.shape, n)


def test_batch_periodic_thin_instances():
    """A periodic batch with 2-D instances of few rows (the pass depth drops so
    that each wraps once) against the oracle and single periodic runs."""
    import torch
    from paper_1107_4650_amd.inputs import random_spinor
    announce("batch periodic thin")
    shapes = [(100, 5), (64, 3), (300,), (80, 40), (70, 9)]
    dx, c = 0.01, C_LIGHT
    psis0 = [random_spinor(s[::-1], seed=k).astype(np.complex64) for k, s in enumerate(shapes)]
    Vs0 = [np.random.default_rng(k).uniform(-2, 2, s[::-1]) * c * c for k, s in enumerate(shapes)]
    nsteps = [13, 8, 21, 10, 9]
    psis = [torch.from_numpy(p).to("cuda") for p in psis0]
    Vs = [torch.from_numpy(v).to("cuda") for v in Vs0]
    with L.Batch(shapes, dx, dx / c, c, 1.0, dtype="c64", bc="periodic") as b:
        b.step(psis, Vs, nsteps)
        torch.cuda.synchronize()
    for s, p0, v0, n, t in zip(shapes, psis0, Vs0, nsteps, psis):
        got = t.cpu().numpy()
        check_oracle(p0, v0, n, got, dt=dx / c, c=c, m=1.0, axes=tuple(range(len(s))),
                     bc="periodic", dtype="c64", what=(s, n))
        psi = torch.from_numpy(p0).to("cuda")
        with L.Plan(s, dx, dx / c, c, 1.0, dtype="c64", bc="periodic") as p:
            p.step(psi, torch.from_numpy(v0).to("cuda"), n)
            torch.cuda.synchronize()
        assert same_bits(got, psi.cpu().numpy()), (s, n)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("graph", [False, True])
def test_lines_kernel_and_depths(dtype, graph):
    """Only 1-D instances (all run whole by the lines kernel, several per
    workgroup) and a mix where a long line stays on the tiles; every pass depth
    gives the bits of the single-plan run and matches the oracle."""
    import torch
    from paper_1107_4650_amd.inputs import packet, potential_tanh
    announce(f"batch lines {dtype} graph={graph}")
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    lines = [(n,) for n in (300, 1000, 4000, 777, 2000, 64, 1500)]
    mixed = lines[:3] + [(96, 80), (200000,)]
    for shapes in (lines, mixed):
        ws = []
        for k, s_ in enumerate(shapes):
            psi = packet(s_, 0.01, delta=0.2, p0=[30.0] + [0.0] * (len(s_) - 1),
                         r0=[0.0] * len(s_))
            ws.append((s_, psi, potential_tanh(s_, 0.01, (0.5 + 0.3 * k) * C_LIGHT ** 2, 0.1)))
        nsteps = [23 + 5 * k for k in range(len(shapes))]
        nsteps[1] = 0
        for depth in (5, 3, 1):
            psis = [torch.from_numpy(p_).to("cuda").to(tdt) for _, p_, _ in ws]
            Vs = [torch.from_numpy(v).to("cuda") for _, _, v in ws]
            with L.Batch(shapes, 0.01, 0.01 / C_LIGHT, C_LIGHT, 1.0, dtype=dtype,
                         graph=graph) as b:
                b.set(seg_len=32, depth=depth)
                info = b.info()
                b.step(psis, Vs, nsteps)
                b.step(psis, Vs, nsteps)  # a second call of the same shape (graph reuse)
                torch.cuda.synchronize()
            # lines of up to 4096 cells always qualify; the 200000-cell one here
            # exceeds four even shares of the batch per compute unit
            n_short = sum(1 for s_ in shapes if len(s_) == 1 and s_[0] <= 4096)
            assert info["lines"] == n_short and info["line_bins"] >= 1, info
            for (s_, p_, v), n, t in zip(ws, nsteps, psis):
                got = t.cpu().numpy()
                start = p_.astype(np.complex64 if dtype == "c64" else np.complex128)
                ax = tuple(range(len(s_)))
                check_oracle(start, v, 2 * n, got, dt=0.01 / C_LIGHT, c=C_LIGHT, m=1.0,
                             axes=ax, bc="zero", dtype=dtype, what=(s_, n, depth))
                tp = torch.from_numpy(p_).to("cuda").to(tdt)
                with L.Plan(s_, 0.01, 0.01 / C_LIGHT, C_LIGHT, 1.0, dtype=dtype) as p:
                    p.step(tp, torch.from_numpy(v).to("cuda"), 2 * n)
                    torch.cuda.synchronize()
                assert same_bits(got, tp.cpu().numpy()), (s_, n, depth)


def test_autotune_cache_file(tmp_path, monkeypatch):
    """The tuner appends its choice keyed by dtype and size class; a new batch of
    the same kind reads it back."""
    import torch
    announce("batch tune cache")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LIBDIRAC_TUNE_CACHE", str(cache))
    ws = _instances(5, seed=21)
    psis = [torch.from_numpy(w.psi0).to("cuda").to(torch.complex64) for w in ws]
    Vs = [torch.from_numpy(w.V).to("cuda") for w in ws]
    args = ([w.shape for w in ws], [w.dx for w in ws], [w.dt for w in ws],
            [w.c for w in ws], [w.m for w in ws])
    with L.Batch(*args, dtype="c64") as b:
        ch = b.autotune(psis, Vs, trials=2)
    text = cache.read_text().split("\n")
    assert f"dirac-batch c64 2d-depth {ch['depth']}" in text
    assert f"dirac-batch c64 1d-threads {ch['line_threads']}" in text
    assert any(t.startswith("dirac-batch c64 2d-rows") for t in text)
    with L.Batch(*args, dtype="c64") as b2:
        assert b2.depth() == ch["depth"] and b2.info()["line_threads"] == ch["line_threads"]
    with L.Batch(*args, dtype="c128") as b3:  # another dtype: defaults
        assert b3.depth() == 5
