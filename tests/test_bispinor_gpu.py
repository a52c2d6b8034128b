"""Two-component 1-D lines (DL_BISPINOR): the stored pair (psi_1 with psi_4
for alpha_x, alpha_y; psi_1 with psi_3 for alpha_z) against the oracle's
four-component step with the other pair zero (FP64 to 1e-12), and bit for
bit against the library's own four-component step (FP32 and FP64): resident
and tiled lines, fused passes, both splittings, both walls; observables of
the pair equal those of the four-component state."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1107_4650_amd.inputs import random_spinor, C_LIGHT
from tests.gpu_util import announce, rel_l2, same_bits

pytestmark = pytest.mark.gpu

C = C_LIGHT
DX = 0.01


def _pair(axis):
    return [0, 3] if axis < 2 else [0, 2]


def _run(psi, V, *, n, axis, bc, dtype, scheme, nsteps, bispinor, resident=True):
    import torch
    from paper_1107_4650_amd import libdirac as L
    tdt = torch.complex64 if dtype == "c64" else torch.complex128
    dt = (2 if scheme == "strang" else 1) * DX / C
    t = torch.from_numpy(np.ascontiguousarray(psi)).to("cuda").to(tdt)
    tV = torch.from_numpy(V).to("cuda")
    with L.Plan((n,), DX, dt, C, 1.0, dtype=dtype, bc=bc, axes=(axis,), scheme=scheme,
                bispinor=bispinor) as p:
        if resident:
            p.set_depth(2)  # the resident kernel serves plans of at most 2 steps per pass
        else:
            p.set_tiling(allow_resident=False)
        p.step(t, tV, nsteps)
        obs = p.observables(t, 0.3)
        torch.cuda.synchronize()
    return t.cpu().numpy(), obs


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
@pytest.mark.parametrize("n,scheme,resident", [(4096, "lie", True), (6000, "lie", False),
                                               (1000, "strang", False), (4099, "lie", False)])
def test_bispinor_line(axis, bc, n, scheme, resident):
    announce(f"bispinor axis={axis} bc={bc} n={n} {scheme} resident={resident}")
    pr = _pair(axis)
    psi4 = random_spinor((n,), seed=n + axis)
    other = [k for k in range(4) if k not in pr]
    psi4[:, other] = 0
    psi2 = np.ascontiguousarray(psi4[:, pr])
    V = np.random.default_rng(axis).uniform(-2, 2, n) * C * C
    nsteps = 37
    dt = (2 if scheme == "strang" else 1) * DX / C
    step = O.step_strang if scheme == "strang" else O.step
    ref = step(psi4, V, dt=dt, c=C, m=1.0, nsteps=nsteps, axes=(axis,), bc=bc)
    kw = dict(n=n, axis=axis, bc=bc, scheme=scheme, nsteps=nsteps, resident=resident)
    g2, obs2 = _run(psi2, V, dtype="c128", bispinor=True, **kw)
    assert rel_l2(g2, ref[:, pr]) <= 1e-12
    g4, obs4 = _run(psi4, V, dtype="c128", bispinor=False, **kw)
    assert same_bits(g2, g4[:, pr])
    assert np.array_equal(obs2, obs4)
    f2, _ = _run(psi2.astype(np.complex64), V, dtype="c64", bispinor=True, **kw)
    f4, _ = _run(psi4.astype(np.complex64), V, dtype="c64", bispinor=False, **kw)
    assert same_bits(f2, f4[:, pr])


def test_bispinor_refusals():
    import torch
    from paper_1107_4650_amd import libdirac as L
    with pytest.raises(L.DiracError):
        L.Plan((16, 16), DX, DX / C, C, 1.0, bispinor=True, dry=True)
    with L.Plan((64,), DX, DX / C, C, 1.0, bispinor=True) as p:
        psi = torch.zeros(p.tshape, dtype=torch.complex64, device="cuda")
        A = torch.zeros((3, 64), dtype=torch.float64, device="cuda")
        with pytest.raises(L.DiracError):
            p.step_field(psi, None, A, 1)
        lam = torch.zeros_like(psi)
        Q = torch.zeros((64,), dtype=torch.float64, device="cuda")
        with pytest.raises(L.DiracError):
            p.seed_adjoint(psi, 0.0, lam, Q)
