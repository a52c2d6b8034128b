"""The 2-D workload at its stated length against the oracle: 2048 x 2048 cells,
10^4 lowest-order steps, zero walls, in the launch configuration the benchmark
times (passes of five fused steps).  The oracle's final state is stored in
tests/golden/config2_2048_1e4.txt (written by make_config2_golden.py beside it,
which calls only the oracle) on 512 cells -- the 256 of largest |psi|^2 and 256
of the packet's tails -- with the observables of the whole grid.  Bars: FP64
state relative L2 1e-12 over the sampled cells and 1e-12 on the observables;
FP32 state 1e-4 (the precision target) and 1e-5 on the observables."""
import os

import numpy as np
import pytest

from paper_1107_4650_amd import libdirac as L
from paper_1107_4650_amd.inputs import config_2d_tanh
from tests.golden_util import GOLDEN_CONFIG2 as GOLDEN, load_golden
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_config2_1e4_steps_vs_stored_oracle_state(dtype):
    import torch
    if not os.path.exists(GOLDEN):
        pytest.skip("golden state not written (tests/golden/make_config2_golden.py)")
    obs_ref, idx, ref = load_golden()
    w = config_2d_tanh(n=2048, nsteps=10000)
    announce(f"2-D 2048^2 x 1e4 steps vs stored oracle state, {dtype}")
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    psi = torch.from_numpy(w.psi0).to("cuda").to(tdt)
    V = torch.from_numpy(w.V).to("cuda")
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype=dtype, xmin=w.xmin) as p:
        assert p.info()["depth"] == 5
        p.step(psi, V, w.nsteps)
        torch.cuda.synchronize()
        obs = np.array(p.observables(psi, 0.0))
    got = psi.reshape(-1, 4)[torch.from_numpy(idx).to("cuda")].cpu().numpy().astype(np.complex128)
    err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    obs_err = float(np.max(np.abs(obs[[0, 1, 2, 4]] - obs_ref[[0, 1, 2, 4]]) /
                           np.abs(obs_ref[[0, 1, 2, 4]])))
    announce(f"rel-L2 over {len(idx)} cells {err:.3e}, observables {obs_err:.3e}")
    if dtype == "c128":
        assert err <= 1e-12 and obs_err <= 1e-12
    else:
        assert err <= 1e-4 and obs_err <= 1e-5
