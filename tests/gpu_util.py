"""Helpers shared by the GPU tests: run the HIP library through the C ABI on
numpy inputs and bring the result back."""
import sys

import numpy as np

from paper_1107_4650_amd import libdirac as L


def announce(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def gpu_step(psi, V, *, dx, dt, c, m, nsteps, axes=None, bc="zero", dtype="c128", tiling=None,
             graph=False, chunks=None, depth=None, scheme="lie", A=None):
    """Run dl_step on a copy of psi (numpy, (..., 4)); returns numpy."""
    import torch
    shape = tuple(reversed(psi.shape[:-1]))
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    t = torch.from_numpy(np.ascontiguousarray(psi)).to("cuda").to(tdt).contiguous()
    tV = None if V is None else torch.from_numpy(np.ascontiguousarray(V, dtype=np.float64)).to("cuda")
    with L.Plan(shape, dx, dt, c, m, dtype=dtype, bc=bc, axes=axes, graph=graph,
                scheme=scheme) as p:
        if tiling:
            p.set_tiling(**tiling)
        if depth is not None:
            p.set_depth(depth)
        if A is not None:
            tA = torch.from_numpy(np.ascontiguousarray(A, dtype=np.float64)).to("cuda")
            p.step_field(t, tV, tA, nsteps)
        elif chunks:
            for k in chunks:
                p.step(t, tV, k)
        else:
            p.step(t, tV, nsteps)
        torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_l2(a, b):
    a = a.astype(np.complex128)
    b = b.astype(np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def same_bits(a, b):
    """Element-wise equality of the real and imaginary parts (+0 == -0)."""
    return bool(np.all(a.real == b.real) and np.all(a.imag == b.imag))
