"""Pins of the oracle's second-order (Strang) step, Sec. 2.4.

* Symbol: for periodic Fourier modes one step must equal the symmetric
  product of the sub-step symbols, E_first E_second D E_second E_first with
  E_d = expm(-i alpha_d k_d a) (a one-cell transport, c dt/2 = a) and
  D = expm(-i beta m c^2 dt); in 1-D its trace obeys
  tr M / 4 = cos(m c^2 dt) cos(2 k a).
* Massless data in the +1 eigenspace of alpha move exactly two cells per
  step (two half-step shifts).
* Against the exact continuum evolution (Fourier-space solution, FFT) the
  error falls 4x per halving of the cell (second order), where the
  lowest-order step falls 2x (first order), as Sec. 2.4 states.
* Unitarity on a periodic box; zero walls never create probability.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import reference as R
from paper_1107_4650_amd.inputs import packet, random_spinor

C = 137.036


def strang_symbol(oracle, shape, js, dx, m, axes, c=C):
    nd = len(shape)
    idx = np.meshgrid(*[np.arange(n) for n in shape[::-1]], indexing="ij")
    turns = np.zeros(shape[::-1])
    for d in range(nd):
        turns = turns + ((js[d] * idx[nd - 1 - d]) % shape[d]) / shape[d]
    phase = np.exp(2j * np.pi * turns)
    M = np.zeros((4, 4), complex)
    for col in range(4):
        psi = np.zeros(shape[::-1] + (4,), complex)
        psi[..., col] = phase
        out = oracle.step_strang(psi, dt=2 * dx / c, c=c, m=m, nsteps=1, axes=axes,
                                 bc="periodic")
        v = out / phase[..., None]
        assert np.max(np.abs(v - v.reshape(-1, 4)[0])) < 1e-13
        M[:, col] = v.reshape(-1, 4)[0]
    return M


@pytest.mark.parametrize("shape,axes", [((16,), (0,)), ((16,), (1,)), ((16,), (2,)),
                                        ((8, 8), (0, 1)), ((8, 8), (0, 2)), ((8, 8), (1, 2))])
def test_strang_symbol_is_the_symmetric_product(oracle, shape, axes):
    dx, m = 0.01, 1.0
    dt = 2 * dx / C
    D = scipy.linalg.expm(-1j * R.BETA * m * C * C * dt)
    rng = np.random.default_rng(3)
    modes = [[j] for j in range(shape[0])] if len(shape) == 1 else \
        [list(rng.integers(0, 8, 2)) for _ in range(12)] + [[4, 0], [0, 4], [4, 4]]
    # the order of the sub-steps: by Dirac matrix (A, B, C), whatever the grid dimension
    order = sorted(range(len(shape)), key=lambda d: axes[d])
    for js in modes:
        M = strang_symbol(oracle, shape, js, dx, m, axes)
        E = [scipy.linalg.expm(-1j * R.dirac_alpha(axes[d]) * 2 * np.pi * js[d] / shape[d])
             for d in range(len(shape))]
        # applied first on the right: E_first, E_second, D, E_second, E_first
        expect = np.eye(4, dtype=complex)
        for d in order:
            expect = E[d] @ expect
        expect = D @ expect
        for d in reversed(order):
            expect = E[d] @ expect
        assert np.max(np.abs(M - expect)) < 1e-13, js
        assert np.allclose(M.conj().T @ M, np.eye(4), atol=1e-13)
        if len(shape) == 1:
            ka = 2 * np.pi * js[0] / shape[0]
            assert abs(np.trace(M).real / 4 - np.cos(m * C * C * dt) * np.cos(2 * ka)) < 1e-13


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_strang_massless_eigen_shift_is_two_cells(oracle, axis):
    n, steps = 400, 23
    rng = np.random.default_rng(axis)
    u = rng.uniform(-1, 1, (n, 2)) + 1j * rng.uniform(-1, 1, (n, 2))
    u[:60] = 0
    u[-60:] = 0
    pauli = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]),
             np.array([[1, 0], [0, -1]])][axis]
    psi = np.zeros((n, 4), complex)
    psi[:, :2] = u
    psi[:, 2:] = u @ pauli.T
    out = oracle.step_strang(psi, dt=2 * 0.01 / C, c=C, m=0.0, nsteps=steps, axes=(axis,))
    assert np.array_equal(out, np.roll(psi, 2 * steps, axis=0))


def _conv_errors(oracle, scheme, kind, p0):
    """Relative L2 error at t = 2 against the continuum evolution (c = m = 1
    units, so that m c^2 dt stays small), box +-8, Delta = 1, x-z plane."""
    c, m, L, t = 1.0, 1.0, 16.0, 2.0
    errs = []
    for n in (64, 128, 256):
        dx = L / n
        psi0 = packet((n, n), dx, delta=1.0, kind=kind, p0=p0, axes=(0, 2), c=c, m=m)
        if scheme == "strang":
            dt = 2 * dx / c
            nst = int(round(t / dt))
            out = oracle.step_strang(psi0, dt=dt, c=c, m=m, nsteps=nst, axes=(0, 2),
                                     bc="periodic")
        else:
            dt = dx / c
            nst = int(round(t / dt))
            out = oracle.step(psi0, dt=dt, c=c, m=m, nsteps=nst, axes=(0, 2), bc="periodic")
        ref = R.free_fft(psi0, dx, nst * dt, c, m, axes=(0, 2))
        errs.append(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    return np.array(errs)


@pytest.mark.parametrize("kind,p0", [("spin_up", None), ("positive", [2.0, 1.0])])
def test_strang_is_second_order_lie_first_order(oracle, kind, p0):
    es = _conv_errors(oracle, "strang", kind, p0)
    el = _conv_errors(oracle, "lie", kind, p0)
    rs, rl = es[:-1] / es[1:], el[:-1] / el[1:]
    assert np.all((rs > 3.6) & (rs < 4.6)), rs
    assert np.all((rl > 1.8) & (rl < 2.2)), rl
    assert es[-1] < el[-1] / 3


def test_strang_unitarity_and_walls(oracle):
    shape = (40, 36)
    psi = random_spinor(shape[::-1], seed=9)
    V = np.random.default_rng(2).uniform(-3, 3, shape[::-1]) * C * C
    out = oracle.step_strang(psi, V, dt=2 * 0.01 / C, c=C, m=1.0, nsteps=120, axes=(0, 1),
                             bc="periodic")
    n0, n1 = np.sum(np.abs(psi) ** 2), np.sum(np.abs(out) ** 2)
    assert abs(n1 / n0 - 1) < 1e-12
    norms = [n0]
    cur = psi
    for _ in range(6):
        cur = oracle.step_strang(cur, V, dt=2 * 0.01 / C, c=C, m=1.0, nsteps=10, axes=(1, 2))
        norms.append(np.sum(np.abs(cur) ** 2))
    assert np.all(np.diff(norms) <= 1e-12 * n0)


# ---- 3-D second-order step: A(dt/4) B(dt/2) A(dt/4) C(dt/2) D C B A pattern ----

def test_strang3d_symbol_is_the_printed_product(oracle):
    """On a periodic 3-D box every Fourier mode is multiplied by the product of
    the sub-step symbols in the printed order, with one-cell A and two-cell B,
    C shifts: E_A E_B E_A E_C D E_C E_A E_B E_A (rightmost first),
    E_d(s) = expm(-i alpha_d k_d s a)."""
    shape, dx, m = (8, 8, 8), 0.01, 1.0
    dt = 4 * dx / C
    D = scipy.linalg.expm(-1j * R.BETA * m * C * C * dt)
    rng = np.random.default_rng(5)
    modes = [list(rng.integers(0, 8, 3)) for _ in range(10)] + [[4, 0, 0], [0, 4, 0], [0, 0, 4],
                                                                [1, 2, 3]]
    for js in modes:
        idx = np.meshgrid(*[np.arange(n) for n in shape[::-1]], indexing="ij")
        turns = sum(((js[d] * idx[2 - d]) % shape[d]) / shape[d] for d in range(3))
        phase = np.exp(2j * np.pi * turns)
        M = np.zeros((4, 4), complex)
        for col in range(4):
            psi = np.zeros(shape[::-1] + (4,), complex)
            psi[..., col] = phase
            out = oracle.step_strang(psi, dt=dt, c=C, m=m, nsteps=1, axes=(0, 1, 2),
                                     bc="periodic")
            v = out / phase[..., None]
            assert np.max(np.abs(v - v.reshape(-1, 4)[0])) < 1e-13
            M[:, col] = v.reshape(-1, 4)[0]
        k = [2 * np.pi * js[d] / shape[d] for d in range(3)]
        E = lambda d, s: scipy.linalg.expm(-1j * R.dirac_alpha(d) * k[d] * s)
        seq = [E(0, 1), E(1, 2), E(0, 1), E(2, 2), D, E(2, 2), E(0, 1), E(1, 2), E(0, 1)]
        expect = np.eye(4, dtype=complex)
        for f in seq:
            expect = f @ expect
        assert np.max(np.abs(M - expect)) < 1e-13, js


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_strang3d_massless_eigen_shift_is_four_cells(oracle, axis):
    """Massless data varying along one axis only, in the +1 eigenspace of
    that axis' alpha, move exactly four cells per step (four one-cell A or two
    two-cell B / C shifts; the other transports leave uniform data alone)."""
    n, steps, other = 64, 5, 4
    rng = np.random.default_rng(10 + axis)
    u = rng.uniform(-1, 1, (n, 2)) + 1j * rng.uniform(-1, 1, (n, 2))
    pauli = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]),
             np.array([[1, 0], [0, -1]])][axis]
    line = np.zeros((n, 4), complex)
    line[:, :2] = u
    line[:, 2:] = u @ pauli.T
    shape = [other, other, other]
    shape[axis] = n
    arr_shape = tuple(shape[::-1]) + (4,)
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    psi = np.broadcast_to(line.reshape(tuple(bshape) + (4,)), arr_shape).copy()
    out = oracle.step_strang(psi, dt=4 * 0.01 / C, c=C, m=0.0, nsteps=steps,
                             axes=(0, 1, 2), bc="periodic")
    assert np.array_equal(out, np.roll(psi, 4 * steps, axis=2 - axis))


def test_strang3d_unitarity_and_walls(oracle):
    shape = (12, 10, 9)
    psi = random_spinor(shape[::-1], seed=19)
    V = np.random.default_rng(4).uniform(-3, 3, shape[::-1]) * C * C
    out = oracle.step_strang(psi, V, dt=4 * 0.01 / C, c=C, m=1.0, nsteps=20, axes=(0, 1, 2),
                             bc="periodic")
    n0 = np.sum(np.abs(psi) ** 2)
    assert abs(np.sum(np.abs(out) ** 2) / n0 - 1) < 1e-12
    norms, cur = [n0], psi
    for _ in range(4):
        cur = oracle.step_strang(cur, V, dt=4 * 0.01 / C, c=C, m=1.0, nsteps=3, axes=(0, 1, 2))
        norms.append(np.sum(np.abs(cur) ** 2))
    assert np.all(np.diff(norms) <= 1e-12 * n0)
