"""Pins of the oracle against what the paper and the algebra fix exactly.

* Dirac representation (Sec. 2, eq:dirac_mat) and the Clifford algebra.
* The transport sub-step applies 1/2(I + alpha) to the left neighbour and
  1/2(I - alpha) to the right one (eq:sol_dis_1-3): read back from the oracle's
  response to a single-site delta.
* Exact characteristic shift when c dt = a (Sec. 2.3): alpha-eigen-aligned
  massless data move by exactly one cell per step, with no rounding.
* Unitarity with periodic cells, non-increasing norm with zero walls.
* The local step D equals expm(-i (beta m c^2 + V) dt) (eq:sol_dis_4, A = 0).
"""
import numpy as np
import pytest
import scipy.linalg

from paper_1107_4650_amd.inputs import random_spinor, packet, C_LIGHT

PAULI = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]


def test_dirac_matrices_match_paper_and_clifford(oracle):
    ax, ay, az, beta = oracle.dirac_matrices()
    alphas = [ax, ay, az]
    I4 = np.eye(4)
    # printed blocks: alpha_i = [[0, sigma_i], [sigma_i, 0]], beta = diag(I, -I)
    for a, s in zip(alphas, PAULI):
        assert np.array_equal(a[:2, 2:], s) and np.array_equal(a[2:, :2], s)
        assert np.array_equal(a[:2, :2], np.zeros((2, 2))) and np.array_equal(a[2:, 2:], np.zeros((2, 2)))
    assert np.array_equal(beta, np.diag([1, 1, -1, -1]))
    # Clifford algebra {alpha_i, alpha_j} = 2 delta_ij, {alpha_i, beta} = 0, Hermitian
    for i in range(3):
        assert np.array_equal(alphas[i].conj().T, alphas[i])
        assert np.array_equal(alphas[i] @ beta + beta @ alphas[i], np.zeros((4, 4)))
        for j in range(3):
            anti = alphas[i] @ alphas[j] + alphas[j] @ alphas[i]
            assert np.array_equal(anti, 2 * I4 * (i == j))
    # orientation: alpha_x alpha_y = i diag(sigma_z, sigma_z) (fixes the sign of alpha_y)
    spin_z = np.kron(np.eye(2), PAULI[2])
    assert np.array_equal(ax @ ay, 1j * spin_z)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_transport_matrices_from_delta_response(oracle, axis):
    """Drive the 1-D transport with one unit vector at a time; the response at
    i+1 is 1/2(I + alpha) e_k, at i-1 it is 1/2(I - alpha) e_k."""
    n, i = 9, 4
    Pp = np.zeros((4, 4), complex)
    Pm = np.zeros((4, 4), complex)
    for k in range(4):
        psi = np.zeros((n, 4), complex)
        psi[i, k] = 1.0
        out = oracle.step(psi, dt=1e-4, c=1.0, m=0.0, nsteps=1, axes=(axis,))
        Pp[:, k] = out[i + 1]
        Pm[:, k] = out[i - 1]
        others = np.delete(out, [i - 1, i + 1], axis=0)
        assert np.all(others == 0)
    alpha = oracle.dirac_matrices()[axis]
    I4 = np.eye(4)
    assert np.array_equal(Pp + Pm, I4)
    assert np.array_equal(Pp - Pm, alpha)
    assert np.array_equal(Pp @ Pp, Pp) and np.array_equal(Pm @ Pm, Pm)
    assert np.array_equal(Pp @ Pm, np.zeros((4, 4)))
    assert np.linalg.matrix_rank(Pp) == 2 and np.linalg.matrix_rank(Pm) == 2


def eigen_aligned(axis, sign, n, seed):
    """Random 1-D data lying in the +1 (sign=+1) or -1 eigenspace of alpha_axis,
    built with exact operations only; zero near both walls."""
    rng = np.random.default_rng(seed)
    u = (rng.uniform(-1, 1, (n, 2)) + 1j * rng.uniform(-1, 1, (n, 2)))
    u[:8] = 0
    u[-8:] = 0
    psi = np.zeros((n, 4), complex)
    psi[:, :2] = u
    lower = np.stack([PAULI[axis] @ row for row in u])   # exact: entries 0, +-1, +-i
    psi[:, 2:] = sign * lower
    return psi


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("sign", [+1, -1])
def test_exact_characteristic_shift(oracle, axis, sign):
    n, steps = 64, 5
    psi = eigen_aligned(axis, sign, n, seed=axis * 10 + (sign > 0))
    out = oracle.step(psi, dt=1e-3, c=1.0, m=0.0, nsteps=steps, axes=(axis,))
    expect = np.roll(psi, sign * steps, axis=0)   # zero margin >= steps, no wrap content
    assert np.array_equal(out, expect)
    outf = oracle.stream_f32(psi.astype(np.complex64), nsteps=steps, axes=(axis,))
    assert np.array_equal(outf, expect.astype(np.complex64))


@pytest.mark.parametrize("shape,axes", [((48,), (0,)), ((20, 24), (0, 1)), ((16, 20), (0, 2)),
                                        ((8, 10, 12), (0, 1, 2))])
def test_periodic_unitarity(oracle, shape, axes):
    psi = random_spinor(shape[::-1], seed=3)
    rng = np.random.default_rng(4)
    V = rng.uniform(-3, 3, size=shape[::-1]) * C_LIGHT ** 2
    dx = 0.01
    out = oracle.step(psi, V, dt=dx / C_LIGHT, c=C_LIGHT, m=1.0, nsteps=200, axes=axes,
                      bc="periodic")
    n0, n1 = np.sum(np.abs(psi) ** 2), np.sum(np.abs(out) ** 2)
    assert abs(n1 - n0) / n0 < 1e-13


def test_zero_walls_norm_nonincreasing_and_conserved_inside(oracle):
    dx = 0.01
    shape = (256,)
    psi = packet(shape, dx, delta=0.08, p0=[30.0], r0=[0.0])
    V = np.full(shape, 0.5 * C_LIGHT ** 2)
    for m, Vm in ((1.0, V), (0.0, None)):
        norms = [np.sum(np.abs(psi) ** 2)]
        cur = psi
        for _ in range(40):
            cur = oracle.step(cur, Vm, dt=dx / C_LIGHT, c=C_LIGHT, m=m, nsteps=5)
            norms.append(np.sum(np.abs(cur) ** 2))
        norms = np.array(norms)
        assert np.all(np.diff(norms) <= 1e-15 * norms[0])
        # the packet (8 cells wide, at cell 128) is far from the walls for 25 steps
        assert abs(norms[5] - norms[0]) / norms[0] < 1e-13
    # massless components travel one cell per step: after 200 steps they have
    # crossed the walls and left the box
    assert norms[-1] < 0.5 * norms[0]


def test_local_step_equals_matrix_exponential(oracle):
    """With alpha_x-eigen-aligned massless-transport data the transport is an
    exact shift, so one step isolates D: out(i) = expm(-i(beta m c^2 + V_i) dt) psi(i-1)."""
    n = 40
    psi = eigen_aligned(0, +1, n, seed=7)
    rng = np.random.default_rng(8)
    c, m, dx = C_LIGHT, 1.0, 0.01
    dt = dx / c
    V = rng.uniform(-3, 3, n) * m * c * c
    out = oracle.step(psi, V, dt=dt, c=c, m=m, nsteps=1, axes=(0,))
    beta = np.diag([1.0, 1.0, -1.0, -1.0])
    for i in range(1, n):
        U = scipy.linalg.expm(-1j * (beta * m * c * c + V[i] * np.eye(4)) * dt)
        ref = U @ psi[i - 1]
        assert np.max(np.abs(out[i] - ref)) <= 1e-15 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("bc", ["zero", "periodic"])
def test_one_axis_pairs_decouple(oracle, axis, bc):
    """With one transport axis the components split into two pairs that never
    mix (alpha_x, alpha_y: (1,4) and (2,3); alpha_z: (1,3) and (2,4); beta is
    diagonal): a zero pair stays exactly zero, and the other pair evolves the
    same whatever the zero pair held."""
    n = 300
    first = [0, 3] if axis < 2 else [0, 2]
    other = [k for k in range(4) if k not in first]
    psi = random_spinor((n,), seed=axis)
    V = np.random.default_rng(9).uniform(-2, 2, n) * 137.036 ** 2
    kw = dict(dt=0.01 / 137.036, c=137.036, m=1.0, nsteps=40, axes=(axis,), bc=bc)
    full = oracle.step(psi, V, **kw)
    half = psi.copy()
    half[:, other] = 0
    out = oracle.step(half, V, **kw)
    assert np.all(out[:, other] == 0)
    assert np.max(np.abs(out[:, first] - full[:, first])) <= 1e-15 * np.max(np.abs(full))
