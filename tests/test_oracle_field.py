"""Pins of the oracle's local step with a vector potential (eq:sol_dis_4 with
the closed-form exponential of Dirac matrices, Sec. 2.3).

* On a periodic box a uniform spinor field is left alone by the transports,
  so one step is the local step itself: at every cell it must equal
  expm(-i beta m c^2 dt - i V dt + i alpha . Atilde) computed by scipy,
  for random fields varying from cell to cell (which also fixes the planar
  component layout), for the massless case and for Atilde = 0.
* The one-step symbol of a Fourier mode with a uniform field is
  expm(local) expm(-i alpha k a) (lowest order) and
  E expm(local) E with E = expm(-i alpha k a) (second order).
* With Atilde = 0 the step reduces to the plain step; steps are unitary on a
  periodic box.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import reference as R
from paper_1107_4650_amd.inputs import random_spinor

C = 137.036
DX = 0.01


def local_expm(mu, vdt, a):
    Hs = -mu * R.BETA - vdt * np.eye(4) + sum(a[d] * R.dirac_alpha(d) for d in range(3))
    return scipy.linalg.expm(1j * Hs)


@pytest.mark.parametrize("m", [1.0, 0.0])
def test_field_local_step_is_the_matrix_exponential(oracle, m):
    shape = (6, 5)
    dt = DX / C
    rng = np.random.default_rng(7)
    A = rng.uniform(-3, 3, (3,) + shape[::-1])
    A[:, 0, 0] = 0.0  # one cell without field
    V = rng.uniform(-2, 2, shape[::-1]) * C * C
    for col in range(4):
        psi = np.zeros(shape[::-1] + (4,), complex)
        psi[..., col] = 1.0
        out = oracle.step_field(psi, V, A, dt=dt, c=C, m=m, nsteps=1, axes=(0, 1),
                                bc="periodic")
        for j in range(shape[1]):
            for i in range(shape[0]):
                D = local_expm(m * C * C * dt, V[j, i] * dt, A[:, j, i])
                assert np.max(np.abs(out[j, i] - D[:, col])) < 1e-13, (col, j, i)


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_field_symbol_with_uniform_field(oracle, scheme):
    n, m = 16, 1.0
    dt = (2 if scheme == "strang" else 1) * DX / C
    a = np.array([0.7, -1.3, 0.4])
    A = np.broadcast_to(a[:, None], (3, n)).copy()
    D = local_expm(m * C * C * dt, 0.0, a)
    idx = np.arange(n)
    for j in range(n):
        phase = np.exp(2j * np.pi * j * idx / n)
        E = scipy.linalg.expm(-1j * R.dirac_alpha(0) * 2 * np.pi * j / n)
        expect = E @ D @ E if scheme == "strang" else D @ E
        M = np.zeros((4, 4), complex)
        for col in range(4):
            psi = np.zeros((n, 4), complex)
            psi[:, col] = phase
            out = oracle.step_field(psi, None, A, dt=dt, c=C, m=m, nsteps=1, axes=(0,),
                                    bc="periodic", scheme=scheme)
            M[:, col] = (out / phase[:, None])[3]
        assert np.max(np.abs(M - expect)) < 1e-13, j


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_field_zero_reduces_to_plain_step_and_is_unitary(oracle, scheme):
    shape = (24, 18)
    dt = (2 if scheme == "strang" else 1) * DX / C
    psi = random_spinor(shape[::-1], seed=3)
    V = np.random.default_rng(4).uniform(-3, 3, shape[::-1]) * C * C
    plain = (oracle.step_strang if scheme == "strang" else oracle.step)(
        psi, V, dt=dt, c=C, m=1.0, nsteps=20, axes=(0, 2))
    zero = oracle.step_field(psi, V, np.zeros((3,) + shape[::-1]), dt=dt, c=C, m=1.0, nsteps=20,
                             axes=(0, 2), scheme=scheme)
    assert np.linalg.norm(zero - plain) / np.linalg.norm(plain) < 1e-13
    A = np.random.default_rng(5).uniform(-2, 2, (3,) + shape[::-1])
    out = oracle.step_field(psi, V, A, dt=dt, c=C, m=1.0, nsteps=40, axes=(0, 2), bc="periodic",
                            scheme=scheme)
    assert abs(np.sum(np.abs(out) ** 2) / np.sum(np.abs(psi) ** 2) - 1) < 1e-12


def test_field_symbol_3d_second_order(oracle):
    """3-D second-order step with a uniform field on a periodic box: the symbol
    of a Fourier mode is EA EB EA EC D EC EA EB EA with EA the one-cell shift
    along x, EB and EC the two-cell shifts along y and z (c dt = 4 a) and D
    the local step; modes with distinct wave numbers on every axis, so a
    swapped, dropped or doubled sub-step fails."""
    n = (6, 5, 4)
    m = 1.0
    dt = 4 * DX / C
    a = np.array([-0.9, 0.6, 1.1])
    A = np.broadcast_to(a[:, None, None, None], (3,) + n[::-1]).copy()
    D = local_expm(m * C * C * dt, 0.0, a)
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    for jx, jy, jz in [(1, 2, 1), (2, 1, 3), (5, 3, 2), (0, 4, 1)]:
        th = 2 * np.pi * np.array([jx / n[0], jy / n[1], jz / n[2]])
        phase = np.exp(1j * (th[0] * i + th[1] * j + th[2] * k))
        EA = scipy.linalg.expm(-1j * R.dirac_alpha(0) * th[0])
        EB = scipy.linalg.expm(-1j * R.dirac_alpha(1) * 2 * th[1])
        EC = scipy.linalg.expm(-1j * R.dirac_alpha(2) * 2 * th[2])
        expect = EA @ EB @ EA @ EC @ D @ EC @ EA @ EB @ EA
        M = np.zeros((4, 4), complex)
        for col in range(4):
            psi = np.zeros(n[::-1] + (4,), complex)
            psi[..., col] = phase
            out = oracle.step_field(psi, None, A, dt=dt, c=C, m=m, nsteps=1, axes=(0, 1, 2),
                                    bc="periodic", scheme="strang")
            ratio = out / phase[..., None]
            assert np.max(np.abs(ratio - ratio[1, 2, 3])) < 1e-13  # one symbol for all cells
            M[:, col] = ratio[1, 2, 3]
        assert np.max(np.abs(M - expect)) < 1e-13, (jx, jy, jz)


def test_field_zero_3d_second_order_is_the_plain_step(oracle):
    """Atilde = 0 in the 3-D second-order step gives the plain 3-D
    second-order step; with a varying field the step stays unitary on a
    periodic box and differs from the field-free step."""
    shape = (10, 8, 6)
    dt = 4 * DX / C
    psi = random_spinor(shape[::-1], seed=11)
    V = np.random.default_rng(12).uniform(-3, 3, shape[::-1]) * C * C
    plain = oracle.step_strang(psi, V, dt=dt, c=C, m=1.0, nsteps=6)
    zero = oracle.step_field(psi, V, np.zeros((3,) + shape[::-1]), dt=dt, c=C, m=1.0, nsteps=6,
                             scheme="strang")
    assert np.linalg.norm(zero - plain) / np.linalg.norm(plain) < 1e-13
    A = np.random.default_rng(13).uniform(-2, 2, (3,) + shape[::-1])
    out = oracle.step_field(psi, V, A, dt=dt, c=C, m=1.0, nsteps=10, bc="periodic",
                            scheme="strang")
    assert abs(np.sum(np.abs(out) ** 2) / np.sum(np.abs(psi) ** 2) - 1) < 1e-12
    free = oracle.step_strang(psi, V, dt=dt, c=C, m=1.0, nsteps=10, bc="periodic")
    assert np.linalg.norm(out - free) > 1e-2 * np.linalg.norm(free)
