"""Dispersion of the oracle's one-step operator (Sec. 3, no fermion doubling).

The symbol M(k) of one step is read back from the oracle by stepping periodic
Fourier modes, then compared with what Sec. 3 fixes:
  * massless 1-D: M(k) = expm(-i alpha k a) exactly (eq:sol_dis), eigenphases
    +-k a, linear dispersion E = +-c p_k;
  * massive 1-D: M = exp(-i beta m c^2 dt) exp(-i alpha k a), whose
    eigenphases obey cos(w) = cos(m c^2 dt) cos(k a); the only minimum of |w|
    is at k = 0 and k = pi/a sits at the band top w = pi - m c^2 dt, whereas the
    central-difference operator has a second zero there (the doubler);
  * 2-D: tr M / 4 = cos(m c^2 dt) prod_d cos(k_d a); no zero on the axes'
    zone boundary (pi/a, 0); the zone corner aliases k = 0 for this first-order
    splitting (recorded, see the design notes on the 2-D/3-D claim).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import reference as R

C = 137.036


def symbol(oracle, shape, js, dx, m, axes):
    """Measure the 4x4 one-step symbol of the periodic Fourier mode with integer
    wave numbers js (per grid dim), i.e. k_d a = 2 pi js[d] / n_d."""
    nd = len(shape)
    idx = np.meshgrid(*[np.arange(n) for n in shape[::-1]], indexing="ij")
    turns = np.zeros(shape[::-1])
    for d in range(nd):
        turns = turns + ((js[d] * idx[nd - 1 - d]) % shape[d]) / shape[d]
    phase = np.exp(2j * np.pi * turns)
    M = np.zeros((4, 4), complex)
    for c in range(4):
        psi = np.zeros(shape[::-1] + (4,), complex)
        psi[..., c] = phase
        out = oracle.step(psi, dt=dx / C, c=C, m=m, nsteps=1, axes=axes, bc="periodic")
        col = out / phase[..., None]
        # translation invariance: every site gives the same column
        assert np.max(np.abs(col - col.reshape(-1, 4)[0])) < 1e-14
        M[:, c] = col.reshape(-1, 4)[0]
    return M


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_massless_symbol_is_exact_exponential(oracle, axis):
    n, dx = 32, 0.01
    alpha = R.dirac_alpha(axis)
    for j in range(n):
        k = 2 * np.pi * j / (n * dx)
        M = symbol(oracle, (n,), [j], dx, 0.0, (axis,))
        assert np.max(np.abs(M - scipy.linalg.expm(-1j * alpha * k * dx))) < 1e-14
        ev = np.linalg.eigvals(M)
        for e in (np.exp(-1j * k * dx), np.exp(1j * k * dx)):
            assert np.sum(np.abs(ev - e) < 1e-7) >= 2
        assert np.max(np.min(np.abs(ev[:, None] - np.array(
            [np.exp(-1j * k * dx), np.exp(1j * k * dx)])[None, :]), axis=1)) < 1e-7


def test_massive_dispersion_has_no_doubler(oracle):
    n, dx, m = 64, 0.01, 1.0
    mu = m * C * C * dx / C
    ks = 2 * np.pi * np.arange(n) / (n * dx)
    omegas = []
    for j, k in enumerate(ks):
        M = symbol(oracle, (n,), [j], dx, m, (0,))
        assert np.allclose(M.conj().T @ M, np.eye(4), atol=1e-14)
        cosw = np.trace(M).real / 4
        assert abs(cosw - np.cos(mu) * np.cos(k * dx)) < 1e-13
        ev = np.linalg.eigvals(M)
        # two doubly degenerate eigenvalues e^{-+i w}
        w = np.abs(np.angle(ev))
        assert np.max(np.abs(w - np.arccos(np.clip(cosw, -1, 1)))) < 1e-6
        omegas.append(np.arccos(np.clip(cosw, -1, 1)))
    omegas = np.array(omegas)
    # |w| minimal only at k = 0 (w = mu), maximal at k = pi/a (w = pi - mu)
    assert np.argmin(omegas) == 0
    assert abs(omegas[n // 2] - (np.pi - mu)) < 1e-12
    assert np.all(omegas[1:] > mu)
    # the central-difference operator has its second zero at k = pi/a
    E_cd = R.central_difference_symbol(ks, dx)
    assert abs(E_cd[n // 2]) < 1e-10 and abs(E_cd[0]) < 1e-12


@pytest.mark.parametrize("axes", [(0, 1), (0, 2)])
def test_2d_trace_identity_and_zone_boundary(oracle, axes):
    n, dx, m = 8, 0.01, 1.0
    mu = m * C * dx
    for jx in range(n):
        for jy in range(n):
            kx = 2 * np.pi * jx / (n * dx)
            ky = 2 * np.pi * jy / (n * dx)
            M = symbol(oracle, (n, n), [jx, jy], dx, m, axes)
            assert abs(np.trace(M).real / 4 - np.cos(mu) * np.cos(kx * dx) * np.cos(ky * dx)) < 1e-13
    # massless: quasi-energy vanishes at k = 0; on the zone boundary of one axis it is pi
    M = symbol(oracle, (n, n), [n // 2, 0], dx, 0.0, axes)
    assert np.allclose(M, -np.eye(4), atol=1e-14)
    # the zone corner aliases k = 0 for the first-order split step
    M = symbol(oracle, (n, n), [n // 2, n // 2], dx, 0.0, axes)
    assert np.allclose(M, np.eye(4), atol=1e-14)
