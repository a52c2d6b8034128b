"""Closed forms and continuum solutions the oracle is pinned to.

TEST INFRASTRUCTURE ONLY (see oracle.py).  Nothing here runs the discrete
scheme; these are the mathematics the scheme must approach.

  * free_fft: the exact free continuum evolution in Fourier space
    (App. B and App. C): psi^(t, p) = [cos(E t) - i (c alpha.p + beta m c^2)/E sin(E t)] psi^(0, p),
    applied with numpy's FFT on a box large enough that the packet never
    wraps.
  * klein_T: transmission through the smooth step V0/2 (1 + tanh(x/L))
    (Sec. 5.2.1, eq:trans_co).
  * massless 2-D packet values at r = 0 (Dawson form) and r = ct
    (2F2 forms) (Sec. 5.1.1 and App. B), in the readings listed in the
    design notes: ct (not t) in the r = 0 form, and ψ3, ψ4 at r = ct with
    the factor (ct)^2 / (2 Delta^2) and a positive sign.
  * the symbol of the central-difference operator, which has the doubler
    (Sec. 3).
"""
from __future__ import annotations

import math

import numpy as np

SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def dirac_alpha(d: int) -> np.ndarray:
    a = np.zeros((4, 4), dtype=np.complex128)
    a[:2, 2:] = SIGMA[d]
    a[2:, :2] = SIGMA[d]
    return a


BETA = np.diag([1.0, 1.0, -1.0, -1.0]).astype(np.complex128)


def free_fft(psi0: np.ndarray, dx: float, t: float, c: float, m: float, axes=None) -> np.ndarray:
    """Exact free evolution of the sampled spinor field psi0 (shape (..., 4))."""
    nd = psi0.ndim - 1
    axes = tuple(range(nd)) if axes is None else tuple(axes)
    # momentum grids, array axis k (0 = slowest) corresponds to grid dim nd-1-k
    ps = [2.0 * np.pi * np.fft.fftfreq(psi0.shape[k], d=dx) for k in range(nd)]
    mesh = np.meshgrid(*ps, indexing="ij")
    p_phys = [np.zeros_like(mesh[0]) for _ in range(3)]
    for d in range(nd):
        p_phys[axes[d]] = mesh[nd - 1 - d]
    E = np.sqrt(c * c * (p_phys[0] ** 2 + p_phys[1] ** 2 + p_phys[2] ** 2) + (m * c * c) ** 2)
    fh = np.fft.fftn(psi0, axes=tuple(range(nd)))
    H = (c * (p_phys[0][..., None, None] * dirac_alpha(0)
              + p_phys[1][..., None, None] * dirac_alpha(1)
              + p_phys[2][..., None, None] * dirac_alpha(2))
         + m * c * c * BETA)
    cosEt = np.cos(E * t)[..., None, None]
    # sin(Et)/E, finite at E = 0 (massless zero mode)
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(E > 0, np.sin(E * t) / np.where(E > 0, E, 1.0), t)[..., None, None]
    U = cosEt * np.eye(4) - 1j * H * sinc
    out = np.einsum("...ij,...j->...i", U, fh)
    return np.fft.ifftn(out, axes=tuple(range(nd)))


def klein_T(k0: float, V0: float, L: float, c: float, m: float = 1.0) -> float:
    """eq:trans_co with k = sqrt((E - V0)^2 - m^2 c^4)/c, k' = -sqrt(E^2 - m^2 c^4)/c,
    E = sqrt(k0^2 c^2 + m^2 c^4); zero where k is not real (total reflection)."""
    E = math.sqrt(k0 * k0 * c * c + m * m * c ** 4)
    disc = (E - V0) ** 2 - m * m * c ** 4
    if disc <= 0.0:
        return 0.0
    k = math.sqrt(disc) / c
    kp = -math.sqrt(E * E - m * m * c ** 4) / c
    num = math.sinh(math.pi * k * L) * math.sinh(math.pi * kp * L)
    den = (math.sinh(math.pi * (V0 / c + k + kp) * L / 2.0)
           * math.sinh(math.pi * (V0 / c - k - kp) * L / 2.0))
    return -num / den


def massless_2d_origin(ct: float, delta: float) -> float:
    """psi_1(t, 0) / N for the spin-up packet exp(-r^2/(4 Delta^2)):
    1 - 2 z F(z), z = ct / (2 Delta), F the Dawson function."""
    from scipy.special import dawsn
    z = ct / (2.0 * delta)
    return 1.0 - 2.0 * z * float(dawsn(z))


def massless_2d_front(ct: float, delta: float):
    """(psi_1, |psi_3| + |psi_4| amplitude) / N on the circle r = ct:
    psi_1 = 2F2(1/4, 3/4; 1/2, 1/2; -(ct)^2/Delta^2),
    amplitude of (psi_3, psi_4) = (ct)^2/(2 Delta^2) 2F2(5/4, 7/4; 3/2, 5/2; -(ct)^2/Delta^2);
    in the x-z plane psi_3 = amp sin(phi), psi_4 = amp cos(phi)."""
    import mpmath as mp
    x = -(ct * ct) / (delta * delta)
    p1 = float(mp.hyp2f2(0.25, 0.75, 0.5, 0.5, x))
    amp = (ct * ct) / (2.0 * delta * delta) * float(mp.hyp2f2(1.25, 1.75, 1.5, 2.5, x))
    return p1, amp


def central_difference_symbol(k: np.ndarray, a: float) -> np.ndarray:
    """Energy of the massless 1-D symmetric-difference operator, in units of c:
    E(k) = sin(k a) / a (Sec. 3), which vanishes again at k = pi / a."""
    return np.sin(k * a) / a
