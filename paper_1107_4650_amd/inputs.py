"""Seeded synthetic inputs: Gaussian spinor packets and potentials.

This module only draws and samples initial data and potentials; it holds
none of the time-stepping arithmetic.  Both the oracle-based tests and the GPU
path take their inputs from here.

Conventions (atomic units, Sec. 5):
  * c = 137.036 (1/alpha), m = 1, hbar = |e| = 1.
  * Grid dimension 0 is the fastest (x).  Arrays are C-contiguous with the
    spinor component last: (Nx, 4), (N1, Nx, 4), (Nz, Ny, Nx, 4).
  * Cell centres x_d = xmin_d + (i + 1/2) dx (Sec. 2.3); by default the box is
    symmetric, xmin_d = -n_d dx / 2.
  * V is the potential energy at the cell centres (it enters the Hamiltonian
    as + V times the identity).
  * A packet is  psi0 = N u(p0) exp(i p0.r) exp(-|r - r0|^2 / (4 Delta^2))
    with the free positive-energy spin-up spinor
        u(p) = (1, 0, c p_z / (E + m c^2), c (p_x + i p_y) / (E + m c^2)),
        E = sqrt(c^2 p^2 + m^2 c^4),
    which for p along x is the paper's travelling packet (eq:trav_wave), and
    N fixed so that dV * sum |psi0|^2 = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 137.036
M_E = 1.0


def default_xmin(shape_x_first, dx):
    return [-n * dx / 2.0 for n in shape_x_first]


def centres(n: int, dx: float, xmin: float) -> np.ndarray:
    return xmin + (np.arange(n, dtype=np.float64) + 0.5) * dx


def _grid_axes(shape_x_first, dx, xmin):
    if xmin is None:
        xmin = default_xmin(shape_x_first, dx)
    return [centres(n, dx, x0) for n, x0 in zip(shape_x_first, xmin)], list(xmin)


def spinor_u(p_phys, c=C_LIGHT, m=M_E, kind="positive"):
    """Spinor of the packet.  kind='positive': u(p) above; 'spin_up': (1,0,0,0)."""
    if kind == "spin_up":
        return np.array([1, 0, 0, 0], dtype=np.complex128)
    px, py, pz = p_phys
    E = math.sqrt(c * c * (px * px + py * py + pz * pz) + m * m * c ** 4)
    den = E + m * c * c
    return np.array([1.0, 0.0, c * pz / den, c * (px + 1j * py) / den], dtype=np.complex128)


def packet(shape_x_first, dx, *, delta, p0=None, r0=None, axes=None, c=C_LIGHT, m=M_E,
           xmin=None, kind="positive", normalise=True) -> np.ndarray:
    """Gaussian packet on a grid given as (n_x, n_1, ...), x first.

    p0, r0: per grid dimension.  axes: physical axis (0=x, 1=y, 2=z) carried by
    each grid dimension (default 0, 1, 2).  Returns complex128 of shape
    (..., n_1, n_x, 4)."""
    nd = len(shape_x_first)
    axes = tuple(range(nd)) if axes is None else tuple(axes)
    p0 = [0.0] * nd if p0 is None else list(p0)
    r0 = [0.0] * nd if r0 is None else list(r0)
    coords, _ = _grid_axes(shape_x_first, dx, xmin)
    p_phys = [0.0, 0.0, 0.0]
    for d in range(nd):
        p_phys[axes[d]] = p0[d]
    u = spinor_u(p_phys, c, m, kind)
    # separable scalar envelope, built dimension by dimension
    f = np.ones((1,) * nd, dtype=np.complex128)
    for d in range(nd):
        x = coords[d]
        g = np.exp(1j * p0[d] * x) * np.exp(-((x - r0[d]) ** 2) / (4.0 * delta * delta))
        shape = [1] * nd
        shape[nd - 1 - d] = len(x)
        f = f * g.reshape(shape)
    psi = f[..., None] * u
    if normalise:
        dV = dx ** nd
        psi = psi / math.sqrt(dV * float(np.sum(np.abs(psi) ** 2)))
    return np.ascontiguousarray(psi)


def coord_mesh(shape_x_first, dx, xmin=None):
    """Broadcastable coordinate arrays (x, x1, x2) in array order."""
    coords, _ = _grid_axes(shape_x_first, dx, xmin)
    nd = len(shape_x_first)
    out = []
    for d in range(nd):
        shape = [1] * nd
        shape[nd - 1 - d] = shape_x_first[d]
        out.append(coords[d].reshape(shape))
    return out


def potential_step(shape_x_first, dx, V0, xmin=None):
    """V = V0 * Theta(x): 1 for cell centres with x > 0."""
    X = coord_mesh(shape_x_first, dx, xmin)[0]
    return np.broadcast_to(np.where(X > 0, float(V0), 0.0), tuple(shape_x_first[::-1])).copy()


def potential_tanh(shape_x_first, dx, V0, L, xmin=None):
    """V = V0 * tanh(x / L)."""
    X = coord_mesh(shape_x_first, dx, xmin)[0]
    return np.broadcast_to(V0 * np.tanh(X / L), tuple(shape_x_first[::-1])).copy()


def potential_sauter(shape_x_first, dx, V0, L, xmin=None):
    """Smooth Klein step V = V0/2 (1 + tanh(x / L)) (Sec. 5.2.1)."""
    X = coord_mesh(shape_x_first, dx, xmin)[0]
    return np.broadcast_to(0.5 * V0 * (1.0 + np.tanh(X / L)), tuple(shape_x_first[::-1])).copy()


def potential_sphere(shape_x_first, dx, V0, xmin=None, width2=4.0):
    """V = V0 exp(-r^2 / width2)."""
    mesh = coord_mesh(shape_x_first, dx, xmin)
    r2 = sum(x * x for x in mesh)
    return np.ascontiguousarray(np.broadcast_to(V0 * np.exp(-r2 / width2),
                                                tuple(shape_x_first[::-1])))


def bump_basis(shape_x_first, dx, centres_xy, sigma, xmin=None) -> np.ndarray:
    """Unit Gaussian bumps g_j(r) = exp(-|r - r_j|^2 / (2 sigma^2)), shape (nb, grid)."""
    mesh = coord_mesh(shape_x_first, dx, xmin)
    G = []
    for rj in centres_xy:
        r2 = sum((mesh[d] - rj[d]) ** 2 for d in range(len(mesh)))
        G.append(np.broadcast_to(np.exp(-r2 / (2.0 * sigma * sigma)), tuple(shape_x_first[::-1])))
    return np.ascontiguousarray(np.stack(G))


@dataclass
class Workload:
    """One Dirac run: grid, constants, initial spinor (complex128) and V (float64)."""
    name: str
    shape: tuple                 # grid shape, x first
    dx: float
    dt: float
    c: float
    m: float
    nsteps: int
    psi0: np.ndarray
    V: np.ndarray | None
    axes: tuple = (0, 1, 2)
    bc: str = "zero"
    xmin: list = field(default_factory=list)
    extra: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def sites(self):
        return int(np.prod(self.shape))


def config_1d_step(n=4096, nsteps=2000) -> Workload:
    """1-D, N = 4096, dx = 0.01, Delta = 2, p0 = 50 at x0 = -10, V = 2 m c^2 Theta(x)."""
    dx, c, m = 0.01, C_LIGHT, M_E
    shape = (n,)
    xmin = default_xmin(shape, dx)
    psi = packet(shape, dx, delta=2.0, p0=[50.0], r0=[-10.0], c=c, m=m)
    V = potential_step(shape, dx, 2.0 * m * c * c)
    return Workload("1d-step-4096", shape, dx, dx / c, c, m, nsteps, psi, V, (0,), "zero", xmin)


def config_2d_tanh(n=2048, nsteps=10000, seed=0, dx=0.01) -> Workload:
    """2-D (x, y), Delta = 1.5, p0 = (40, 0), seed-drawn centre and barrier
    height, V = V0 tanh(x / 0.1) with V0 ~ U[0, 3] m c^2."""
    c, m = C_LIGHT, M_E
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-6.0, -3.0)
    y0 = rng.uniform(-2.0, 2.0)
    V0 = rng.uniform(0.0, 3.0) * m * c * c
    shape = (n, n)
    xmin = default_xmin(shape, dx)
    psi = packet(shape, dx, delta=1.5, p0=[40.0, 0.0], r0=[x0, y0], c=c, m=m)
    V = potential_tanh(shape, dx, V0, 0.1)
    return Workload(f"2d-tanh-{n}", shape, dx, dx / c, c, m, nsteps, psi, V, (0, 1), "zero",
                    xmin, {"x0": x0, "y0": y0, "V0": V0})


def config_3d_sphere(n=512, nsteps=2000, dx=0.02) -> Workload:
    """3-D, Delta = 2, p0 = (30, 10, 0) at (-2.5, 0, 0), V = 1.5 m c^2 exp(-r^2/4)."""
    c, m = C_LIGHT, M_E
    shape = (n, n, n)
    xmin = default_xmin(shape, dx)
    psi = packet(shape, dx, delta=2.0, p0=[30.0, 10.0, 0.0], r0=[-2.5, 0.0, 0.0], c=c, m=m)
    V = potential_sphere(shape, dx, 1.5 * m * c * c)
    return Workload(f"3d-sphere-{n}", shape, dx, dx / c, c, m, nsteps, psi, V, (0, 1, 2),
                    "zero", xmin)


def config_adjoint(n=1024, nsteps=4000, nb=64, dx=0.02, seed_pos=1, seed_amp=2) -> Workload:
    """2-D (x, y) periodic, Delta = 1, p0 = (20, 0) at (-5, 0);
    V = m c^2 sum_j theta_j g_j, g_j unit Gaussians of sigma 0.5 at r_j ~ U[-3, 3]^2,
    theta_j ~ U[-1, 1]; loss = probability past x_b = 5."""
    c, m = C_LIGHT, M_E
    shape = (n, n)
    xmin = default_xmin(shape, dx)
    rj = np.random.default_rng(seed_pos).uniform(-3.0, 3.0, size=(nb, 2))
    theta = np.random.default_rng(seed_amp).uniform(-1.0, 1.0, size=nb)
    G = bump_basis(shape, dx, rj, 0.5)
    dVdtheta = (m * c * c) * G
    V = np.tensordot(theta, dVdtheta, axes=1)
    psi = packet(shape, dx, delta=1.0, p0=[20.0, 0.0], r0=[-5.0, 0.0], c=c, m=m)
    return Workload(f"adjoint-{n}", shape, dx, dx / c, c, m, nsteps, psi, V, (0, 1), "periodic",
                    xmin, {"theta": theta, "centres": rj, "dVdtheta": dVdtheta, "x_b": 5.0})


def config_batch(count=256, nsteps=5000, seed=0, dx=0.01, sides=(256, 512, 1024),
                 n1d=(1024, 65536), max_side=None):
    """Batched instances: a fair coin picks 1-D or 2-D; 1-D N log-uniform in
    n1d; 2-D side uniform in `sides`; V0 ~ U[0, 3] m c^2 (tanh step, L = 0.1),
    p0 ~ U[10, 80] along x, Delta = 1.5, centre at -1/4 of the box."""
    c, m = C_LIGHT, M_E
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        two_d = rng.random() < 0.5
        if two_d:
            side = int(rng.choice(sides))
            if max_side:
                side = min(side, max_side)
            shape = (side, side)
        else:
            lo, hi = math.log2(n1d[0]), math.log2(n1d[1])
            shape = (int(round(2.0 ** rng.uniform(lo, hi))),)
        V0 = rng.uniform(0.0, 3.0) * m * c * c
        p0 = rng.uniform(10.0, 80.0)
        xmin = default_xmin(shape, dx)
        r0 = [xmin[0] / 2.0] + [0.0] * (len(shape) - 1)
        psi = packet(shape, dx, delta=1.5, p0=[p0] + [0.0] * (len(shape) - 1), r0=r0, c=c, m=m)
        V = potential_tanh(shape, dx, V0, 0.1)
        axes = tuple(range(len(shape)))
        out.append(Workload(f"batch-{k}", shape, dx, dx / c, c, m, nsteps, psi, V, axes, "zero",
                            xmin, {"V0": V0, "p0": p0}))
    return out


# The 2-D Klein run of Sec. 5.2.2: x-z plane, box x in [-15, 15], z in [-5, 5],
# packet k0 = 100 along x with Delta = 1 and spinor (1, 0, 0, C), Sauter step
# of thickness L = 0.0025 at x = 0, second-order steps with c dt = 2a.  The
# paper's grid is 24576 x 8192 cells and 12000 steps (t = 0.214).  Readings:
# the height is V0 = 2 m c^2 + 1e4 (the printed m c^2 + 1e4 lies in the total
# reflection window; 2 m c^2 + 1e4 gives the printed analytic T = 0.2621), and
# the packet starts at (x0, z0) = (-10, 0) as in the 1-D run.
KLEIN2D = dict(x_half=15.0, z_half=5.0, k0=100.0, delta=1.0, L=0.0025, x0=-10.0, z0=0.0,
               extra_height=1.0e4)


def klein2d_factors(nx=24576, nz=8192, c=C_LIGHT, m=M_E):
    """Separable pieces of the 2-D Klein inputs (so that large grids can be
    assembled on the device): cell-centre coordinates, the normalised 1-D
    envelopes along x and z, the spinor, the potential along x, dx and dt."""
    k = KLEIN2D
    dx = 2.0 * k["x_half"] / nx
    if abs(2.0 * k["z_half"] / nz - dx) > 1e-15 * dx:
        raise ValueError("the x and z cells must be equal: nx / nz = 3")
    xs = centres(nx, dx, -k["x_half"])
    zs = centres(nz, dx, -k["z_half"])
    gx = np.exp(1j * k["k0"] * xs) * np.exp(-((xs - k["x0"]) ** 2) / (4.0 * k["delta"] ** 2))
    gz = np.exp(-((zs - k["z0"]) ** 2) / (4.0 * k["delta"] ** 2)).astype(np.complex128)
    u = spinor_u([k["k0"], 0.0, 0.0], c, m)
    # dV sum |gz gx u|^2 = 1
    gx = gx / math.sqrt(dx * float(np.sum(np.abs(gx) ** 2)))
    gz = gz / math.sqrt(dx * float(np.sum(np.abs(gz) ** 2)) * float(np.sum(np.abs(u) ** 2)))
    V0 = 2.0 * m * c * c + k["extra_height"]
    Vx = 0.5 * V0 * (1.0 + np.tanh(xs / k["L"]))
    return dict(dx=dx, dt=2.0 * dx / c, xs=xs, zs=zs, gx=gx, gz=gz, u=u, Vx=Vx, V0=V0,
                xmin=[-k["x_half"], -k["z_half"]])


def klein2d_workload(nx=24576, nz=8192, nsteps=12000) -> Workload:
    """The 2-D Klein run as host arrays (for grids small enough to hold)."""
    c, m = C_LIGHT, M_E
    f = klein2d_factors(nx, nz, c, m)
    psi = (f["gz"][:, None, None] * f["gx"][None, :, None]) * f["u"][None, None, :]
    V = np.ascontiguousarray(np.broadcast_to(f["Vx"][None, :], (nz, nx)))
    return Workload(f"klein2d-{nx}x{nz}", (nx, nz), f["dx"], f["dt"], c, m, nsteps,
                    np.ascontiguousarray(psi), V, (0, 2), "zero", f["xmin"],
                    {"V0": f["V0"], "scheme": "strang"})


def random_spinor(shape_arr, seed=0, dtype=np.complex128, scale=1.0) -> np.ndarray:
    """Uniform random complex spinor field in [-scale, scale] (re and im), for
    parity checks that must not depend on smoothness."""
    rng = np.random.default_rng(seed)
    re = rng.uniform(-scale, scale, size=tuple(shape_arr) + (4,))
    im = rng.uniform(-scale, scale, size=tuple(shape_arr) + (4,))
    return (re + 1j * im).astype(dtype)
