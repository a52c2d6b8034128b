"""Pins of the oracle's time-dependent field: a laser pulse with a linear
turn-on ramp (Sec. 2.3 names such a pulse as one whose field integral
eq:field_dis1 is known in closed form), A(t, x) = f(t) P(x),
f(t) = w(t) sin(omega t + phase), w a trapezoid envelope.

The oracle integrates f over each step by Gauss-Legendre quadrature on the
pieces between the envelope's corners.  Pinned here against scipy's adaptive
quadrature, against the closed form of the ramp written out independently,
the 16-point rule against numpy's, and the pulse step against the static
field step (a constant f) and against exact unitarity on a periodic box."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from paper_1107_4650_amd.inputs import C_LIGHT, packet, random_spinor

PULSE = dict(omega=0.057, phase=0.3, t_on=10.0, t_flat=5.0, t_off=10.0)


def _f(p, t):
    t_on, t1, t2 = p["t_on"], p["t_on"] + p["t_flat"], p["t_on"] + p["t_flat"] + p["t_off"]
    if t < 0.0 or t >= t2:
        w = 0.0
    elif t < t_on:
        w = t / t_on
    elif t < t1:
        w = 1.0
    else:
        w = (t2 - t) / p["t_off"]
    return w * math.sin(p["omega"] * t + p["phase"])


def _quad(p, a, b):
    pts = [x for x in (0.0, p["t_on"], p["t_on"] + p["t_flat"],
                       p["t_on"] + p["t_flat"] + p["t_off"]) if a < x < b]
    return quad(lambda t: _f(p, t), a, b, points=pts or None, epsabs=0.0, epsrel=1e-13,
                limit=200)[0]


def test_gauss_legendre_rule(oracle):
    x, w = oracle.gauss_legendre16()
    xr, wr = np.polynomial.legendre.leggauss(16)
    i = np.argsort(x)
    assert np.max(np.abs(x[i] - xr)) < 1e-15
    assert np.max(np.abs(w[i] - wr)) < 1e-15


@pytest.mark.parametrize("a,b", [(-1.0, -0.5), (-0.3, 0.2), (0.5, 0.5001), (3.0, 3.0 + 7.3e-5),
                                 (9.99, 10.01), (12.0, 12.5), (14.9, 15.2), (24.99, 25.3),
                                 (26.0, 27.0), (-1.0, 30.0)])
def test_pulse_integral_vs_adaptive_quadrature(oracle, a, b):
    got = oracle.pulse_integral(PULSE, a, b)
    ref = _quad(PULSE, a, b)
    assert abs(got - ref) <= 1e-13 * max(abs(ref), (b - a) * 1e-3), (got, ref)


def test_pulse_integral_fast_carrier_and_dc(oracle):
    """A carrier of many periods per interval (the quadrature must subdivide)
    and omega = 0 (a ramped constant), against scipy."""
    fast = dict(PULSE, omega=40.0)
    for a, b in ((1.0, 2.0), (9.5, 15.5)):
        ref = _quad(fast, a, b)
        assert abs(oracle.pulse_integral(fast, a, b) - ref) <= 1e-12 * max(abs(ref), 1e-3)
    dc = dict(PULSE, omega=0.0, phase=math.pi / 2)
    # w(t) integrated exactly: the ramp from 2 to 12 is 1/20 (10^2 - 2^2) + 2 = 6.8
    assert abs(oracle.pulse_integral(dc, 2.0, 12.0) - (0.05 * (100.0 - 4.0) + 2.0)) < 1e-13


def test_pulse_integral_on_the_ramp_closed_form(oracle):
    """On the turn-on ramp w = t / t_on; with phase 0 the integral of
    (t / T) sin(omega t) is [sin(omega t) - omega t cos(omega t)] / (omega^2 T)."""
    p = dict(PULSE, phase=0.0)
    om, T = p["omega"], p["t_on"]
    F = lambda t: (math.sin(om * t) - om * t * math.cos(om * t)) / (om * om * T)  # noqa: E731
    for a, b in ((1.0, 4.0), (2.0, 9.0), (0.0, 10.0)):
        assert abs(oracle.pulse_integral(p, a, b) - (F(b) - F(a))) < 1e-13


def test_constant_pulse_equals_static_field(oracle):
    """omega = 0, phase = pi/2 and a box envelope give f = 1, so each step's
    field integral is dt P: the pulse step equals the static field step with
    Atilde = dt P (to the rounding of the quadrature's weights)."""
    shape, dx, c = (40, 30), 0.02, C_LIGHT
    dt = dx / c
    rng = np.random.default_rng(3)
    psi = random_spinor(shape[::-1], seed=4)
    V = rng.uniform(-1, 1, shape[::-1]) * c * c
    P = rng.uniform(-1, 1, (3,) + shape[::-1]) * 2000.0
    box = dict(omega=0.0, phase=math.pi / 2, t_on=0.0, t_flat=1e6, t_off=0.0)
    got = oracle.step_pulse(psi, V, P, box, t0=0.1, dt=dt, c=c, m=1.0, nsteps=12, axes=(0, 1))
    ref = oracle.step_field(psi, V, dt * P, dt=dt, c=c, m=1.0, nsteps=12, axes=(0, 1))
    assert np.max(np.abs(got - ref)) < 1e-13


def test_constant_pulse_equals_static_field_3d_second_order(oracle):
    """The same identity through the 3-D second-order step (c dt = 4 a)."""
    shape, dx, c = (12, 10, 8), 0.02, C_LIGHT
    dt = 4 * dx / c
    rng = np.random.default_rng(6)
    psi = random_spinor(shape[::-1], seed=7)
    V = rng.uniform(-1, 1, shape[::-1]) * c * c
    P = rng.uniform(-1, 1, (3,) + shape[::-1]) * 500.0
    box = dict(omega=0.0, phase=math.pi / 2, t_on=0.0, t_flat=1e6, t_off=0.0)
    got = oracle.step_pulse(psi, V, P, box, t0=0.1, dt=dt, c=c, m=1.0, nsteps=5,
                            scheme="strang")
    ref = oracle.step_field(psi, V, dt * P, dt=dt, c=c, m=1.0, nsteps=5, scheme="strang")
    assert np.max(np.abs(got - ref)) < 1e-13
    free = oracle.step_strang(psi, V, dt=dt, c=c, m=1.0, nsteps=5)
    assert np.linalg.norm(got - free) > 1e-2 * np.linalg.norm(free)


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_pulse_steps_are_unitary(oracle, scheme):
    """Periodic box: transports and U are unitary, so the norm stays within
    rounding over 150 steps through the ramp of a strong pulse."""
    shape, dx, c = (48, 20), 0.02, C_LIGHT
    dt = (2 if scheme == "strang" else 1) * dx / c
    psi = packet(shape, dx, delta=0.1, p0=[20.0, 5.0], r0=[0.0, 0.0])
    P = np.zeros((3,) + shape[::-1])
    P[0], P[1], P[2] = 3000.0, -1500.0, 800.0
    pulse = dict(omega=300.0, phase=0.1, t_on=150 * dt / 2, t_flat=0.0, t_off=150 * dt)
    n0 = np.sum(np.abs(psi) ** 2)
    out = oracle.step_pulse(psi, None, P, pulse, dt=dt, c=c, m=1.0, nsteps=150, axes=(0, 1),
                            bc="periodic", scheme=scheme)
    assert abs(np.sum(np.abs(out) ** 2) / n0 - 1.0) < 1e-12
    # and the field did act: the result differs from the field-free run
    free = oracle.step_pulse(psi, None, 0.0 * P, pulse, dt=dt, c=c, m=1.0, nsteps=150,
                             axes=(0, 1), bc="periodic", scheme=scheme)
    assert np.linalg.norm(out - free) > 1e-3 * np.linalg.norm(free)


def test_pulse_step_uses_each_steps_own_interval(oracle):
    """Step n carries the integral over [t0 + n dt, t0 + (n + 1) dt]: the pulse
    step equals single static-field steps whose Atilde is P times scipy's
    integral over that interval, through the ramp's corner at t_on."""
    shape, dx, c = (30,), 0.02, C_LIGHT
    dt = dx / c
    P = np.zeros((3,) + shape[::-1])
    P[0], P[1], P[2] = 4000.0, 2500.0, -3000.0
    pulse = dict(omega=2000.0, phase=0.4, t_on=5.5 * dt, t_flat=2 * dt, t_off=3 * dt)
    psi = random_spinor(shape[::-1], seed=9)
    V = np.linspace(-1, 1, shape[0]) * c * c
    t0 = -1.5 * dt
    got = oracle.step_pulse(psi, V, P, pulse, t0=t0, dt=dt, c=c, m=1.0, nsteps=14, axes=(0,))
    ref = psi
    for n in range(14):
        F = _quad(pulse, t0 + n * dt, t0 + (n + 1) * dt)
        ref = oracle.step_field(ref, V, F * P, dt=dt, c=c, m=1.0, nsteps=1, axes=(0,))
    assert np.max(np.abs(got - ref)) < 1e-13
    # the field matters here: without it the result is far from this one
    free = oracle.step(psi, V, dt=dt, c=c, m=1.0, nsteps=14, axes=(0,))
    assert np.max(np.abs(got - free)) > 1e-2
