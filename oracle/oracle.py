"""ctypes front end of the FP64 CPU oracle (dirac_oracle.c).

TEST INFRASTRUCTURE ONLY: the oracle is what the HIP library is checked
against.  Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  It imports nothing from the GPU package.

Arrays follow one layout: complex spinors with the component index last,
C-contiguous, shape (Nx, 4), (N1, Nx, 4) or (Nz, Ny, Nx, 4); grid dimension 0
is the fastest (x).  The potential has the grid shape, float64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dirac_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -O2, IEEE arithmetic: no contraction into FMA, no fast-math.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-Wall"]


def build(force: bool = False) -> str:
    """Compile dirac_oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # DIRAC_ORACLE_LIB: a build of the oracle from a modified copy of its
        # source, used by the test that plants mistakes to show the pins fail
        path = os.environ.get("DIRAC_ORACLE_LIB") or build()
        lib = ctypes.CDLL(path)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.c_void_p
        lib.oracle_step.argtypes = [ctypes.c_int, i64p, ip, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int64,
                                    ctypes.c_int]
        lib.oracle_adjoint_step.argtypes = lib.oracle_step.argtypes
        lib.oracle_step_strang.argtypes = lib.oracle_step.argtypes
        lib.oracle_step_field.argtypes = [ctypes.c_int, i64p, ip, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, dp,
                                          dp, dp, ctypes.c_int64, ctypes.c_int]
        lib.oracle_step_pulse.argtypes = [ctypes.c_int, i64p, ip, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double, dp,
                                          dp, dp, ctypes.c_double, dp, ctypes.c_int64,
                                          ctypes.c_int]
        lib.oracle_pulse_integral.argtypes = [dp, ctypes.c_double, ctypes.c_double]
        lib.oracle_pulse_integral.restype = ctypes.c_double
        lib.oracle_gauss_legendre.argtypes = [dp, dp]
        lib.oracle_gauss_legendre.restype = None
        lib.oracle_stream_f32.argtypes = [ctypes.c_int, i64p, ip, ctypes.c_int, dp,
                                          ctypes.c_int64, ctypes.c_int]
        lib.oracle_observables.argtypes = [ctypes.c_int, i64p, ctypes.c_double, dp, dp,
                                           ctypes.c_double, dp]
        lib.oracle_grad.argtypes = [ctypes.c_int, i64p, ip, ctypes.c_int, ctypes.c_double, dp,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp,
                                    ctypes.c_int64, ctypes.c_double, ctypes.c_int64, dp, dp, dp,
                                    ctypes.c_int]
        lib.oracle_dirac_matrices.argtypes = [dp]
        lib.oracle_max_threads.restype = ctypes.c_int
        for f in (lib.oracle_step, lib.oracle_adjoint_step, lib.oracle_step_strang,
                  lib.oracle_step_field, lib.oracle_step_pulse,
                  lib.oracle_stream_f32,
                  lib.oracle_observables, lib.oracle_grad):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _grid_args(psi: np.ndarray, axes):
    if psi.ndim < 2 or psi.shape[-1] != 4:
        raise ValueError("spinor array must have shape (..., 4)")
    ndim = psi.ndim - 1
    n = (ctypes.c_int64 * 3)(*([int(s) for s in psi.shape[-2::-1]] + [1] * (3 - ndim)))
    if axes is None:
        axes = tuple(range(ndim))
    if len(axes) != ndim:
        raise ValueError("one Dirac axis per grid dimension")
    ax = (ctypes.c_int * 3)(*(list(axes) + [0] * (3 - ndim)))
    return ndim, n, ax


def _bc(bc) -> int:
    return {"zero": 0, "periodic": 1, 0: 0, 1: 1}[bc]


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _check_V(V, psi):
    if V is None:
        return None
    V = np.ascontiguousarray(V, dtype=np.float64)
    if V.shape != psi.shape[:-1]:
        raise ValueError("V must have the grid shape")
    return V


def step(psi, V=None, *, dt, c, m, nsteps, axes=None, bc="zero", threads=0):
    """Return psi after `nsteps` Lie steps D C B A (Sec. 2.1; eq:sol_dis_1-4)."""
    psi = np.array(psi, dtype=np.complex128, order="C", copy=True)
    V = _check_V(V, psi)
    ndim, n, ax = _grid_args(psi, axes)
    rc = _load().oracle_step(ndim, n, ax, _bc(bc), dt, c, m,
                             None if V is None else _ptr(V), _ptr(psi), int(nsteps), int(threads))
    if rc:
        raise RuntimeError(f"oracle_step failed ({rc})")
    return psi


def step_strang(psi, V=None, *, dt, c, m, nsteps, axes=None, bc="zero", threads=0):
    """Return psi after `nsteps` second-order steps (Sec. 2.4).  1-D and 2-D:
    half-step transports in the order A, B, C, D over dt, half-step transports
    in the reverse order; each half step is a one-cell shift (c dt = 2a).
    3-D: A(dt/4) B(dt/2) A(dt/4) C(dt/2) D C(dt/2) A(dt/4) B(dt/2) A(dt/4),
    A a one-cell shift, B and C two-cell shifts (c dt = 4a)."""
    psi = np.array(psi, dtype=np.complex128, order="C", copy=True)
    V = _check_V(V, psi)
    ndim, n, ax = _grid_args(psi, axes)
    rc = _load().oracle_step_strang(ndim, n, ax, _bc(bc), dt, c, m,
                                    None if V is None else _ptr(V), _ptr(psi), int(nsteps),
                                    int(threads))
    if rc:
        raise RuntimeError(f"oracle_step_strang failed ({rc})")
    return psi


def step_field(psi, V=None, A=None, *, dt, c, m, nsteps, axes=None, bc="zero", scheme="lie",
               threads=0):
    """Return psi after `nsteps` steps whose local step carries a vector
    potential: D = U exp(-i V dt) with the 4x4 U of Sec. 2.3.  A: the field
    integral Atilde per cell, shape (3,) + grid (x, y, z components), or None."""
    psi = np.array(psi, dtype=np.complex128, order="C", copy=True)
    V = _check_V(V, psi)
    if A is not None:
        A = np.ascontiguousarray(A, dtype=np.float64)
        if A.shape != (3,) + psi.shape[:-1]:
            raise ValueError("A must have shape (3,) + grid")
    ndim, n, ax = _grid_args(psi, axes)
    rc = _load().oracle_step_field(ndim, n, ax, _bc(bc), {"lie": 0, "strang": 1}[scheme], dt, c,
                                   m, None if V is None else _ptr(V),
                                   None if A is None else _ptr(A), _ptr(psi), int(nsteps),
                                   int(threads))
    if rc:
        raise RuntimeError(f"oracle_step_field failed ({rc})")
    return psi


def _pulse_params(pulse) -> np.ndarray:
    return np.ascontiguousarray([float(pulse[k]) for k in
                                 ("omega", "phase", "t_on", "t_flat", "t_off")], dtype=np.float64)


def pulse_integral(pulse, ta, tb) -> float:
    """int_ta^tb f(t) dt for the pulse f(t) = w(t) sin(omega t + phase) with
    the trapezoid envelope w (dict with omega, phase, t_on, t_flat, t_off)."""
    pp = _pulse_params(pulse)
    return float(_load().oracle_pulse_integral(_ptr(pp), float(ta), float(tb)))


def gauss_legendre16():
    """The oracle's 16-point Gauss-Legendre nodes and weights on [-1, 1]."""
    x = np.zeros(16)
    w = np.zeros(16)
    _load().oracle_gauss_legendre(_ptr(x), _ptr(w))
    return x, w


def step_pulse(psi, V=None, P=None, pulse=None, *, t0=0.0, dt, c, m, nsteps, axes=None,
               bc="zero", scheme="lie", threads=0):
    """Return psi after `nsteps` steps whose local step carries the field
    integral Atilde^n = P * int_{t_n}^{t_{n+1}} f of the pulse f (t_n =
    t0 + n dt); P: shape (3,) + grid."""
    psi = np.array(psi, dtype=np.complex128, order="C", copy=True)
    V = _check_V(V, psi)
    P = np.ascontiguousarray(P, dtype=np.float64)
    if P.shape != (3,) + psi.shape[:-1]:
        raise ValueError("P must have shape (3,) + grid")
    pp = _pulse_params(pulse)
    ndim, n, ax = _grid_args(psi, axes)
    rc = _load().oracle_step_pulse(ndim, n, ax, _bc(bc), {"lie": 0, "strang": 1}[scheme], dt, c,
                                   m, None if V is None else _ptr(V), _ptr(P), _ptr(pp),
                                   float(t0), _ptr(psi), int(nsteps), int(threads))
    if rc:
        raise RuntimeError(f"oracle_step_pulse failed ({rc})")
    return psi


def adjoint_step(lam, V=None, *, dt, c, m, nsteps, axes=None, bc="zero", threads=0):
    """Return (S^H)^nsteps lam, the adjoint of `step`."""
    lam = np.array(lam, dtype=np.complex128, order="C", copy=True)
    V = _check_V(V, lam)
    ndim, n, ax = _grid_args(lam, axes)
    rc = _load().oracle_adjoint_step(ndim, n, ax, _bc(bc), dt, c, m,
                                     None if V is None else _ptr(V), _ptr(lam), int(nsteps),
                                     int(threads))
    if rc:
        raise RuntimeError(f"oracle_adjoint_step failed ({rc})")
    return lam


def stream_f32(psi, *, nsteps, axes=None, bc="zero", threads=0):
    """Float instance of the transport sub-steps only (m = 0, V = 0, D skipped)."""
    psi = np.array(psi, dtype=np.complex64, order="C", copy=True)
    ndim, n, ax = _grid_args(psi, axes)
    rc = _load().oracle_stream_f32(ndim, n, ax, _bc(bc), _ptr(psi), int(nsteps), int(threads))
    if rc:
        raise RuntimeError(f"oracle_stream_f32 failed ({rc})")
    return psi


def observables(psi, *, dx, xmin, x_b):
    """(N, <x0>, <x1>, <x2>, P_T) as defined in dirac_oracle.c."""
    psi = np.ascontiguousarray(psi, dtype=np.complex128)
    ndim, n, _ = _grid_args(psi, None)
    xm = np.zeros(3)
    xm[:ndim] = np.asarray(xmin, dtype=np.float64).reshape(-1)[:ndim]
    out = np.zeros(5)
    rc = _load().oracle_observables(ndim, n, dx, _ptr(xm), _ptr(psi), x_b, _ptr(out))
    if rc:
        raise RuntimeError(f"oracle_observables failed ({rc})")
    return out


def grad(psi0, V, *, dx, xmin, dt, c, m, nsteps, x_b, axes=None, bc="zero", ckpt=16,
         threads=0):
    """Return (loss, dL/dV, psi_N) for L = P_T(psi_N) (see oracle_grad)."""
    psi0 = np.ascontiguousarray(psi0, dtype=np.complex128)
    V = _check_V(V, psi0)
    ndim, n, ax = _grid_args(psi0, axes)
    xm = np.zeros(3)
    xm[:ndim] = np.asarray(xmin, dtype=np.float64).reshape(-1)[:ndim]
    dLdV = np.zeros(psi0.shape[:-1])
    psiN = np.zeros_like(psi0)
    loss = np.zeros(1)
    rc = _load().oracle_grad(ndim, n, ax, _bc(bc), dx, _ptr(xm), dt, c, m,
                             None if V is None else _ptr(V), _ptr(psi0), int(nsteps), x_b,
                             int(ckpt), _ptr(dLdV), _ptr(psiN), _ptr(loss), int(threads))
    if rc:
        raise RuntimeError(f"oracle_grad failed ({rc})")
    return float(loss[0]), dLdV, psiN


def dirac_matrices():
    """(alpha_x, alpha_y, alpha_z, beta) as the oracle builds them."""
    buf = np.zeros(4 * 16 * 2)
    _load().oracle_dirac_matrices(_ptr(buf))
    z = buf[0::2] + 1j * buf[1::2]
    z = z.reshape(4, 4, 4)
    return z[0], z[1], z[2], z[3]


def max_threads() -> int:
    return int(_load().oracle_max_threads())
