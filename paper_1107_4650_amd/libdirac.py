"""Python binding of libdirac (ctypes): argument marshalling only.

Every computation runs in the HIP library; this module checks tensor
metadata, passes raw device pointers and the current HIP stream, and turns
non-OK status codes into exceptions.  Importing it does not need a GPU;
loading fails loudly if libdirac.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libdirac.so")

DL_OK, DL_ERR_ARG, DL_ERR_CFL, DL_ERR_DTYPE, DL_ERR_ALIGN, DL_ERR_NOMEM, DL_ERR_HIP, DL_ERR_STATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
DL_ERR_NONFINITE, DL_WARN_NORM = -8, 1
STATUS_NAMES = {0: "DL_OK", -1: "DL_ERR_ARG", -2: "DL_ERR_CFL", -3: "DL_ERR_DTYPE",
                -4: "DL_ERR_ALIGN", -5: "DL_ERR_NOMEM", -6: "DL_ERR_HIP", -7: "DL_ERR_STATE",
                -8: "DL_ERR_NONFINITE", 1: "DL_WARN_NORM"}
DL_C64, DL_C128 = 0, 1
DL_BC_ZERO, DL_BC_PERIODIC = 0, 1
DL_DRY, DL_GRAPH, DL_STRANG, DL_BISPINOR = 1, 2, 4, 8

# every entry point of include/libdirac.h
EXPORTS = ("dl_plan_create", "dl_plan_destroy", "dl_step", "dl_step_field", "dl_step_pulse",
           "dl_step_out",
           "dl_step_fused_out",
           "dl_observables", "dl_step_observables", "dl_observables_noalloc",
           "dl_plan_set_norm_check",
           "dl_seed_adjoint",
           "dl_grad_step", "dl_project", "dl_expand", "dl_batch_create", "dl_batch_step",
           "dl_plan_set_tiling", "dl_plan_set_depth", "dl_plan_info", "dl_batch_set",
           "dl_batch_autotune", "dl_last_error", "dl_version")


class DiracError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class NormWarning(UserWarning):
    """dl_observables reported DL_WARN_NORM: the norm left the band of the
    plan's norm check."""


class Pulse(ctypes.Structure):
    """dl_pulse: f(t) = w(t) sin(omega t + phase), w the trapezoid envelope
    (rise t_on, plateau t_flat, fall t_off)."""
    _fields_ = [("omega", ctypes.c_double), ("phase", ctypes.c_double),
                ("t_on", ctypes.c_double), ("t_flat", ctypes.c_double),
                ("t_off", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int64 * 3), ("axis", ctypes.c_int * 3),
                ("xmin", ctypes.c_double * 3)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libdirac.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    # The library must run on PyTorch's HIP runtime (the tensors it is handed
    # are PyTorch's): importing torch first puts that runtime in the process's
    # global scope, where libdirac's HIP symbols then resolve.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "dl_plan_create": [P(vp), P(Grid), dbl, dbl, dbl, dbl, ci, ci, ctypes.c_uint],
        "dl_plan_destroy": [vp],
        "dl_step": [vp, vp, vp, i64, vp],
        "dl_step_out": [vp, vp, vp, vp, vp],
        "dl_step_field": [vp, vp, vp, vp, i64, vp],
        "dl_step_pulse": [vp, vp, vp, vp, P(Pulse), dbl, i64, vp],
        "dl_step_fused_out": [vp, vp, vp, vp, i64, vp],
        "dl_plan_set_depth": [vp, ci],
        "dl_observables": [vp, vp, dbl, P(dbl), vp],
        "dl_step_observables": [vp, vp, vp, i64, dbl, P(dbl), vp],
        "dl_plan_set_norm_check": [vp, dbl, dbl],
        "dl_observables_noalloc": [P(Grid), dbl, ci, ctypes.c_uint, vp, dbl, vp, vp],
        "dl_seed_adjoint": [vp, vp, dbl, vp, vp, vp],
        "dl_grad_step": [vp, vp, vp, vp, vp, i64, vp],
        "dl_project": [vp, vp, vp, ci, vp, vp],
        "dl_expand": [vp, vp, vp, ci, vp, vp],
        "dl_batch_create": [P(vp), P(Grid), P(dbl), P(dbl), P(dbl), P(dbl), ci, ci, ci,
                            ctypes.c_uint],
        "dl_batch_step": [vp, P(vp), P(vp), P(i64), vp],
        "dl_plan_set_tiling": [vp, ci, ci, ci, ci],
        "dl_batch_autotune": [vp, P(vp), P(vp), ci, P(ci), vp],
        "dl_batch_set": [vp, ci, ci],
        "dl_plan_info": [vp, P(i64), ci],
        "dl_version": [],
        "dl_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ci
    lib.dl_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(code: int):
    if code != DL_OK:
        raise DiracError(code, load().dl_last_error().decode())


def _dtype_code(dtype) -> int:
    s = str(dtype)
    if s in ("c64", "complex64", "torch.complex64"):
        return DL_C64
    if s in ("c128", "complex128", "torch.complex128"):
        return DL_C128
    raise ValueError(f"unknown dtype {dtype}")


def _bc_code(bc) -> int:
    return {"zero": DL_BC_ZERO, "periodic": DL_BC_PERIODIC, 0: 0, 1: 1}[bc]


def make_grid(shape, axes=None, xmin=None, dx=None) -> Grid:
    """shape: cells per grid dimension, x first."""
    nd = len(shape)
    g = Grid()
    g.ndim = nd
    for d in range(3):
        g.n[d] = int(shape[d]) if d < nd else 1
        g.axis[d] = (int(axes[d]) if axes is not None else d) if d < nd else 0
        if xmin is not None and d < nd:
            g.xmin[d] = float(xmin[d])
        elif dx is not None and d < nd:
            g.xmin[d] = -0.5 * shape[d] * dx
        else:
            g.xmin[d] = 0.0
    return g


def _stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Plan:
    """A libdirac plan for one grid (see include/libdirac.h)."""

    def __init__(self, shape, dx, dt, c, m, dtype="c64", bc="zero", axes=None, xmin=None,
                 dry=False, graph=False, scheme="lie", bispinor=False):
        """scheme: "lie" (lowest order, c dt = dx) or "strang" (second order,
        c dt = 2 dx on 1-D and 2-D grids, 4 dx on 3-D grids).  bispinor: 1-D line stored as the
        pair of components that contains psi_1 (tensor shape (n, 2))."""
        if scheme not in ("lie", "strang"):
            raise ValueError(f"unknown scheme {scheme!r}")
        self.lib = load()
        self.shape = tuple(int(s) for s in shape)           # x first
        self.tshape = tuple(reversed(self.shape)) + (2 if bispinor else 4,)  # tensor shape
        self.dtype_code = _dtype_code(dtype)
        self.dx, self.dt, self.c, self.m = float(dx), float(dt), float(c), float(m)
        self.bc = bc
        self.grid = make_grid(self.shape, axes, xmin, dx)
        flags = ((DL_DRY if dry else 0) | (DL_GRAPH if graph else 0)
                 | (DL_STRANG if scheme == "strang" else 0) | (DL_BISPINOR if bispinor else 0))
        h = ctypes.c_void_p()
        check(self.lib.dl_plan_create(ctypes.byref(h), ctypes.byref(self.grid), self.dx, self.dt,
                                      self.c, self.m, self.dtype_code, _bc_code(bc), flags))
        self.handle = h

    # -- tensor checks --------------------------------------------------------
    def _state(self, t, name="psi"):
        import torch
        want = torch.complex64 if self.dtype_code == DL_C64 else torch.complex128
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != want:
            raise TypeError(f"{name} must be {want}, got {t.dtype}")
        if tuple(t.shape) != self.tshape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.tshape}")
        return ctypes.c_void_p(t.data_ptr())

    def _cells(self, t, name, allow_none=True):
        import torch
        if t is None:
            if allow_none:
                return None
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if tuple(t.shape) != self.tshape[:-1] or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.tshape[:-1]}")
        return ctypes.c_void_p(t.data_ptr())

    # -- operations -------------------------------------------------------------
    def step(self, psi, V=None, nsteps=1):
        check(self.lib.dl_step(self.handle, self._state(psi), self._cells(V, "V"), int(nsteps),
                               _stream_handle()))
        return psi

    def step_field(self, psi, V=None, A=None, nsteps=1):
        """dl_step with the field integrals A (float64, shape (3,) + grid) in
        the local step."""
        check(self.lib.dl_step_field(self.handle, self._state(psi), self._cells(V, "V"),
                                     self._field(A), int(nsteps), _stream_handle()))
        return psi

    def step_pulse(self, psi, V=None, P=None, pulse=None, t0=0.0, nsteps=1):
        """dl_step_pulse: steps whose field integral is P times the integral
        of the pulse over each step; pulse: dict (omega, phase, t_on, t_flat,
        t_off); P: float64, shape (3,) + grid."""
        if P is None or pulse is None:
            raise ValueError("P and pulse are required")
        pk = Pulse(*[float(pulse[k]) for k in ("omega", "phase", "t_on", "t_flat", "t_off")])
        check(self.lib.dl_step_pulse(self.handle, self._state(psi), self._cells(V, "V"),
                                     self._field(P), ctypes.byref(pk), float(t0), int(nsteps),
                                     _stream_handle()))
        return psi

    def _field(self, A):
        import torch
        if A is None:
            return None
        if not isinstance(A, torch.Tensor) or A.device.type != "cuda" or A.dtype != torch.float64:
            raise TypeError("A must be a float64 CUDA tensor")
        if tuple(A.shape) != (3,) + self.tshape[:-1] or not A.is_contiguous():
            raise ValueError(f"A must be contiguous with shape {(3,) + self.tshape[:-1]}")
        return ctypes.c_void_p(A.data_ptr())

    def step_out(self, src, dst, V=None):
        check(self.lib.dl_step_out(self.handle, self._state(src, "src"), self._state(dst, "dst"),
                                   self._cells(V, "V"), _stream_handle()))
        return dst

    def step_fused_out(self, src, dst, V=None, nsteps=2):
        check(self.lib.dl_step_fused_out(self.handle, self._state(src, "src"),
                                         self._state(dst, "dst"), self._cells(V, "V"),
                                         int(nsteps), _stream_handle()))
        return dst

    def set_depth(self, depth):
        """Cap on the steps fused into one pass over memory (1 .. 5)."""
        check(self.lib.dl_plan_set_depth(self.handle, int(depth)))

    def observables(self, psi, x_b=0.0) -> np.ndarray:
        """[N, <x>, <y>, <z>, P_T].  Raises DiracError (DL_ERR_NONFINITE) for a
        state holding a NaN or an infinity; warns (NormWarning) when the norm
        check set with set_norm_check trips."""
        out = (ctypes.c_double * 5)()
        rc = self.lib.dl_observables(self.handle, self._state(psi), float(x_b), out,
                                     _stream_handle())
        return self._observables_result(rc, out)

    def step_observables(self, psi, V=None, nsteps=1, x_b=0.0) -> np.ndarray:
        """step(psi, V, nsteps), then observables(psi, x_b), in one call: on 2-D
        lowest-order plans the last pass sums the observables as it stores
        the state (dl_step_observables)."""
        out = (ctypes.c_double * 5)()
        rc = self.lib.dl_step_observables(self.handle, self._state(psi), self._cells(V, "V"),
                                          int(nsteps), float(x_b), out, _stream_handle())
        return self._observables_result(rc, out)

    def _observables_result(self, rc, out) -> np.ndarray:
        if rc == DL_WARN_NORM:
            import warnings
            warnings.warn(self.lib.dl_last_error().decode(), NormWarning, stacklevel=3)
        else:
            check(rc)
        return np.array(out[:])

    def set_norm_check(self, N_ref, tol):
        """Norm watchdog of observables(): warn when N > N_ref (1 + tol), or on a
        periodic box N < N_ref (1 - tol); tol = 0 turns it off."""
        check(self.lib.dl_plan_set_norm_check(self.handle, float(N_ref), float(tol)))

    def seed_adjoint(self, psi, x_b, lam, Q):
        check(self.lib.dl_seed_adjoint(self.handle, self._state(psi), float(x_b),
                                       self._state(lam, "lam"), self._cells(Q, "Q", False),
                                       _stream_handle()))

    def grad_step(self, psi, lam, V, Q, nsteps):
        check(self.lib.dl_grad_step(self.handle, self._state(psi), self._state(lam, "lam"),
                                    self._cells(V, "V"), self._cells(Q, "Q", False), int(nsteps),
                                    _stream_handle()))

    def project(self, Q, G, out):
        import torch
        nb = int(G.shape[0])
        if G.dtype != torch.float64 or not G.is_contiguous() or G.device.type != "cuda":
            raise TypeError("G must be a contiguous float64 CUDA tensor")
        if tuple(G.shape[1:]) != self.tshape[:-1]:
            raise ValueError("G must have shape (nb,) + grid shape")
        if out.dtype != torch.float64 or out.numel() != nb or out.device.type != "cuda":
            raise TypeError("out must be a float64 CUDA tensor of nb elements")
        check(self.lib.dl_project(self.handle, self._cells(Q, "Q", False),
                                  ctypes.c_void_p(G.data_ptr()), nb,
                                  ctypes.c_void_p(out.data_ptr()), _stream_handle()))
        return out

    def expand(self, G, theta, V):
        import torch
        nb = int(G.shape[0])
        for t, name in ((G, "G"), (theta, "theta"), (V, "V")):
            if t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda":
                raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
        if tuple(G.shape[1:]) != self.tshape[:-1] or theta.numel() != nb:
            raise ValueError("G must have shape (nb,) + grid shape and theta nb elements")
        check(self.lib.dl_expand(self.handle, ctypes.c_void_p(G.data_ptr()),
                                 ctypes.c_void_p(theta.data_ptr()), nb,
                                 self._cells(V, "V", False), _stream_handle()))
        return V

    def set_tiling(self, waves_per_cu=0, seg_len=0, allow_resident=True, graph_pairs=32):
        """Tuning knobs: waves_per_cu 0 sizes the grid from the kernel's
        occupancy; seg_len 0 derives the march segment from it."""
        check(self.lib.dl_plan_set_tiling(self.handle, int(waves_per_cu), int(seg_len),
                                          int(bool(allow_resident)), int(graph_pairs)))

    def info(self) -> dict:
        buf = (ctypes.c_int64 * 15)()
        check(self.lib.dl_plan_info(self.handle, buf, 15))
        keys = ("blocks", "seg_len", "nseg", "nstrips", "ntiles", "resident", "res_threads",
                "waves_per_cu", "xcd_remap", "graph_pairs", "depth", "blocks_1", "reverse_depth",
                "field_depth", "deep_1d_depth")
        return dict(zip(keys, buf[:]))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dl_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Independent 1-D / 2-D instances advanced by shared launches."""

    def __init__(self, shapes, dx, dt, c, m, dtype="c64", bc="zero", axes=None, xmins=None,
                 dry=False, graph=True):
        self.lib = load()
        self.count = len(shapes)
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.tshapes = [tuple(reversed(s)) + (4,) for s in self.shapes]
        self.dtype_code = _dtype_code(dtype)
        grids = (Grid * self.count)()
        for k, s in enumerate(self.shapes):
            g = make_grid(s, None if axes is None else axes[k],
                          None if xmins is None else xmins[k], _at(dx, k))
            grids[k] = g
        arr = lambda v: (ctypes.c_double * self.count)(*[_at(v, k) for k in range(self.count)])
        flags = (DL_DRY if dry else 0) | (DL_GRAPH if graph else 0)
        h = ctypes.c_void_p()
        check(self.lib.dl_batch_create(ctypes.byref(h), grids, arr(dx), arr(dt), arr(c), arr(m),
                                       self.count, self.dtype_code, _bc_code(bc), flags))
        self.handle = h

    def _ptrs(self, psis, Vs):
        import torch
        want = torch.complex64 if self.dtype_code == DL_C64 else torch.complex128
        if len(psis) != self.count:
            raise ValueError("one state per instance")
        P = (ctypes.c_void_p * self.count)()
        for k, t in enumerate(psis):
            if t.device.type != "cuda" or t.dtype != want or not t.is_contiguous() \
                    or tuple(t.shape) != self.tshapes[k]:
                raise ValueError(f"psi[{k}] must be a contiguous {want} CUDA tensor of shape "
                                 f"{self.tshapes[k]}")
            P[k] = t.data_ptr()
        Vp = None
        if Vs is not None:
            Vp = (ctypes.c_void_p * self.count)()
            for k, v in enumerate(Vs):
                if v is None:
                    Vp[k] = None
                    continue
                if v.device.type != "cuda" or v.dtype != torch.float64 or not v.is_contiguous() \
                        or tuple(v.shape) != self.tshapes[k][:-1]:
                    raise ValueError(f"V[{k}] must be a contiguous float64 CUDA tensor")
                Vp[k] = v.data_ptr()
        return P, Vp

    def step(self, psis, Vs, nsteps):
        P, Vp = self._ptrs(psis, Vs)
        ns = (ctypes.c_int64 * self.count)(*[int(_at(nsteps, k)) for k in range(self.count)])
        check(self.lib.dl_batch_step(self.handle, P, Vp, ns, _stream_handle()))

    def autotune(self, psis, Vs, trials=4) -> dict:
        """Tune the tile shapes on a copy of the states; returns the choice
        (depth, line_threads, seg_len of the largest 2-D size class)."""
        P, Vp = self._ptrs(psis, Vs)
        out = (ctypes.c_int * 3)()
        check(self.lib.dl_batch_autotune(self.handle, P, Vp, int(trials), out,
                                         _stream_handle()))
        return {"depth": out[0], "line_threads": out[1], "seg_len": out[2]}

    def set(self, seg_len=64, depth=None):
        """Segment length of every 2-D size class and steps per pass (None:
        the current depth)."""
        check(self.lib.dl_batch_set(self.handle, int(seg_len),
                                    int(self.depth() if depth is None else depth)))

    def info(self) -> dict:
        buf = (ctypes.c_int64 * 17)()
        check(self.lib.dl_plan_info(self.handle, buf, 17))
        return {"depth": int(buf[10]), "lines": int(buf[14]), "line_bins": int(buf[15]),
                "line_threads": int(buf[16])}

    def depth(self) -> int:
        """Steps fused per pass of the batch."""
        return self.info()["depth"]

    def close(self):
        if getattr(self, "handle", None):
            self.lib.dl_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _at(v, k):
    return v[k] if isinstance(v, (list, tuple)) or hasattr(v, "__len__") else v
