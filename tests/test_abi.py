"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/libdirac.h, and a dry plan validates its arguments
(status codes of the header) without touching HIP."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1107_4650_amd import libdirac as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libdirac.h")
C = 137.036


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1107_4650_amd import build
        build.build()
    return L.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dl_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (dl_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None
    # and nothing is exported that the header does not declare
    assert exported == set(declared_functions()), exported ^ set(declared_functions())
    assert lib.dl_version() == 1


def dry(shape, dx=0.01, dt=None, c=C, m=1.0, dtype="c64", bc="zero", axes=None, scheme="lie"):
    return L.Plan(shape, dx, dx / c if dt is None else dt, c, m, dtype=dtype, bc=bc, axes=axes,
                  dry=True, scheme=scheme)


def code_of(fn):
    with pytest.raises(L.DiracError) as ei:
        fn()
    return ei.value.code


def test_library_links_the_trace_ranges(lib):
    """The entry points open named roctx ranges (rocprofv3 --marker-trace), so
    the library depends on the roctx library, found at run time."""
    import shutil
    import subprocess
    if not shutil.which("readelf"):
        pytest.skip("readelf not available")
    dyn = subprocess.run(["readelf", "-d", L.LIB_PATH], capture_output=True, text=True).stdout
    assert "librocprofiler-sdk-roctx" in dyn


def test_dry_plan_accepts_valid_grids(lib):
    for shape, axes in (((64,), (0,)), ((64,), (2,)), ((32, 16), (0, 1)), ((32, 16), (0, 2)),
                        ((32, 16), (1, 2)), ((8, 8, 8), (0, 1, 2))):
        for dtype in ("c64", "c128"):
            for bc in ("zero", "periodic"):
                p = dry(shape, dtype=dtype, bc=bc, axes=axes)
                p.close()


def test_dry_plan_rejections(lib):
    assert code_of(lambda: dry((64,), dt=0.0101 / C)) == L.DL_ERR_CFL
    assert code_of(lambda: dry((64,), dt=2 * 0.01 / C)) == L.DL_ERR_CFL      # two-cell shifts: Strang only
    assert code_of(lambda: dry((64,), dt=0.01 / C * (1 + 1e-9))) == L.DL_ERR_CFL
    assert code_of(lambda: dry((1,))) == L.DL_ERR_ARG
    assert code_of(lambda: dry((8, 8, 8, 8))) == L.DL_ERR_ARG
    assert code_of(lambda: dry((16, 16), axes=(1, 0))) == L.DL_ERR_ARG
    assert code_of(lambda: dry((16, 16), axes=(0, 0))) == L.DL_ERR_ARG
    assert code_of(lambda: dry((16, 16), axes=(0, 3))) == L.DL_ERR_ARG
    assert code_of(lambda: dry((8, 8, 8), axes=(0, 1, 1))) == L.DL_ERR_ARG
    assert code_of(lambda: dry((64,), m=-1.0)) == L.DL_ERR_ARG
    assert code_of(lambda: dry((64,), m=float("nan"))) == L.DL_ERR_ARG
    assert code_of(lambda: dry((64,), dx=-0.01)) == L.DL_ERR_ARG
    assert code_of(lambda: dry((64,), c=0.0, dt=1.0)) == L.DL_ERR_ARG


def test_dry_strang_plans(lib):
    """Second-order plans: c dt = 2 dx on 1-D and 2-D grids, 4 dx on 3-D grids."""
    for shape, axes in (((64,), (0,)), ((32, 16), (0, 2)), ((32, 16), (0, 1)), ((32, 16), (1, 2))):
        for dtype in ("c64", "c128"):
            p = dry(shape, dtype=dtype, axes=axes, dt=2 * 0.01 / C, scheme="strang")
            p.close()
    assert code_of(lambda: dry((64,), dt=0.01 / C, scheme="strang")) == L.DL_ERR_CFL
    assert code_of(lambda: dry((64,), dt=2 * 0.01 / C * (1 + 1e-9), scheme="strang")) == L.DL_ERR_CFL
    assert code_of(lambda: dry((8, 8, 8), dt=2 * 0.01 / C, scheme="strang")) == L.DL_ERR_CFL
    for dtype in ("c64", "c128"):
        p = dry((8, 8, 8), dtype=dtype, dt=4 * 0.01 / C, scheme="strang")
        assert p.info()["depth"] == 5  # steps grouped per launch sequence
        p.set_depth(1)
        assert p.info()["depth"] == 1
        p.close()
    assert code_of(lambda: dry((64,), dt=4 * 0.01 / C, scheme="strang")) == L.DL_ERR_CFL
    with pytest.raises(ValueError):
        dry((64,), scheme="rk4")


def test_dry_3d_pass_depth(lib):
    """3-D plans fuse two steps per pass (workgroup tiles write 60 columns of
    8 rows); rows of 2^28 cells or more and a depth cap of one keep single
    steps."""
    p = dry((64, 30, 16))
    info = p.info()
    assert info["depth"] == 2 and info["nstrips"] == 2
    assert info["ntiles"] == 2 * 4 * info["nseg"]  # workgroup tiles of 8 rows
    p.set_depth(1)
    assert p.info()["depth"] == 1 and p.info()["nstrips"] == 1
    p.close()
    p = dry((64, 30, 16), dtype="c128")
    info = p.info()
    assert info["depth"] == 2 and info["nstrips"] == 2
    assert info["ntiles"] == 2 * 4 * info["nseg"]  # tiles of 8 rows with FP64 state too
    p.close()
    assert dry((64, 30)).info()["reverse_depth"] == 3
    assert dry((64, 30), dtype="c128").info()["reverse_depth"] == 2
    assert dry((64, 6), bc="periodic").info()["reverse_depth"] == 3
    assert dry((64, 30, 8)).info()["reverse_depth"] == 1
    assert dry((64, 30)).info()["field_depth"] == 3
    assert dry((64, 30), dtype="c128").info()["field_depth"] == 3
    assert dry((64, 30), dt=2 * 0.01 / C, scheme="strang").info()["field_depth"] == 1
    p3 = dry((16, 8, 8), dt=4 * 0.01 / C, scheme="strang")
    assert p3.info()["field_depth"] == p3.info()["depth"] >= 2  # one D per pass, steps grouped
    p3.close()
    assert dry((64, 4), bc="periodic").info()["field_depth"] == 2
    p = dry((1 << 28, 2, 2))
    assert p.info()["depth"] == 1
    p.close()
    p = dry(((1 << 28) - 1, 2, 2))
    assert p.info()["depth"] == 2
    p.close()


def test_dry_second_order_depths(lib):
    """Second-order 1-D / 2-D passes fuse up to three steps (both state types),
    fewer on periodic boxes of few rows; 3-D second-order plans group a call's
    steps."""
    for dtype in ("c64", "c128"):
        assert dry((64, 30), dt=2 * 0.01 / C, scheme="strang", dtype=dtype).info()["depth"] == 3
        assert dry((300,), dt=2 * 0.01 / C, scheme="strang", dtype=dtype).info()["depth"] == 3
    # a periodic box needs 2 stages x 2 rows per fused step
    assert dry((64, 8), dt=2 * 0.01 / C, scheme="strang", bc="periodic").info()["depth"] == 2
    p = dry((64, 30), dt=2 * 0.01 / C, scheme="strang")
    p.set_depth(2)
    assert p.info()["depth"] == 2
    p.close()


def test_dry_deep_1d_passes(lib):
    """1-D lowest-order plans run passes of 24 steps first; second-order
    plans, plans on more axes and a depth cap have none."""
    assert dry((777,)).info()["deep_1d_depth"] == 24
    assert dry((777,), dtype="c128", bc="periodic").info()["deep_1d_depth"] == 24
    assert dry((777,), dt=2 * 0.01 / C, scheme="strang").info()["deep_1d_depth"] == 0
    assert dry((64, 30)).info()["deep_1d_depth"] == 0
    assert dry((65536,)).info()["deep_1d_depth"] == 24
    assert dry((65537,)).info()["deep_1d_depth"] == 0  # long lines: passes of up to 5
    p = dry((777,))
    p.set_depth(3)
    assert p.info()["deep_1d_depth"] == 0
    p.close()


def test_dry_resident_choice(lib):
    """1-D lines of up to 4096 cells run on the one-workgroup kernel only when
    the plan fuses at most two steps per pass."""
    p = dry((4096,), dtype="c128")
    assert p.info()["resident"] == 0 and p.info()["depth"] == 5
    p.set_depth(2)
    assert p.info()["resident"] == 1
    p.set_tiling(allow_resident=False)
    assert p.info()["resident"] == 0
    p.close()
    p = dry((4097,))
    p.set_depth(1)
    assert p.info()["resident"] == 0
    p.close()


def test_dry_batch_depth(lib):
    """Batches fuse 5 steps per pass; a periodic batch drops the depth until
    every 2-D instance has at least twice as many rows."""
    with L.Batch([(64,), (32, 16)], 0.01, 0.01 / C, C, 1.0, dtype="c64", dry=True) as b:
        assert b.depth() == 5
    with L.Batch([(64,), (32, 16)], 0.01, 0.01 / C, C, 1.0, dtype="c128", dry=True) as b:
        assert b.depth() == 5
    with L.Batch([(64,), (32, 7)], 0.01, 0.01 / C, C, 1.0, dtype="c64", bc="periodic",
                 dry=True) as b:
        assert b.depth() == 3


def test_raw_abi_argument_errors(lib):
    g = L.make_grid((64,), dx=0.01)
    h = ctypes.c_void_p()
    assert lib.dl_plan_create(None, ctypes.byref(g), 0.01, 0.01 / C, C, 1.0, 0, 0, L.DL_DRY) \
        == L.DL_ERR_ARG
    assert lib.dl_plan_create(ctypes.byref(h), None, 0.01, 0.01 / C, C, 1.0, 0, 0, L.DL_DRY) \
        == L.DL_ERR_ARG
    assert lib.dl_plan_create(ctypes.byref(h), ctypes.byref(g), 0.01, 0.01 / C, C, 1.0, 7, 0,
                              L.DL_DRY) == L.DL_ERR_DTYPE
    assert h.value is None
    assert lib.dl_plan_create(ctypes.byref(h), ctypes.byref(g), 0.01, 0.01 / C, C, 1.0, 0, 5,
                              L.DL_DRY) == L.DL_ERR_ARG
    assert lib.dl_plan_create(ctypes.byref(h), ctypes.byref(g), 0.01, 0.01 / C, C, 1.0, 0, 0,
                              L.DL_DRY) == L.DL_OK
    # a dry plan refuses device work before touching HIP
    assert lib.dl_step(h, ctypes.c_void_p(256), None, 1, None) == L.DL_ERR_STATE
    out = (ctypes.c_double * 5)()
    assert lib.dl_observables(h, ctypes.c_void_p(256), 0.0, out, None) == L.DL_ERR_STATE
    assert b"dry plan" in lib.dl_last_error()
    assert lib.dl_plan_destroy(h) == L.DL_OK
    assert lib.dl_plan_destroy(None) == L.DL_OK
    assert lib.dl_step(None, ctypes.c_void_p(256), None, 1, None) == L.DL_ERR_ARG


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        L.load()


def test_dry_batch_validation(lib):
    shapes = [(128,), (64, 32)]
    b = L.Batch(shapes, 0.01, 0.01 / C, C, 1.0, dry=True)
    b.close()
    with pytest.raises(L.DiracError) as ei:
        L.Batch([(128,), (8, 8, 8)], 0.01, 0.01 / C, C, 1.0, dry=True)
    assert ei.value.code == L.DL_ERR_ARG
    with pytest.raises(L.DiracError) as ei:
        L.Batch([(128,), (64, 32)], [0.01, 0.01], [0.01 / C, 0.02 / C], C, 1.0, dry=True)
    assert ei.value.code == L.DL_ERR_CFL


def test_dry_norm_check_arguments(lib):
    """dl_plan_set_norm_check records its band on any plan and rejects bad values."""
    p = dry((64,))
    p.set_norm_check(1.0, 1e-6)
    p.set_norm_check(1.0, 0.0)  # off
    for ref, tol in ((0.0, 1e-6), (-1.0, 1e-6), (1.0, -1e-6), (float("nan"), 1e-6),
                     (1.0, float("inf"))):
        assert code_of(lambda: p.set_norm_check(ref, tol)) == L.DL_ERR_ARG
    p.close()
    assert lib.dl_plan_set_norm_check(None, 1.0, 0.0) == L.DL_ERR_ARG
