#!/usr/bin/env python3
"""Benchmark of the fused Dirac sweep on one MI355X.

Headline (`value`): spinor site-updates per second of the FP32-storage sweep
on the 2-D 2048 x 2048 tanh-step workload (complex64 state, FP64 potential
and phases), inputs resident in HBM.  A "step" is one full time step of the
hot path: x transport, y transport and the local phase step, fused in one
launch.  The same line carries the FP64 path, the FP32-vs-FP64 error after
the timed steps, the roofline of the sweep kernel, the CPU oracle baseline
and the secondary workloads (1-D resident, 3-D, observables, batched,
adjoint).

  python bench.py [--steps K] [--warmup W] [--gpus 1]
  python bench.py --only sweep --steps 20     # kernel loop only (profiling)
  python bench.py --calibrate-copy            # a plain copy of known size
  python bench.py --only klein                # the paper's 2-D Klein run alone
  python bench.py --only 3d                   # the 3-D 512^3 runs alone
  python bench.py --only observables          # the observables calls alone (2048^2 FP32)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_F32 = 72                 # read psi 32 B + write psi 32 B + read V 8 B per site-update
BYTES_F64 = 136                # read psi 64 B + write psi 64 B + read V 8 B
METRIC = "spinor site-updates/s + % HBM roofline, FP32 vs FP64 at rel-L2 <=1e-4"
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("dirac_device.h", "dirac_sweep_impl.h", "dirac_sweep2d_kernels.h",
              "dirac_sweep2d_f32_hi.hip", "dirac_launch.h"):
        with open(os.path.join(ROOT, "paper_1107_4650_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def timed_sweep(plan, psi, V, steps, warmup, fused=1):
    """Advance psi by `steps` time steps (rounded down to whole passes of
    `fused` steps) and time it.  The steps run as one dl_step call, which
    enqueues the passes back to back in the library (ping-ponging psi and the
    plan's buffer, ending in psi for an even pass count); HIP events are
    recorded on the launch stream before and after the call (the pass count
    is rounded down to an even number).  Returns
    (wall seconds, mean per-launch ms from the events, final tensor, steps
    timed)."""
    import torch
    nl, nw = max(1, steps // fused), max(0, warmup // fused)
    if nl > 1 and nl % 2:
        nl -= 1  # an even pass count ends in psi: no copy back inside the timed region
    if fused > 1 and plan.info()["depth"] != fused:
        plan.set_depth(fused)
    if nw:
        plan.step(psi, V, nw * fused)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    plan.step(psi, V, nl * fused)
    end.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = start.elapsed_time(end) / nl
    return wall, per, psi, nl * fused


def to_dev(x, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x)).to("cuda")
    return t if dtype is None else t.to(dtype)


def rel_l2(a, b):
    import torch
    a = a.to(torch.complex128)
    b = b.to(torch.complex128)
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def load_profile(kernel_name):
    """Counter figures for one kernel from the committed rocprofv3 PMC summaries
    (HBM bytes per launch, VALU busy fraction), if they were taken on the
    current kernel source; None otherwise."""
    path = os.path.join(PROFILES, "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    ent = t.get(kernel_name)
    if not ent or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent


GOLDEN_CONFIG2 = os.path.join(ROOT, "tests", "golden", "config2_2048_1e4.txt")


def golden_check(L, V):
    """The 2-D workload run for its stated 10^4 steps (untimed) against the
    oracle's final state stored in tests/golden/ (512 cells and the grid's
    observables, written by a script that calls only the oracle): relative L2
    over the cells for FP32 and FP64 state."""
    import torch
    from paper_1107_4650_amd.inputs import config_2d_tanh
    if not os.path.exists(GOLDEN_CONFIG2):
        return None
    idx, vals = [], []
    with open(GOLDEN_CONFIG2) as f:
        for line in f:
            if line.startswith("cell "):
                parts = line.split()
                idx.append(int(parts[1]))
                ri = np.array([float(v) for v in parts[2:]])
                vals.append(ri[0::2] + 1j * ri[1::2])
    ref = torch.from_numpy(np.array(vals)).to("cuda")
    tidx = torch.tensor(idx, device="cuda")
    w = config_2d_tanh(n=2048, nsteps=10000)
    out = {"steps": w.nsteps, "cells": len(idx), "reference": "tests/golden/config2_2048_1e4.txt"}
    for dt in ("c64", "c128"):
        tdt = torch.complex64 if dt == "c64" else torch.complex128
        with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype=dt, xmin=w.xmin) as p:
            psi = to_dev(w.psi0, tdt)
            p.step(psi, V, w.nsteps)
            torch.cuda.synchronize()
            got = psi.reshape(-1, 4)[tidx]
        out[("fp32" if dt == "c64" else "fp64") + "_rel_l2"] = rel_l2(got, ref)
        del psi
    return out


def bench_main(args):
    import torch
    from paper_1107_4650_amd import libdirac as L
    from paper_1107_4650_amd.inputs import config_2d_tanh

    L.load()
    w = config_2d_tanh(n=2048, nsteps=args.steps)
    sites = w.sites
    log(f"workload {w.name}: {sites} sites, {args.steps} steps, warmup {args.warmup}")
    V = to_dev(w.V)
    res = {}

    # ---- FP32 storage (headline) -------------------------------------------
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c64", xmin=w.xmin) as p32:
        d32 = p32.info()["depth"]
        psi32 = to_dev(w.psi0, torch.complex64)
        wall32, per32, out32, n32 = timed_sweep(p32, psi32, V, args.steps, args.warmup, d32)
        info = p32.info()
        obs32 = p32.observables(out32, 0.0)
    res["fp32"] = dict(wall=wall32, per_launch_ms=per32)
    log(f"fp32: {wall32 * 1e3 / n32:.4f} ms/step wall, {per32:.4f} ms per {d32}-step launch")
    if args.only == "sweep":
        return None

    # ---- FP64 path on the same steps (also the reference for the FP32 error) -
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c128", xmin=w.xmin) as p64:
        d64 = p64.info()["depth"]
        psi64 = to_dev(w.psi0)
        wall64, per64, out64, n64 = timed_sweep(p64, psi64, V, n32, args.warmup - args.warmup % d32,
                                                d64)
        obs64 = p64.observables(out64, 0.0)
    # both runs advanced the same number of steps from the same initial state
    assert n64 == n32, (n64, n32)
    err = rel_l2(out32, out64)
    log(f"fp64: {wall64 * 1e3 / n64:.4f} ms/step wall; fp32 vs fp64 rel-L2 {err:.3e}")
    del psi32, psi64, out32, out64
    torch.cuda.empty_cache()
    gold = golden_check(L, V)
    if gold:
        log(f"vs stored oracle state after {gold['steps']} steps: fp32 rel-L2 "
            f"{gold['fp32_rel_l2']:.3e}, fp64 {gold['fp64_rel_l2']:.3e}")

    # one launch advances every cell d32 steps, reading psi and V once and
    # writing psi once: 72 B per cell per launch, 72 / d32 B per site-update
    achieved = BYTES_F32 * sites / (per32 * 1e-3) / 1e9
    kname = f"sweep2d_d{d32}_f32_2048"
    prof = load_profile(kname)
    traffic = prof.get("bytes_per_launch") if prof else None
    line = {
        "metric": METRIC,
        "value": sites * n32 / wall32,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": n32,
        "warmup": args.warmup - args.warmup % d32,
        "ms_per_step": wall32 * 1e3 / n32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2-D Dirac, 2048x2048 cells, tanh step V0*tanh(x/0.1), "
                               "Gaussian packet sigma 1.5 p0=(40,0), complex64 state, FP64 V "
                               "and phases, dx=0.01, c*dt=dx, zero walls",
                   "grid": [2048, 2048], "steps_per_launch": d32,
                   "tiling": info},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "kernel": f"k_sweep2d<float, LieStep, {d32}, 0, 1, 2, 4>",
                     "bytes_per_launch_per_cell": BYTES_F32,
                     "bytes_per_site_update": BYTES_F32 / d32,
                     "per_launch_ms": per32, "site_updates_per_launch": d32 * sites,
                     # the fused pass recomputes halo cells and converts to FP64 for the
                     # phase; rocprofv3 counters (SQ_INSTS_VALU) show the SIMDs' VALU
                     # issue as the limiter of the five-step pass
                     "valu_busy": prof.get("valu_busy") if prof else None,
                     "profile": prof.get("summary") if prof else None,
                     # a sweep that reads and writes psi (and reads V) once per step
                     # cannot exceed 8 TB/s / 72 B site-updates/s; the fused pass
                     # does fewer bytes per step, so its rate is compared with that
                     "one_step_per_pass_ceiling": HBM_PEAK_GBS * 1e9 / BYTES_F32,
                     "value_over_that_ceiling": (sites * n32 / wall32)
                                                / (HBM_PEAK_GBS * 1e9 / BYTES_F32)},
        "fp64": {"value": sites * n64 / wall64, "unit": "site-updates/s",
                 "ms_per_step": wall64 * 1e3 / n64, "per_launch_ms": per64,
                 "steps_per_launch": d64,
                 "roofline_frac": BYTES_F64 * sites / (per64 * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "fp32_vs_fp64_rel_l2": err,
        "fp32_vs_fp64_steps": n32 + args.warmup - args.warmup % d32,
        "vs_oracle_after_1e4_steps": gold,
        "norm_fp32": obs32[0], "norm_fp64": obs64[0],
    }
    return line


def bench_extras(args, line):
    """Secondary workloads of the same library (not the headline)."""
    import torch
    from paper_1107_4650_amd import libdirac as L
    from paper_1107_4650_amd.inputs import config_1d_step
    ex = {}
    # 1-D N = 4096, 2000 steps, complex128 (passes of 24 steps, then 5 and 3); the
    # warm-up takes the same passes, so the plan's buffers exist before the timing
    w = config_1d_step()
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c128", xmin=w.xmin) as p:
        psi = to_dev(w.psi0)
        V = to_dev(w.V)
        p.step(psi, V, w.nsteps)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        p.step(psi, V, w.nsteps)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e)
    ex["1d_4096_c128"] = {"steps": w.nsteps, "ms": ms,
                          "site_updates_per_s": w.sites * w.nsteps / (ms * 1e-3)}
    log(f"1-D 4096 x {w.nsteps}: {ms:.3f} ms")
    # the same line as a two-component state (the packet lives in (psi_1, psi_4))
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c128", xmin=w.xmin, bispinor=True) as p:
        psi2 = to_dev(np.ascontiguousarray(w.psi0[:, [0, 3]]))
        p.step(psi2, V, w.nsteps)
        torch.cuda.synchronize()
        s.record()
        p.step(psi2, V, w.nsteps)
        e.record()
        torch.cuda.synchronize()
        ms2 = s.elapsed_time(e)
    ex["1d_4096_c128"]["bispinor_ms"] = ms2
    ex["1d_line_4M_f32"] = bench_long_line()
    # 3-D 512^3 FP32 and FP64, a prefix of the 2000-step run
    ex["3d_512"] = bench_3d(args)
    # observables pass on the 2048^2 FP32 state
    ex["observables_2048_f32"] = bench_observables()
    # adjoint: 1024^2 periodic, forward + reversible backward
    ex["adjoint_1024"] = bench_adjoint(args)
    # batch of 256 uneven instances vs the same instances one at a time
    ex["batch_256"] = bench_batch(args)
    # local step with a static vector potential on the 2048^2 FP32 workload
    ex["field_2048_f32"] = bench_field(args)
    if args.klein_steps > 0:
        ex["klein2d_24576x8192_strang"] = bench_klein2d(args)
    line["extras"] = ex


def bench_long_line(n=1 << 22, steps=400):
    """A long 1-D line (4M cells, the 1-D workload's packet and step potential
    stretched over a 41.9 a.u. box), complex64: the four-component state vs
    the two-component one, passes of 5 steps each."""
    import torch
    from paper_1107_4650_amd import libdirac as L
    from paper_1107_4650_amd.inputs import packet, potential_step, C_LIGHT, M_E
    dx = 0.01
    shape = (n,)
    psi = packet(shape, dx, delta=2.0, p0=[50.0], r0=[-10.0])
    V = to_dev(potential_step(shape, dx, 2.0 * M_E * C_LIGHT ** 2))
    out = {"cells": n, "steps": steps}
    for name, nc in (("four_component", 4), ("two_component", 2)):
        src = psi if nc == 4 else np.ascontiguousarray(psi[:, [0, 3]])
        with L.Plan(shape, dx, dx / C_LIGHT, C_LIGHT, M_E, dtype="c64", bispinor=(nc == 2)) as p:
            t = to_dev(src, torch.complex64)
            p.step(t, V, 20)
            torch.cuda.synchronize()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            p.step(t, V, steps)
            e.record()
            torch.cuda.synchronize()
            ms = s.elapsed_time(e)
            depth = p.info()["depth"]
        out[name] = {"ms_per_step": ms / steps, "site_updates_per_s": n * steps / (ms * 1e-3),
                     "steps_per_pass": depth, "bytes_per_cell_per_pass": 8 * 2 * nc + 8}
        del t
    torch.cuda.empty_cache()
    log(f"1-D 4M line: {out['four_component']['ms_per_step'] * 1e3:.1f} vs "
        f"{out['two_component']['ms_per_step'] * 1e3:.1f} us/step (4 vs 2 components)")
    return out


def bench_field(args, steps=400):
    """The 2-D 2048^2 tanh-step workload with a static vector potential in the
    local step (field integral At_y = 0.05 sin(2 pi x / 5) per step, a
    synthetic smooth field), complex64 state: dl_step_field at the plan's depth."""
    import torch
    from paper_1107_4650_amd import libdirac as L
    from paper_1107_4650_amd.inputs import config_2d_tanh, coord_mesh
    w = config_2d_tanh(n=2048, nsteps=steps)
    X = coord_mesh(w.shape, w.dx)[0]
    A = np.zeros((3,) + w.shape[::-1])
    A[1] = np.broadcast_to(0.05 * np.sin(2 * np.pi * X / 5.0), w.shape[::-1])
    V, At = to_dev(w.V), to_dev(A)
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c64", xmin=w.xmin) as p:
        psi = to_dev(w.psi0, torch.complex64)
        p.step_field(psi, V, At, 20)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        p.step_field(psi, V, At, steps)
        e.record()
        torch.cuda.synchronize()
        ms = s.elapsed_time(e)
        norm = p.observables(psi, 0.0)[0]
        K = p.info()["field_depth"]
    del psi, V, At
    torch.cuda.empty_cache()
    # per pass of K steps: psi read + written (64 B), V (8 B), At (24 B) per cell
    return {"steps": steps, "ms_per_step": ms / steps, "steps_per_pass": K,
            "site_updates_per_s": w.sites * steps / (ms * 1e-3),
            "bytes_per_site_update": 96 / K,
            "hbm_frac": 96 * w.sites / (K * ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "norm": norm}


def bench_klein2d(args):
    """The paper's 2-D Klein run (Sec. 5.2.2): 24576 x 8192 cells in the x-z
    plane, second-order steps, 12000 steps to t = 0.214, complex64 state; the
    transmitted probability beyond x = 0 against the paper's numeric 0.2407
    and the analytic 0.2621.  Inputs are assembled on the device from their
    separable 1-D pieces (input generation only)."""
    import torch
    from paper_1107_4650_amd import libdirac as L
    from paper_1107_4650_amd.inputs import klein2d_factors, C_LIGHT, M_E
    nx, nz = 24576, 8192
    f = klein2d_factors(nx, nz)
    gx = torch.from_numpy(f["gx"]).to("cuda")
    gz = torch.from_numpy(f["gz"]).to("cuda")
    u = torch.from_numpy(f["u"]).to("cuda")
    psi = torch.empty((nz, nx, 4), dtype=torch.complex64, device="cuda")
    for k0 in range(0, nz, 512):  # row blocks keep the complex128 temporaries small
        k1 = min(nz, k0 + 512)
        psi[k0:k1] = (gz[k0:k1, None, None] * gx[None, :, None] * u).to(torch.complex64)
    V = torch.from_numpy(f["Vx"]).to("cuda")[None, :].expand(nz, nx).contiguous()
    del gx, gz
    steps = args.klein_steps
    with L.Plan((nx, nz), f["dx"], f["dt"], C_LIGHT, M_E, dtype="c64", axes=(0, 2),
                xmin=f["xmin"], scheme="strang") as p:
        obs0 = p.observables(psi, 0.0)
        torch.cuda.synchronize()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        s.record()
        p.step(psi, V, steps)
        e.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = s.elapsed_time(e)
        obs = p.observables(psi, 0.0)
        depth = p.info()["depth"]
    del psi, V
    torch.cuda.empty_cache()
    sites = nx * nz
    T = obs[4] / obs[0]
    log(f"2-D Klein 24576x8192 strang: {steps} steps in {ms / 1e3:.2f} s, T = {T:.4f}")
    return {"grid": [nx, nz], "steps": steps, "t_final": steps * f["dt"], "scheme": "strang",
            "dtype": "c64", "steps_per_pass": depth, "seconds": ms / 1e3, "wall_s": wall,
            "site_updates_per_s": sites * steps / (ms * 1e-3),
            "norm_initial": obs0[0], "norm_final": obs[0],
            "T": T, "R": 1.0 - T, "T_paper_numeric": 0.2407, "T_analytic": 0.2621,
            "paper_seconds": 22 * 3600, "paper_processors": 256}


def bench_3d(args):
    import torch
    from paper_1107_4650_amd import libdirac as L
    n, dx = 512, 0.02
    c, m = 137.036, 1.0
    steps = args.steps3d
    # separable packet and spherical barrier built on the device (input generation only)
    x = (torch.arange(n, dtype=torch.float64, device="cuda") + 0.5) * dx - n * dx / 2
    delta = 2.0
    gx = torch.exp(1j * 30.0 * x) * torch.exp(-((x + 2.5) ** 2) / (4 * delta * delta))
    gy = torch.exp(1j * 10.0 * x) * torch.exp(-(x ** 2) / (4 * delta * delta))
    gz = torch.exp(-(x ** 2) / (4 * delta * delta)).to(torch.complex128)
    p0 = np.array([30.0, 10.0, 0.0])
    E = np.sqrt(c * c * (p0 ** 2).sum() + m * m * c ** 4)
    u = torch.tensor([1.0, 0.0, c * p0[2] / (E + m * c * c), c * (p0[0] + 1j * p0[1]) / (E + m * c * c)],
                     dtype=torch.complex128, device="cuda")
    out = {}
    r2 = (x[:, None, None] ** 2 + x[None, :, None] ** 2 + x[None, None, :] ** 2)
    V = (1.5 * m * c * c) * torch.exp(-r2 / 4.0)
    del r2
    runs = (("f32", torch.complex64, BYTES_F32, None), ("f32_one_step_per_pass", torch.complex64,
                                                        BYTES_F32, 1),
            ("f64", torch.complex128, BYTES_F64, None),
            ("f32_second_order", torch.complex64, None, None),
            ("f32_vector_potential", torch.complex64, None, None),
            ("f32_adjoint", torch.complex64, None, None))
    for dt_name, tdt, bps, depth in runs:
        f = (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
        psi = (f[..., None] * u).to(tdt).contiguous()
        del f
        if dt_name.endswith("vector_potential"):
            # a smooth static field integral along y, one step per pass
            At = torch.zeros((3, n, n, n), dtype=torch.float64, device="cuda")
            At[1] = (0.05 * torch.sin(2 * np.pi * x / 5.0))[None, None, :]
            with L.Plan((n, n, n), dx, dx / c, c, m, dtype="complex64") as p:
                p.step_field(psi, V, At, 2)
                torch.cuda.synchronize()
                s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                nf = min(steps, 10)
                s_.record()
                p.step_field(psi, V, At, nf)
                e_.record()
                torch.cuda.synchronize()
                msf = s_.elapsed_time(e_) / nf
            # psi read + written (64 B), V (8 B), At (24 B) per cell and step
            out[dt_name] = {"steps": nf, "ms_per_step": msf, "steps_per_pass": 1,
                            "site_updates_per_s": n ** 3 / (msf * 1e-3),
                            "hbm_frac": 96 * n ** 3 / (msf * 1e-3) / 1e9 / HBM_PEAK_GBS}
            log(f"3-D 512^3 {dt_name}: {msf:.3f} ms/step")
            del psi, At
            torch.cuda.empty_cache()
            continue
        if dt_name.endswith("adjoint"):
            # reverse steps (dl_grad_step) from lambda = [x > 0] psi: one pass per step
            # (the dL/dV term, D^H, T_z^H, T_y^H, T_x^H)
            with L.Plan((n, n, n), dx, dx / c, c, m, dtype="complex64") as p:
                lam = torch.empty_like(psi)
                Q = torch.empty_like(V)
                p.seed_adjoint(psi, 0.0, lam, Q)
                p.grad_step(psi, lam, V, Q, 1)
                torch.cuda.synchronize()
                s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                nr = min(steps, 10)
                s_.record()
                p.grad_step(psi, lam, V, Q, nr)
                e_.record()
                torch.cuda.synchronize()
                msr = s_.elapsed_time(e_) / nr
            # psi, lambda, V and Q read, both fields and Q written: 152 B per cell
            out[dt_name] = {"reverse_steps": nr, "ms_per_reverse_step": msr,
                            "passes_per_reverse_step": 1,
                            "site_updates_per_s": n ** 3 / (msr * 1e-3),
                            "hbm_frac": 152 * n ** 3 / (msr * 1e-3) / 1e9 / HBM_PEAK_GBS}
            log(f"3-D 512^3 {dt_name}: {msr:.3f} ms per reverse step")
            del psi, lam, Q
            torch.cuda.empty_cache()
            continue
        strang = dt_name.endswith("second_order")
        if strang:
            # c dt = 4 dx: one pass per step plus a closing one per call, four times
            # the time per step
            with L.Plan((n, n, n), dx, 4 * dx / c, c, m, dtype="complex64", scheme="strang") as p:
                K = p.info()["depth"]
                wall, per, _, done = timed_sweep(p, psi, V, max(K, min(steps, 20)), K, fused=K)
            out[dt_name] = {"steps": done, "ms_per_step": wall * 1e3 / done,
                            "steps_per_call": done, "passes_per_call": done + 1,
                            "dt_over_lowest_order_dt": 4,
                            "site_updates_per_s": n ** 3 * done / wall}
            log(f"3-D 512^3 {dt_name}: {wall * 1e3 / done:.3f} ms/step (c dt = 4 dx)")
            del psi
            torch.cuda.empty_cache()
            continue
        with L.Plan((n, n, n), dx, dx / c, c, m, dtype=str(tdt).split(".")[1]) as p:
            if depth is not None:
                p.set_depth(depth)
            K = p.info()["depth"]
            wall, per, _, done = timed_sweep(p, psi, V, steps, 2 * K, fused=K)
        sites = n ** 3
        # every launch reads and writes psi once and reads V once, whatever its depth
        out[dt_name] = {"steps": done, "steps_per_launch": K, "ms_per_step": wall * 1e3 / done,
                        "per_launch_ms": per, "site_updates_per_s": sites * done / wall,
                        "roofline_frac": bps * sites / (per * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"3-D 512^3 {dt_name}: {per:.3f} ms/launch of {K} step(s)")
        del psi
        torch.cuda.empty_cache()
    # two steps and the observables: two calls, or one whose two-step pass sums
    # the observables as it stores the state
    f = (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
    psi = (f[..., None] * u).to(torch.complex64).contiguous()
    del f
    with L.Plan((n, n, n), dx, dx / c, c, m, dtype="complex64") as p:
        def per_call(fn, reps=5):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            return (time.perf_counter() - t0) * 1e3 / reps
        out["f32_step2_observables"] = {
            "two_calls_ms": per_call(lambda: (p.step(psi, V, 2), p.observables(psi, 0.0))),
            "fused_ms": per_call(lambda: p.step_observables(psi, V, 2, 0.0)),
            "observables_alone_ms": per_call(lambda: p.observables(psi, 0.0))}
    log(f"3-D 512^3 two steps + observables: {out['f32_step2_observables']}")
    del psi
    torch.cuda.empty_cache()
    if args.accuracy3d_steps > 0:
        out["f32_vs_f64"] = accuracy_3d(n, dx, c, m, gx, gy, gz, u, V, args.accuracy3d_steps)
    return out


def accuracy_3d(n, dx, c, m, gx, gy, gz, u, V, steps):
    """The 3-D workload's stated check: FP32 bulk vs the FP64 GPU run after
    `steps` steps (2000 by default, the workload's length), relative L2 over
    every cell, with each run's time."""
    import torch
    from paper_1107_4650_amd import libdirac as L
    res = {}
    for name, tdt in (("c128", torch.complex128), ("c64", torch.complex64)):
        f = (gz[:, None, None] * gy[None, :, None] * gx[None, None, :])
        psi = (f[..., None] * u).to(tdt).contiguous()
        del f
        with L.Plan((n, n, n), dx, dx / c, c, m, dtype=name) as p:
            torch.cuda.synchronize()
            s_, e_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s_.record()
            p.step(psi, V, steps)
            e_.record()
            torch.cuda.synchronize()
            res[name] = (psi, s_.elapsed_time(e_), p.observables(psi, 0.0))
    num = den = 0.0
    for k in range(0, n, 64):
        a = res["c64"][0][k:k + 64].to(torch.complex128)
        b = res["c128"][0][k:k + 64]
        num += float(torch.sum(torch.abs(a - b) ** 2))
        den += float(torch.sum(torch.abs(b) ** 2))
    err = (num / den) ** 0.5
    out = {"steps": steps, "rel_l2": err, "bar": 1e-4,
           "f32_s": res["c64"][1] / 1e3, "f64_s": res["c128"][1] / 1e3,
           "norm_f32": res["c64"][2][0], "norm_f64": res["c128"][2][0]}
    del res
    torch.cuda.empty_cache()
    log(f"3-D 512^3 FP32 vs FP64 after {steps} steps: rel-L2 {err:.3e} "
        f"({out['f32_s']:.2f} s / {out['f64_s']:.2f} s)")
    return out


def bench_observables():
    import torch
    from paper_1107_4650_amd import libdirac as L
    from paper_1107_4650_amd.inputs import config_2d_tanh
    w = config_2d_tanh(n=2048, nsteps=1)
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c64", xmin=w.xmin) as p:
        psi = to_dev(w.psi0, torch.complex64)
        V = to_dev(w.V, torch.float64)
        p.observables(psi, 0.0)
        reps = 20
        t0 = time.perf_counter()
        for _ in range(reps):
            p.observables(psi, 0.0)
        ms = (time.perf_counter() - t0) * 1e3 / reps
        # one pass of five steps, then the observables: two calls, or one
        # call whose pass sums the observables as it stores the state
        def per_call(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                fn()
            return (time.perf_counter() - t0) * 1e3 / reps
        ms_two = per_call(lambda: (p.step(psi, V, 5), p.observables(psi, 0.0)))
        ms_fused = per_call(lambda: p.step_observables(psi, V, 5, 0.0))
    return {"ms_per_call_incl_sync": ms, "bytes_per_site": 32,
            "GBps": 32 * w.sites / (ms * 1e-3) / 1e9,
            "step5_then_observables_ms": ms_two, "step5_observables_fused_ms": ms_fused}


def bench_adjoint(args):
    """Adjoint workload: 1024^2 complex64 periodic box, V from 64 Gaussian bumps,
    forward nsteps (dl_expand + dl_step + observables) and the fused reverse sweep
    (dl_seed_adjoint + dl_grad_step + dl_project)."""
    import torch
    from paper_1107_4650_amd import libdirac as L
    from paper_1107_4650_amd.inputs import config_adjoint
    w = config_adjoint(nsteps=args.adjoint_steps)
    nb = len(w.extra["theta"])
    G = to_dev(w.extra["dVdtheta"])
    theta = to_dev(w.extra["theta"])
    x_b = w.extra["x_b"]
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c64", bc="periodic", xmin=w.xmin) as p:
        psi0 = to_dev(w.psi0, torch.complex64)
        V = torch.empty(w.psi0.shape[:-1], dtype=torch.float64, device="cuda")
        psi = psi0.clone()
        lam = torch.empty_like(psi)
        Q = torch.empty_like(V)
        g = torch.empty(nb, dtype=torch.float64, device="cuda")
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        ev[0].record()
        p.expand(G, theta, V)
        p.step(psi, V, w.nsteps)
        ev[1].record()
        L_T = p.observables(psi, x_b)[4]
        ev[2].record()
        p.seed_adjoint(psi, x_b, lam, Q)
        p.grad_step(psi, lam, V, Q, w.nsteps)
        p.project(Q, G, g)
        ev[3].record()
        torch.cuda.synchronize()
        fwd_ms = ev[0].elapsed_time(ev[1])
        bwd_ms = ev[2].elapsed_time(ev[3])
        rec = rel_l2(psi, psi0)
        gn = float(torch.linalg.vector_norm(g))
        K = p.info()["reverse_depth"]
    sites = w.sites * w.nsteps
    g32 = g.cpu().numpy()
    check = adjoint_checks(w, G, theta, g32)
    log(f"adjoint: fwd {fwd_ms:.2f} ms, bwd {bwd_ms:.2f} ms, reconstruction {rec:.2e}, "
        f"FP32 vs FP64 gradient {check['fp32_vs_fp64_max_rel']:.2e}, "
        f"FD {check['fd_max_rel']:.2e}")
    return {"steps": w.nsteps, "forward_ms": fwd_ms, "backward_ms": bwd_ms,
            "checks": check,
            "forward_site_updates_per_s": sites / (fwd_ms * 1e-3),
            "backward_site_updates_per_s": sites / (bwd_ms * 1e-3),
            # a reverse pass reads psi, lambda, V, Q and writes psi, lambda, Q once
            # per cell, 152 B, whatever its steps
            "backward_steps_per_pass": K, "backward_bytes_per_cell_per_pass": 152,
            "backward_roofline_frac": 152 / K * sites / (bwd_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "loss_P_T": L_T, "grad_norm": gn, "psi0_reconstruction_rel_l2": rec}


def adjoint_checks(w, G, theta, g32, h_au=1e-3, nfd=4):
    """The adjoint workload's stated checks: the FP32 dL/dtheta against the
    FP64 GPU gradient, and the FP64 gradient against central finite
    differences of the FP64 forward run, on the `nfd` bumps of largest
    gradient.  The amplitudes are energies drawn from [-1, 1] m c^2; the
    difference step is h_au = 1e-3 atomic units of energy (1e-3 / (m c^2) in
    the units of theta here, where V = m c^2 sum theta_j g_j)."""
    h = h_au / (w.m * w.c * w.c)
    import torch
    from paper_1107_4650_amd import libdirac as L
    x_b = w.extra["x_b"]
    with L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c128", bc="periodic", xmin=w.xmin) as p:
        V = torch.empty(w.psi0.shape[:-1], dtype=torch.float64, device="cuda")

        def forward(th):
            psi = to_dev(w.psi0)
            p.expand(G, th, V)
            p.step(psi, V, w.nsteps)
            return psi, p.observables(psi, x_b)[4]

        psi, _ = forward(theta)
        lam = torch.empty_like(psi)
        Q = torch.empty_like(V)
        p.seed_adjoint(psi, x_b, lam, Q)
        p.grad_step(psi, lam, V, Q, w.nsteps)
        g = torch.empty(G.shape[0], dtype=torch.float64, device="cuda")
        p.project(Q, G, g)
        g64 = g.cpu().numpy()
        scale = float(np.max(np.abs(g64)))
        fd = {}
        for j in np.argsort(-np.abs(g64))[:nfd]:
            e = torch.zeros_like(theta)
            e[int(j)] = h
            lp = forward(theta + e)[1]
            lm = forward(theta - e)[1]
            fd[int(j)] = ((lp - lm) / (2 * h), float(g64[j]))
        del psi, lam, Q, V
    return {"fp32_vs_fp64_max_rel": float(np.max(np.abs(g32 - g64))) / scale, "bar_fp32": 1e-3,
            "grad_norm_fp64": float(np.linalg.norm(g64)),
            "fd_h_atomic_units": h_au, "theta_unit": "m c^2",
            "fd": {str(j): {"central_difference": a, "adjoint_fp64": b} for j, (a, b) in fd.items()},
            "fd_max_rel": max(abs(a - b) for a, b in fd.values()) / scale, "bar_fd": 1e-5}


def bench_batch(args):
    """256 uneven 1-D/2-D instances in one dl_batch_step call (the 1-D ones run
    whole in the lines kernel, the 2-D ones pass by pass; the call replayed as
    one graph) vs the same instances advanced one at a time with their own
    plans.  The tuner picks the tile shapes first; a warm-up call of the same
    shape captures the graph outside the timed call."""
    import torch
    from paper_1107_4650_amd import libdirac as L
    from paper_1107_4650_amd.inputs import config_batch
    steps = args.batch_steps
    ws = config_batch(count=256, nsteps=steps, seed=0)
    sites = sum(w.sites for w in ws)
    psis = [to_dev(w.psi0, torch.complex64) for w in ws]
    Vs = [to_dev(w.V) for w in ws]
    out = {"instances": len(ws), "sites": sites, "steps": steps,
           "n_1d": sum(1 for w in ws if w.ndim == 1), "n_2d": sum(1 for w in ws if w.ndim == 2)}
    with L.Batch([w.shape for w in ws], [w.dx for w in ws], [w.dt for w in ws],
                 [w.c for w in ws], [w.m for w in ws], dtype="c64", graph=True) as b:
        t0 = time.perf_counter()
        out["autotuned"] = b.autotune(psis, Vs, trials=3)
        out["autotune_s"] = time.perf_counter() - t0
        out["layout"] = b.info()
        K = b.depth()
        work = [t.clone() for t in psis]
        b.step(work, Vs, [steps] * len(ws))  # captures the call's graph
        del work
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(psis, Vs, [steps] * len(ws))
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
    out["batched_s"] = tb
    out["batched_site_updates_per_s"] = sites * steps / tb
    # one pass of K steps reads and writes each state once and reads V once
    out["batched_steps_per_pass"] = K
    out["batched_roofline_frac"] = BYTES_F32 / K * sites * steps / tb / 1e9 / HBM_PEAK_GBS
    # the same instances one plan at a time, from the same initial states
    psis1 = [to_dev(w.psi0, torch.complex64) for w in ws]
    plans = [L.Plan(w.shape, w.dx, w.dt, w.c, w.m, dtype="c64") for w in ws]
    for p, t, v in zip(plans, [t.clone() for t in psis1], Vs):
        p.step(t, v, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, t, v in zip(plans, psis1, Vs):
        p.step(t, v, steps)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    for p in plans:
        p.close()
    # batched and one-at-a-time runs end with the same bits
    out["same_bits_as_single_plans"] = bool(all(torch.equal(a, b_) for a, b_ in zip(psis, psis1)))
    out["one_at_a_time_s"] = ts
    out["one_at_a_time_site_updates_per_s"] = sites * steps / ts
    out["speedup"] = ts / tb
    log(f"batch: {tb:.3f} s batched vs {ts:.3f} s one at a time "
        f"(depth {K}, {out['layout']['lines']} lines in {out['layout']['line_bins']} workgroups)")
    return out


def cpu_baseline(min_seconds=10.0, max_seconds=30.0):
    """The FP64 oracle, as it stands, on the host's cores: bounded sample of the
    same 2048^2 workload (whole steps until ~min_seconds of CPU time)."""
    from oracle import oracle as O
    from paper_1107_4650_amd.inputs import config_2d_tanh
    w = config_2d_tanh(n=2048, nsteps=1)
    threads = O.max_threads()
    psi = w.psi0
    done, t_used, chunk = 0, 0.0, 4
    while t_used < min_seconds and t_used < max_seconds:
        t0 = time.perf_counter()
        psi = O.step(psi, w.V, dt=w.dt, c=w.c, m=w.m, nsteps=chunk, axes=w.axes, threads=threads)
        t_used += time.perf_counter() - t0
        done += chunk
    # the same oracle on one thread, a shorter sample
    psi1, done1, t1 = w.psi0, 0, 0.0
    while t1 < min_seconds / 2:
        t0 = time.perf_counter()
        psi1 = O.step(psi1, w.V, dt=w.dt, c=w.c, m=w.m, nsteps=1, axes=w.axes, threads=1)
        t1 += time.perf_counter() - t0
        done1 += 1
    return {"value": w.sites * done / t_used, "unit": "site-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{done} FP64 steps of the 2048x2048 tanh-step workload "
                      f"({w.sites * done:.3e} site-updates, {t_used:.1f} s, {threads} OpenMP threads)",
            "single_thread": {"value": w.sites * done1 / t1, "unit": "site-updates/s",
                              "sample": f"{done1} steps on one thread, {t1:.1f} s"}}


def calibrate_copy(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling the PMC byte counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--steps3d", type=int, default=50)
    ap.add_argument("--adjoint-steps", type=int, default=4000)
    ap.add_argument("--batch-steps", type=int, default=5000)
    ap.add_argument("--accuracy3d-steps", type=int, default=2000,
                    help="steps of the 3-D FP32-vs-FP64 check (0 skips it)")
    ap.add_argument("--klein-steps", type=int, default=12000,
                    help="steps of the paper's 2-D Klein run (0 skips it)")
    ap.add_argument("--only", choices=["all", "sweep", "main", "klein", "3d", "observables"],
                    default="all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the sweep runs on a single MI355X; "
              f"--gpus {args.gpus} is not supported (the multi-GPU slab decomposition is a "
              f"design, not code).",
              file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.only == "klein":
        print(json.dumps(bench_klein2d(args)), flush=True)
        return
    if args.only == "3d":
        print(json.dumps(bench_3d(args)), flush=True)
        return
    if args.only == "observables":
        print(json.dumps(bench_observables()), flush=True)
        return
    line = bench_main(args)
    if line is None:
        return
    if args.only == "all":
        bench_extras(args, line)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
