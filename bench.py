#!/usr/bin/env python3
"""Throughput of the stencil library on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Headline (`value`): the full 2D stencil set on an 8192 x 8192 FP64 grid with
c ~ U(-1, 1): the 4th-order 5-point second derivative in x and in y, the
9-point cross derivative d4/dx2dy2 of Fig. 1 and the point-function stencil
lap_h(c^3 - c), each periodic and non-periodic (output pre-zeroed): eight
stencil applications per step, inputs resident in HBM.  Unit: grid points
updated per second (8 x 8192^2 per step).

The JSON line also carries the roofline of the dominant kernel (its average
launch time taken with HIP events on the stream it runs on, against the
algorithmic 16 bytes per point), the oracle timed on the host cores on a
bounded sample, and further sections under "extra": the FP32 and BF16 stencil sets,
batched ragged 1D stencils and cyclic tridiagonal solves (65536 lines), the
ADI Cahn-Hilliard step on 1024^2 and 4096^2 FP64 grids (steps/s), the
64-grid FP32/BF16 ensemble against the FP64 path, the WENO advection
variant, and a copy ceiling (the library's identity stencil).
Only the cpu_baseline leg uses the oracle.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
# HBM traffic of the 8192^2 FP64 stencil kernels from rocprofv3 counters
# (FETCH_SIZE, WRITE_SIZE), valid while the kernel sources and the tile
# layout are the ones it was taken with.
TRAFFIC_FILE = os.path.join(HERE, "profiles", "stencil2d_8192_f64_traffic.json")
TRAFFIC_SOURCES = ["paper_1902_09931_amd/csrc/stencil2d.hip", "paper_1902_09931_amd/csrc/mxs_internal.h"]
# tile layouts (rows, order, threads, streaming stores) used by the counter runs
# Counter-run layouts per stencil kind (alternatives after "|"): the
# autotuner's choices for the 8192^2 FP64 set; the 3x3 kernels have been
# tuned to 128 or 256 threads, with or without lane-shift x exchange.
_L33 = "6,1,256,1,8|6,1,128,1,8|6,1,256,1,8,1|6,1,128,1,8,1"
PROFILE_LAYOUTS = f"x=4,1,256,1;y=4,1,256,1,8;xy={_L33};fun={_L33}"
METRIC = "stencil Gpoints/s + % HBM peak; CH ADI steps/s (FP64 vs FP32/batched)"
# The paper's own serial-versus-GPU figures (Sec. 5.4), for context only: a
# different machine and a different program (its whole ADI Cahn-Hilliard code).
PAPER_SPEEDUP = {
    "gpu_vs_serial_cpu": "O(10) for all reasonable grid resolutions, up to 40x for large N",
    "workload": "whole 2D ADI Cahn-Hilliard program (stencils and periodic pentadiagonal solves), "
                "N x N periodic grid to T = 10, FP64",
    "gpu": "NVIDIA Titan X Pascal",
    "cpu": "Intel i7-6850K (6 cores, 3.6 GHz), serial code",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stencil_set(wl, dx):
    d2 = wl.scaled(wl.D2_4TH, 1.0 / dx ** 2)
    return [("x_d2_4th", "X", (2, 2, 0, 0), d2, None),
            ("y_d2_4th", "Y", (0, 0, 2, 2), d2, None),
            ("xy_cross_fig1", "XY", (1, 1, 1, 1), wl.scaled(wl.CROSS_XXYY, 1.0 / dx ** 4), None),
            ("lap_cubic_fun", "XY", (1, 1, 1, 1), wl.scaled(wl.LAPLACE_3X3, 1.0 / dx ** 2),
             wl.CUBIC_MINUS_LINEAR)]


def time_loop(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / 1e3, wall


def bench_stencil_set(torch, b, wl, n, dt, steps, warmup):
    """The eight stencil applications of one step, each autotuned first.
    Inputs and outputs rotate over enough buffer pairs (>= 2 GiB) that
    consecutive launches never find their data in the 256 MB MALL.
    Returns (s per step, wall s per step, per-kernel s, count, layouts)."""
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
    code = {"f64": b.MXS_F64, "f32": b.MXS_F32, "bf16": b.MXS_BF16}[dt]
    dirs = {"X": b.MXS_X, "Y": b.MXS_Y, "XY": b.MXS_XY}
    esz = {"f64": 8, "f32": 4, "bf16": 2}[dt]
    npairs = max(2, (2 << 30) // (2 * esz * n * n))
    u0 = torch.from_numpy(wl.uniform_grid(n, n, seed=1)).to(tdt).cuda()
    ins = [u0] + [u0.clone() for _ in range(npairs - 1)]
    outs = [torch.zeros_like(u0) for _ in range(npairs)]
    dx = 1.0 / n
    plans = []      # (name, [plan per pair])
    layouts = {}
    for name, d, ext, w, coe in stencil_set(wl, dx):
        for periodic in (True, False):
            L, R, T, B = ext
            ps = [b.mxs_create_2d(n, n, n, dirs[d], b.MXS_P if periodic else b.MXS_NP, code,
                                  L, R, T, B, w, coe, ins[k], outs[k]) for k in range(npairs)]
            for p in ps:
                b.mxs_autotune(p)
            key = f"{name}_{'p' if periodic else 'np'}"
            layouts[key] = b.mxs_plan_info(ps[0])
            plans.append((key, ps))
    counter = [0]
    # marker for kernel traces: the launches after this fill are the timed ones
    torch.ones(1, device="cuda").fill_(3.0)

    def step():
        for _, ps in plans:
            b.mxs_compute(ps[counter[0] % npairs])
            counter[0] += 1

    sec, wall = time_loop(torch, step, steps, warmup)
    per_kernel = {}
    reps = max(steps, 10)
    for name, ps in plans:
        k = [0]

        def one():
            b.mxs_compute(ps[k[0] % npairs])
            k[0] += 1

        ks, _ = time_loop(torch, one, reps, 2)
        per_kernel[name] = ks / reps
    for _, ps in plans:
        for p in ps:
            b.mxs_destroy(p)
    del ins, outs, u0
    torch.cuda.empty_cache()
    return sec / steps, wall / steps, per_kernel, len(plans), layouts


def source_digest():
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_stencils(torch, b, wl, n, layouts):
    """Workload for counter runs: the eight stencils of the set in every
    listed tile layout, then a marker fill, two launches of each plan in
    order, and two copies of 512 MiB (the counters' calibration)."""
    lay = {k: v.split("|") for k, v in (kv.split("=") for kv in layouts.split(";"))}
    kind = {"x_d2_4th": "x", "y_d2_4th": "y", "xy_cross_fig1": "xy", "lap_cubic_fun": "fun"}
    u = torch.from_numpy(wl.uniform_grid(n, n, seed=1)).cuda()
    out = torch.zeros_like(u)
    dirs = {"X": b.MXS_X, "Y": b.MXS_Y, "XY": b.MXS_XY}
    plans = []
    for name, d, ext, w, coe in stencil_set(wl, 1.0 / n):
        for periodic in (True, False):
            for tile in lay[kind[name]]:
                os.environ["MXS_STENCIL_TILE"] = tile
                p = b.mxs_create_2d(n, n, n, dirs[d], b.MXS_P if periodic else b.MXS_NP, b.MXS_F64,
                                    *ext, w, coe, u, out)
                plans.append((f"{name}_{'p' if periodic else 'np'}", p))
    os.environ.pop("MXS_STENCIL_TILE", None)
    for _, p in plans:
        b.mxs_compute(p)
    torch.cuda.synchronize()
    torch.ones(1, device="cuda").fill_(2.0)      # marker
    for _, p in plans:
        for _ in range(2):
            b.mxs_compute(p)
    a = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    for _ in range(2):
        c.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profile_order": [k for k, _ in plans],
                      "layouts": [b.mxs_plan_info(p) for _, p in plans]}), flush=True)
    for _, p in plans:
        b.mxs_destroy(p)


def traffic_summary(fetch_dir, write_dir, layouts_json):
    """Turn the two counter runs of profile_stencils into per-launch HBM bytes
    of each stencil kernel, scaled by what the counters read for the 512 MiB
    copies; writes TRAFFIC_FILE and prints a markdown table."""
    def dispatches(d):
        rows = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                k = int(r["Dispatch_Id"])
                rows.setdefault(k, [r["Kernel_Name"], 0.0])[1] += float(r["Counter_Value"])
        ks = sorted(rows)
        m = max(i for i, k in enumerate(ks) if "FillFunctor" in rows[k][0])
        return [rows[k] for k in ks[m + 1:]]
    info = json.loads([ln for ln in open(layouts_json) if ln.startswith("{")][-1])
    order, layouts = info["profile_order"], info["layouts"]
    fe, wr = dispatches(fetch_dir), dispatches(write_dir)
    ns = 2 * len(order)
    copy_bytes = float(8 << 26)
    fetch_scale = copy_bytes / (sum(v for _, v in fe[ns:ns + 2]) / 2 * 1024)
    write_scale = copy_bytes / (sum(v for _, v in wr[ns:ns + 2]) / 2 * 1024)
    kern = {}   # stencil -> one entry per profiled layout
    for i, name in enumerate(order):
        fk = (fe[2 * i][1] + fe[2 * i + 1][1]) / 2
        wk = (wr[2 * i][1] + wr[2 * i + 1][1]) / 2
        kern.setdefault(name, []).append({"layout": layouts[i], "fetch_kib": fk, "write_kib": wk,
                                          "bytes": fk * 1024 * fetch_scale + wk * 1024 * write_scale})
    out = {"digest": source_digest(), "workload": "8192x8192 FP64 stencil set",
           "fetch_scale": fetch_scale, "write_scale": write_scale,
           "algorithmic_bytes_per_launch": 2 * 8 * 8192 * 8192, "kernels": kern}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(f"copy calibration: FETCH_SIZE x {fetch_scale:.3f}, WRITE_SIZE x {write_scale:.3f}\n")
    print("| stencil | threads | x exchange | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | HBM bytes (scaled) | / algorithmic |")
    print("|---|---:|---|---:|---:|---:|---:|")
    for name, ks in kern.items():
        for k in ks:
            kv = dict(f.split("=", 1) for f in k["layout"].split() if "=" in f)
            nwx = int(kv.get("window", "1x1").split("x")[0])
            xex = "-" if nwx == 1 else "lanes" if kv.get("xshuffle") == "1" else "LDS"
            print(f"| {name} | {kv.get('threads')} | {xex} | "
                  f"{k['fetch_kib']:.0f} | {k['write_kib']:.0f} | {k['bytes']:.4g} | "
                  f"{k['bytes'] / out['algorithmic_bytes_per_launch']:.3f} |")


def layout_form(info):
    """The fields of a stencil layout that decide its HBM traffic: window,
    output rows per workgroup, threads, block rows and x exchange (the tile
    order and the store kind change only the schedule)."""
    kv = dict(f.split("=", 1) for f in info.split() if "=" in f)
    return tuple(kv.get(k) for k in ("dtype", "window", "rows", "threads", "block", "xshuffle"))


def measured_traffic(kernel, layout):
    """HBM bytes per launch of a stencil kernel from the committed counter
    summary, or None when the sources or the layout's form differ from it."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("digest") != source_digest():
        return None
    for k in t.get("kernels", {}).get(kernel, []):
        if layout_form(k.get("layout", "")) == layout_form(layout):
            return k["bytes"]
    return None


def bench_ragged_1d(torch, b, wl, dt, steps, warmup):
    tdt = {"f64": torch.float64, "f32": torch.float32}[dt]
    code = {"f64": b.MXS_F64, "f32": b.MXS_F32}[dt]
    lengths, offs = wl.ragged_lengths()
    total = int(offs[-1])
    v = torch.from_numpy(wl.ragged_values(total)).to(tdt).cuda()
    o = torch.empty_like(v)
    p = b.mxs_create_1d_batch(offs, b.MXS_P, code, 2, 2, list(wl.D1_4TH), None, v, o)
    sec, _ = time_loop(torch, lambda: b.mxs_compute(p), steps, warmup)
    b.mxs_destroy(p)
    per = sec / steps
    nbytes = 2 * total * v.element_size()
    return {"points": total, "signals": int(len(lengths)), "s_per_pass": per,
            "gpoints_per_s": total / per / 1e9, "gb_per_s": nbytes / per / 1e9,
            "frac_hbm_peak": nbytes / per / 1e9 / HBM_PEAK_GBS}


def bench_cyclic_tri(torch, b, wl, dt, steps, warmup):
    """65536 periodic lines, lengths U{64..4096}: A x = r with circ(-1, 2.5, -1)."""
    tdt = {"f64": torch.float64, "f32": torch.float32}[dt]
    code = {"f64": b.MXS_F64, "f32": b.MXS_F32}[dt]
    lengths, offs = wl.ragged_lengths()
    total = int(offs[-1])
    import numpy as np
    r = torch.from_numpy(np.random.default_rng(5).uniform(-1, 1, total)).to(tdt).cuda()
    x = torch.empty_like(r)
    p = b.mxs_create_cyclic_solve(1, [2.5, -1.0], b.MXS_LINES_RAGGED, 0, 0, 0, offs, code, r, x)
    b.mxs_autotune(p)
    layout = b.mxs_plan_info(p)
    sec, _ = time_loop(torch, lambda: b.mxs_compute(p), steps, warmup)
    b.mxs_destroy(p)
    per = sec / steps
    nbytes = 2 * total * r.element_size()
    return {"points": total, "lines": int(len(lengths)), "s_per_pass": per, "layout": layout,
            "gpoints_per_s": total / per / 1e9, "gb_per_s": nbytes / per / 1e9,
            "frac_hbm_peak": nbytes / per / 1e9 / HBM_PEAK_GBS}


def bench_weno(torch, b, n, steps, warmup):
    """The WENO advection variant (Sec. 4.3) on an n x n periodic FP64 grid:
    phi, u, v ~ U(-1, 1) (seeds 8, 9, 10), out = u phi_x + v phi_y.  The four
    arrays (2 GiB at 8192^2) are eight times the memory-side cache, so
    back-to-back launches find none of their data cached."""
    import numpy as np
    arrs = [torch.from_numpy(np.random.default_rng(sd).uniform(-1, 1, (n, n))).cuda() for sd in (8, 9, 10)]
    out = torch.empty_like(arrs[0])
    h = 1.0 / n
    p = b.mxs_create_weno_adv(n, n, n, h, h, b.MXS_F64, arrs[0], arrs[1], arrs[2], out)
    b.mxs_autotune(p)
    layout = b.mxs_plan_info(p)
    sec, _ = time_loop(torch, lambda: b.mxs_compute(p), steps, warmup)
    b.mxs_destroy(p)
    del arrs, out
    torch.cuda.empty_cache()
    per = sec / steps
    nbytes = 4 * 8 * n * n
    return {"grid": [n, n], "s_per_pass": per, "layout": layout, "gpoints_per_s": n * n / per / 1e9,
            "algorithmic_bytes_per_pass": nbytes, "gb_per_s": nbytes / per / 1e9,
            "frac_hbm_peak": nbytes / per / 1e9 / HBM_PEAK_GBS}


def ch_buffers(torch, c0, tdt):
    a = torch.from_numpy(c0).to(tdt).cuda()
    return [a, a.clone(), torch.zeros_like(a)]


def bench_ch(torch, b, wl, n, steps, warmup):
    """Periodic n x n FP64 ADI Cahn-Hilliard, dt = 0.1 dx^2, D = 1, gamma = 0.01."""
    import math
    c0 = wl.ch_initial(n, n, seed=2)
    dx = 2 * math.pi / n
    bufs = ch_buffers(torch, c0, torch.float64)
    p = b.mxs_ch_create(n, n, dx, dx, 0.1 * dx * dx, 1.0, 0.01, b.MXS_F64, *bufs)
    b.mxs_autotune(p)
    layout = b.mxs_plan_info(p)
    sec, _ = time_loop(torch, lambda: b.mxs_ch_step(p, 1, True), steps, warmup)
    m = b.mxs_ch_mass(p)[0]
    forms = {}
    # every step form the grid allows, each graph-replayed (the persistent
    # one for rows of at most 1024 elements)
    modes = (((b.MXS_CH_PERSISTENT, "persistent"),) if n <= 1024 else ()) + \
        ((b.MXS_CH_FUSED, "fused"), (b.MXS_CH_SEPARATE, "separate"))
    for mode, key in modes:
        b.mxs_ch_set_step_mode(p, mode)
        fs, _ = time_loop(torch, lambda: b.mxs_ch_step(p, 1, True), steps, warmup)
        forms[f"{key}_steps_per_s"] = steps / fs
    b.mxs_ch_mass(p)
    b.mxs_destroy(p)
    per = sec / steps
    floor = 56 * n * n
    return {"steps_timed": steps, "s_per_step": per, "steps_per_s": 1.0 / per, "layout": layout, **forms,
            "floor_bytes_per_step": floor, "gb_per_s_at_floor": floor / per / 1e9,
            "frac_hbm_peak_at_floor": floor / per / 1e9 / HBM_PEAK_GBS,
            "mass_drift": abs(m - float(c0.sum())) / float(abs(c0).sum())}


def bench_ensemble(torch, b, wl, steps, warmup):
    """64 grids of sizes 256^2..1024^2: FP32 and BF16 storage ensembles (one
    launch per kernel per step, graph-replayed) against the plain FP64 path,
    both as an FP64 ensemble and one grid at a time."""
    import math
    sizes = wl.ensemble_sizes()
    c0s = wl.ensemble_initial(sizes)
    pts = sum(n * n for n in sizes)
    dxs = [2 * math.pi / n for n in sizes]
    dts = [0.1 * d * d for d in dxs]
    out = {"instances": len(sizes), "points": pts, "steps_timed": steps}
    for name, tdt, code in (("f32", torch.float32, b.MXS_F32), ("bf16", torch.bfloat16, b.MXS_BF16),
                            ("f64", torch.float64, b.MXS_F64)):
        bufs = [ch_buffers(torch, c0, tdt) for c0 in c0s]
        p = b.mxs_ch_ensemble_create(sizes, sizes, dxs, dxs, dts, 1.0, 0.01, code,
                                     [q[0] for q in bufs], [q[1] for q in bufs], [q[2] for q in bufs])
        b.mxs_autotune(p)
        out[f"ensemble_{name}_layout"] = b.mxs_plan_info(p)
        sec, _ = time_loop(torch, lambda: b.mxs_ch_step(p, 1, True), steps, warmup)
        out[f"ensemble_{name}_steps_per_s"] = steps / sec
        # every step form, each graph-replayed: one persistent launch per
        # step, the right-hand side inside the row solves, and the separate
        # launches
        for mode, key in ((b.MXS_CH_PERSISTENT, "persistent"), (b.MXS_CH_FUSED, "fused"),
                          (b.MXS_CH_SEPARATE, "separate")):
            b.mxs_ch_set_step_mode(p, mode)
            sec, _ = time_loop(torch, lambda: b.mxs_ch_step(p, 1, True), steps, warmup)
            out[f"ensemble_{name}_{key}_steps_per_s"] = steps / sec
        b.mxs_ch_mass(p, len(sizes))       # raises if a grid barrier failed
        b.mxs_destroy(p)
        del bufs
    bufs = [ch_buffers(torch, c0, torch.float64) for c0 in c0s]
    plans = [b.mxs_ch_create(n, n, d, d, t, 1.0, 0.01, b.MXS_F64, *q)
             for n, d, t, q in zip(sizes, dxs, dts, bufs)]
    for p in plans:
        b.mxs_autotune(p)

    def seq_step():
        for p in plans:
            b.mxs_ch_step(p, 1, True)

    sec, _ = time_loop(torch, seq_step, max(steps // 5, 10), 2)
    out["f64_one_grid_at_a_time_steps_per_s"] = max(steps // 5, 10) / sec
    for p in plans:
        b.mxs_destroy(p)
    del bufs
    torch.cuda.empty_cache()
    for name in ("f32", "bf16", "f64"):
        out[f"ensemble_{name}_vs_f64_one_at_a_time"] = (out[f"ensemble_{name}_steps_per_s"] /
                                                        out["f64_one_grid_at_a_time_steps_per_s"])
    return out


def copy_ceiling(torch, b, wl, n=8192):
    """Copy ceilings, read + write bytes / time: the library's identity
    stencil (a one-tap X window of weight 1, i.e. the stencil kernel as a
    plain streaming copy, autotuned, over the same rotation of 2 GiB of
    buffers as the stencil set) and, for context, torch's copy kernel on
    1 GiB."""
    u0 = torch.from_numpy(wl.uniform_grid(n, n, seed=1)).cuda()
    npairs = max(2, (2 << 30) // (2 * 8 * n * n))
    ins = [u0] + [u0.clone() for _ in range(npairs - 1)]
    outs = [torch.empty_like(u0) for _ in range(npairs)]
    ps = [b.mxs_create_2d(n, n, n, b.MXS_X, b.MXS_P, b.MXS_F64, 0, 0, 0, 0, [1.0], None, ins[k], outs[k])
          for k in range(npairs)]
    for p in ps:
        b.mxs_autotune(p)
    k = [0]

    def one():
        b.mxs_compute(ps[k[0] % npairs])
        k[0] += 1

    sec, _ = time_loop(torch, one, 40, 5)
    layout = b.mxs_plan_info(ps[0])
    for p in ps:
        b.mxs_destroy(p)
    ident = 2 * 8 * n * n / (sec / 40) / 1e9
    del ins, outs, u0
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    sec, _ = time_loop(torch, lambda: c.copy_(a), 20, 3)
    tgbs = 2 * a.numel() * 8 / (sec / 20) / 1e9
    del a, c
    torch.cuda.empty_cache()
    return {"identity_stencil_gb_per_s": ident, "identity_stencil_layout": layout,
            "identity_stencil_frac_hbm_peak": ident / HBM_PEAK_GBS, "torch_copy_gb_per_s": tgbs}


def cpu_model():
    """The host CPU's model name (first processor in /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_ch(n, steps=2):
    """The oracle (single thread) on the FP64 ADI Cahn-Hilliard step of an
    n x n grid, in steps per second."""
    import math
    import oracle
    from paper_1902_09931_amd import workloads as wl
    c0 = wl.ch_initial(n, n, seed=2)
    dx = 2 * math.pi / n
    t0 = time.perf_counter()
    oracle.ch_run(c0, c0, steps, dx, dx, 0.1 * dx * dx, 1.0, 0.01)
    sec = time.perf_counter() - t0
    return {"value": steps / sec, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the {n}^2 FP64 ADI Cahn-Hilliard step ({sec:.1f} s, "
                      f"single-threaded C on {cpu_model()})"}


def cpu_baseline(wl, n, rows):
    """The oracle (single thread) on the same eight stencils over a
    rows x n slice of the grid."""
    import oracle
    u = wl.uniform_grid(rows, n, seed=1)
    dx = 1.0 / n
    t0 = time.perf_counter()
    for name, d, ext, w, coe in stencil_set(wl, dx):
        for periodic in (True, False):
            oracle.stencil2d(u, *ext, w, periodic, coe=coe)
    sec = time.perf_counter() - t0
    pts = 8 * rows * n
    return {"value": pts / sec / 1e9, "unit": "Gpoints/s", "cores": 1, "kind": "oracle",
            "sample": f"the eight stencils of one step on a {rows} x {n} slice "
                      f"({pts} point updates, {sec:.1f} s, single-threaded C, "
                      f"{os.cpu_count()} host cores visible, {cpu_model()})"}


def cpu_baseline_threads(wl, n, rows):
    """The same oracle calls spread over the host cores: each thread runs the
    eight stencils on its own band of rows of the slice (independent calls of
    the unchanged oracle, which releases the GIL inside its C code)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    nthreads = max(1, min(len(os.sched_getaffinity(0)), 16))
    band = (rows + nthreads - 1) // nthreads
    u = wl.uniform_grid(rows, n, seed=1)
    bands = [np_ascontig(u[k:k + band]) for k in range(0, rows, band)]
    dx = 1.0 / n

    def work(ub):
        for name, d, ext, w, coe in stencil_set(wl, dx):
            for periodic in (True, False):
                oracle.stencil2d(ub, *ext, w, periodic, coe=coe)

    with ThreadPoolExecutor(len(bands)) as pool:
        t0 = time.perf_counter()
        list(pool.map(work, bands))
        sec = time.perf_counter() - t0
    pts = 8 * rows * n
    return {"value": pts / sec / 1e9, "unit": "Gpoints/s", "cores": len(bands), "kind": "oracle",
            "sample": f"the eight stencils of one step on a {rows} x {n} slice split into "
                      f"{len(bands)} bands of rows, one thread each ({pts} point updates, "
                      f"{sec:.2f} s)"}


def np_ascontig(a):
    import numpy as np
    return np.ascontiguousarray(a)


def host_threads():
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def timed(fn):
    t0 = time.perf_counter()
    fn()
    return time.perf_counter() - t0


def threaded(jobs):
    """Run independent oracle calls (closures) on one thread each; the oracle
    releases the GIL inside its C code.  Returns the wall time."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(len(jobs)) as pool:
        t0 = time.perf_counter()
        list(pool.map(lambda f: f(), jobs))
        return time.perf_counter() - t0


def split_batch(offs, parts):
    """Split a ragged batch (offsets) into `parts` contiguous signal ranges of
    about equal point counts: list of (values slice start, stop, local offsets)."""
    import numpy as np
    total = int(offs[-1])
    cuts = [int(np.searchsorted(offs, total * k / parts)) for k in range(parts)] + [len(offs) - 1]
    out = []
    for a, z in zip(cuts[:-1], cuts[1:]):
        if z > a:
            out.append((int(offs[a]), int(offs[z]), np.ascontiguousarray(offs[a:z + 1] - offs[a])))
    return out


def cpu_baseline_sections(wl):
    """The oracle on every other workload of the bench, on the host cores:
    single-threaded (the paper's serial baseline) and with independent
    signals, lines or grids spread over the host threads.  Each figure is
    per pass or per step of the whole workload; CH steps are timed over one
    step and stated as extrapolated."""
    import math
    import numpy as np
    import oracle
    nt = host_threads()
    out = {"host_cpu": cpu_model(), "host_threads_used": nt}
    lengths, offs = wl.ragged_lengths()
    total = int(offs[-1])
    v = wl.ragged_values(total)
    parts = split_batch(offs, nt)
    d1 = list(wl.D1_4TH)
    t1 = timed(lambda: oracle.stencil1d_batch(v, offs, 2, 2, d1, True))
    tn = threaded([lambda a=a, z=z, o=o: oracle.stencil1d_batch(v[a:z], o, 2, 2, d1, True)
                   for a, z, o in parts])
    out["ragged1d_stencil"] = {"s_per_pass_1_thread": t1, "s_per_pass_all_threads": tn,
                               "gpoints_per_s_1_thread": total / t1 / 1e9,
                               "gpoints_per_s_all_threads": total / tn / 1e9,
                               "sample": f"the whole batch: {len(lengths)} signals, {total} points"}
    r = np.random.default_rng(5).uniform(-1, 1, total)
    bands = oracle.circulant_bands([2.5, -1.0])
    t1 = timed(lambda: oracle.cyclic_solve_batch(bands, offs, r))
    tn = threaded([lambda a=a, z=z, o=o: oracle.cyclic_solve_batch(bands, o, r[a:z])
                   for a, z, o in parts])
    out["cyclic_tri_batch"] = {"s_per_pass_1_thread": t1, "s_per_pass_all_threads": tn,
                               "gpoints_per_s_1_thread": total / t1 / 1e9,
                               "gpoints_per_s_all_threads": total / tn / 1e9,
                               "sample": f"the whole batch: {len(lengths)} lines, {total} points"}
    n = 4096
    c0 = wl.ch_initial(n, n, seed=2)
    dx = 2 * math.pi / n
    t1 = timed(lambda: oracle.ch_run(c0, c0, 1, dx, dx, 0.1 * dx * dx, 1.0, 0.01))
    out["ch_adi_4096_f64"] = {"s_per_step_1_thread": t1, "steps_per_s_1_thread": 1.0 / t1,
                              "sample": "one step of the 4096^2 FP64 ADI step (extrapolated)"}
    del c0
    sizes = wl.ensemble_sizes()
    c0s = wl.ensemble_initial(sizes)
    jobs = []
    for nn, c in zip(sizes, c0s):
        d = 2 * math.pi / nn
        jobs.append(lambda c=c, d=d: oracle.ch_run(c, c, 1, d, d, 0.1 * d * d, 1.0, 0.01))
    t1 = timed(lambda: [f() for f in jobs])
    # instances dealt to threads largest first, so the threads finish together
    order = sorted(range(len(sizes)), key=lambda k: -sizes[k])
    groups = [[] for _ in range(nt)]
    load = [0] * nt
    for k in order:
        g = load.index(min(load))
        groups[g].append(jobs[k])
        load[g] += sizes[k] ** 2
    tn = threaded([lambda grp=grp: [f() for f in grp] for grp in groups if grp])
    out["ch_ensemble_64_f64"] = {"s_per_step_1_thread": t1, "s_per_step_all_threads": tn,
                                 "steps_per_s_1_thread": 1.0 / t1, "steps_per_s_all_threads": 1.0 / tn,
                                 "sample": f"one FP64 step of all {len(sizes)} grids "
                                           f"({sum(s * s for s in sizes)} points; extrapolated)"}
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu-sections", action="store_true",
                    help="time the oracle on the stencil set and the 1024^2 CH step only")
    ap.add_argument("--sections-only", action="store_true",
                    help="skip the headline stencil set (for profiling the sections)")
    ap.add_argument("--sections", default="f32,bf16,ragged,tri,weno,ch,ensemble,copy",
                    help="extra sections to run (comma list)")
    ap.add_argument("--ch-steps", type=int, default=0,
                    help="override the Cahn-Hilliard step counts (0: 1000 at 1024^2, 200 at 4096^2)")
    ap.add_argument("--profile-stencils", nargs="?", const=PROFILE_LAYOUTS, default=None,
                    metavar="LAYOUTS", help="run the counter workload for the stencil set only")
    ap.add_argument("--traffic-summary", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "LAYOUTS_JSON"),
                    help="summarise the two counter runs (no GPU needed)")
    args = ap.parse_args()
    if args.traffic_summary:
        traffic_summary(*args.traffic_summary)
        return
    sections = set(args.sections.split(",")) if not args.no_extra else set()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1902_09931_amd import binding as b
    from paper_1902_09931_amd import workloads as wl

    n = args.n
    if args.profile_stencils:
        profile_stencils(torch, b, wl, n, args.profile_stencils)
        return
    log(f"device {torch.cuda.get_device_name(0)}; stencil set {n}^2 f64")
    if args.sections_only:
        sec, wall, napps, layouts = 1.0, 1.0, 8, {}
        per_kernel = {"none": 1.0}
        layouts["none"] = ""
    else:
        sec, wall, per_kernel, napps, layouts = bench_stencil_set(torch, b, wl, n, "f64", args.steps,
                                                                  args.warmup)
    pts = napps * n * n
    dominant = max(per_kernel, key=per_kernel.get)
    bytes_per_launch = 2 * 8 * n * n
    achieved = bytes_per_launch / per_kernel[dominant] / 1e9
    result = {
        "metric": METRIC,
        "value": pts / sec / 1e9,
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D stencil set on a {n}x{n} FP64 grid, c~U(-1,1) seed 1: "
                               "4th-order 5-point d2/dx2 and d2/dy2, Fig. 1 cross d4/dx2dy2, "
                               "5-point Laplacian of c^3-c; periodic and non-periodic",
                   "grid": [n, n], "stencil_applications_per_step": napps},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dominant, layouts[dominant]) if n == 8192 else None,
                     "kernel": dominant, "avg_launch_us": per_kernel[dominant] * 1e6,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    extra = {"wall_ms_per_step": wall * 1e3, "f64_layouts": layouts,
             "f64_kernels_us": {k: v * 1e6 for k, v in per_kernel.items()},
             "f64_hbm_frac_per_kernel": {k: bytes_per_launch / v / 1e9 / HBM_PEAK_GBS
                                         for k, v in per_kernel.items()}}
    # reduced-precision storage (FP32 accumulation): the same set in FP32 and BF16
    for dt, esz in (("f32", 4), ("bf16", 2)):
        if dt in sections:
            log(f"stencil set {dt}")
            sr, _, pkr, _, layr = bench_stencil_set(torch, b, wl, n, dt, args.steps, args.warmup)
            extra[f"{dt}_layouts"] = layr
            extra[f"{dt}_gpoints_per_s"] = pts / sr / 1e9
            extra[f"{dt}_kernels_us"] = {k: v * 1e6 for k, v in pkr.items()}
            extra[f"{dt}_hbm_frac_per_kernel"] = {k: 2 * esz * n * n / v / 1e9 / HBM_PEAK_GBS
                                                  for k, v in pkr.items()}
    for dt in ("f64", "f32"):
        if "ragged" in sections:
            log(f"ragged 1D stencil {dt}")
            extra[f"ragged1d_stencil_{dt}"] = bench_ragged_1d(torch, b, wl, dt, args.steps, args.warmup)
        if "tri" in sections:
            log(f"batched cyclic tridiagonal {dt}")
            extra[f"cyclic_tri_batch_{dt}"] = bench_cyclic_tri(torch, b, wl, dt, args.steps, args.warmup)
    if "weno" in sections:
        log("WENO advection f64")
        extra["weno_adv_f64"] = bench_weno(torch, b, n, args.steps, args.warmup)
    if "ch" in sections:
        for nn in (1024, 4096):
            log(f"Cahn-Hilliard ADI {nn}^2 f64")
            k = args.ch_steps or (1000 if nn == 1024 else 200)
            extra[f"ch_adi_{nn}_f64"] = bench_ch(torch, b, wl, nn, k, min(10, k))
    if "ensemble" in sections:
        log("Cahn-Hilliard ensemble")
        k = args.ch_steps or 500
        extra["ch_ensemble_64"] = bench_ensemble(torch, b, wl, k, min(10, k))
    if "copy" in sections:
        log("copy ceiling")
        extra["copy_ceiling"] = copy_ceiling(torch, b, wl, n)
    result["extra"] = extra
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(wl, n, rows=min(n, 3072))
        extra["cpu_baseline_all_cores"] = cpu_baseline_threads(wl, n, rows=min(n, 3072))
        extra["cpu_baseline_ch_1024"] = cpu_baseline_ch(1024)
        if not args.no_cpu_sections:
            cs = cpu_baseline_sections(wl)
            extra["cpu_baseline_sections"] = cs
            # GPU speed-up over the oracle, beside each GPU figure
            for dt in ("f64", "f32"):
                for key, cpu in (("ragged1d_stencil", cs["ragged1d_stencil"]),
                                 ("cyclic_tri_batch", cs["cyclic_tri_batch"])):
                    sec = extra.get(f"{key}_{dt}")
                    if sec:
                        sec["oracle_s_per_pass_1_thread"] = cpu["s_per_pass_1_thread"]
                        sec["oracle_s_per_pass_all_threads"] = cpu["s_per_pass_all_threads"]
                        sec["speedup_vs_oracle_1_thread"] = cpu["s_per_pass_1_thread"] / sec["s_per_pass"]
                        sec["speedup_vs_oracle_all_threads"] = (cpu["s_per_pass_all_threads"] /
                                                                sec["s_per_pass"])
            ch = extra.get("ch_adi_4096_f64")
            if ch:
                ch["oracle_steps_per_s_1_thread"] = cs["ch_adi_4096_f64"]["steps_per_s_1_thread"]
                ch["speedup_vs_oracle_1_thread"] = ch["steps_per_s"] / ch["oracle_steps_per_s_1_thread"]
            ens = extra.get("ch_ensemble_64")
            if ens:
                ce = cs["ch_ensemble_64_f64"]
                ens["oracle_f64_steps_per_s_1_thread"] = ce["steps_per_s_1_thread"]
                ens["oracle_f64_steps_per_s_all_threads"] = ce["steps_per_s_all_threads"]
                for name in ("f32", "bf16", "f64"):
                    ens[f"ensemble_{name}_speedup_vs_oracle_all_threads"] = (
                        ens[f"ensemble_{name}_steps_per_s"] / ce["steps_per_s_all_threads"])
        extra["paper_speedup"] = PAPER_SPEEDUP
    if args.sections_only:     # no headline was measured: report the sections alone
        result = {"sections_only": True, "extra": extra}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
