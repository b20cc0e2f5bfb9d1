"""Throughput benchmark of the FDTD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1|bare:N]
                    [--schemes systolic,plain,plain_fused] [--no-cpu-baseline]

A "step" is one full Yee time step (E half-step, sources, H half-step) over
the whole grid of the workload.  The default workload is the 1024x1024x512
PEC box with 2000 random dielectric boxes and three dipoles, FP32.  Inputs
are resident in HBM before the timed region; the timed region is K steps
bracketed by stream synchronisation.  Prints ONE JSON line for the headline
scheme (systolic when available, else plain), with the two plain schemes'
figures alongside (one launch per half-step, and the fused one launch per
step), a roofline object for the dominant kernel (per-launch
device time from HIP events recorded on the library's stream inside the
timed region) and the oracle timed on the host cores over a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
# FP32 vector peak without FMA and without packed math: 256 CUs x 64 lanes x 2.4 GHz
VALU_FP32_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12
FLOPS_PER_CELL = 36            # 6 components x 6 flops (Section 2)
PLAIN_E_BYTES, PLAIN_H_BYTES = 48, 36   # algorithmic bytes per cell, per half-step kernel
PLAIN_BYTES_PER_UPDATE = PLAIN_E_BYTES + PLAIN_H_BYTES
# fused plain step: E, H and cE in, E and H out
PLAIN_FUSED_BYTES_PER_UPDATE = 60


def systolic_alg_bytes_per_update(tile, band, conductive=False, fp16=False, materials=False):
    """Algorithmic HBM bytes per cell update of the systolic scheme: what the
    method itself must move (Section 4's accounting).  Every step a tile of
    V = Wx*Wy*Wz updated cells takes in its three leading faces (A = WyWz +
    WxWz + WxWy cells: E and H, and the structural coefficients) and puts out
    its three trailing faces (E and H); once per band of K steps the whole
    state goes out (E, H) and comes back in (E, H and the coefficients):

        B = (in + out) * A / V + (out + in) / K,
        in = 6 es + coefficient bytes, out = 6 es,

    es being the stored field element (4 B, or 2 B with FP16 storage) and the
    coefficients cE (3 es) plus, with conductivity, ca (12 B); with material
    indices the coefficients of a cell are its 4-byte index.  FP32 at the
    15x15x15 tile: 60 * 0.2 + 60 / K = 12 + 60 / K, with material indices
    52 * 0.2 + 52 / K = 10.4 + 52 / K."""
    wx, wy, wz = tile
    es = 2 if fp16 else 4
    coef = 4 if materials else 3 * es + (12 if conductive else 0)
    cin, cout = 6 * es + coef, 6 * es
    a, v = wy * wz + wx * wz + wx * wy, wx * wy * wz
    return (cin + cout) * a / v + (cout + cin) / band


def systolic_bytes_per_update(tile, band, conductive=False, fp16=False, materials=False):
    """HBM bytes per cell update of this design's exchange (reported beside
    the algorithmic count; it moves more than the method needs, since the
    z face's coefficients are written to a ring as well as read, and with
    FP16 storage the x and y faces' coefficients too).  Every step a tile of V = Wx*Wy*Wz updated cells takes
    in its three leading faces and puts out its three trailing faces:

    - x face (WyWz cells) and y face (WxWz): E and H (24 B per cell) through
      the face rings both ways, the coefficients (12 B; 24 B with the
      conductive decay) read from their arrays; with FP16 storage the
      coefficients travel through the rings too (in and out);
    - z face (WxWy): E, H and the coefficients through the ring, in and out.

    Once per band the whole state goes out and comes back in: E and H out
    and in, the coefficients in (60 B per cell in FP32, 72 B when conductive,
    30 B with FP16 storage).  With material indices the x and y faces and
    the band start read the 4-byte index instead of the coefficients (the z
    face still carries the 12 B of values, except with the 19-wide tile,
    whose registers and z face hold the index)."""
    wx, wy, wz = tile
    axy, v = wx * wy, wx * wy * wz
    c = 24 if conductive else 12            # coefficient bytes per cell (FP32)
    if materials:
        # (the faces travel in FP32 whatever the storage; the band's state is
        # E and H in the stored format and the index)
        cz = 4 if wx == 19 else c
        per_step = (wy * wz + wx * wz) * (24 + 4 + 24) + axy * (24 + cz) * 2
        return per_step / v + (2 * (12 if fp16 else 24) + 4) / band
    if fp16:
        per_step = (wy * wz + wx * wz + axy) * (24 + c) * 2
        band_bytes = 2 * 12 + 6
    else:
        per_step = (wy * wz + wx * wz) * (24 + c + 24) + axy * (24 + c) * 2
        band_bytes = 2 * 24 + c
    return per_step / v + band_bytes / band


def counter_traffic(kernel: str, source: str, launch: dict):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (profiles/hbm_traffic.json), or None when the summary was taken on another
    version of the kernel's source or another launch configuration."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        tr = json.load(open(path))
        have = hashlib.sha256(open(os.path.join(ROOT, source), "rb").read()).hexdigest()[:16]
        cells = launch["cells"]
        key = {k: v for k, v in launch.items() if k != "cells"}
        if tr["_sources"].get(source) != have or tr[kernel]["launch"] != key:
            return None
        k = tr[kernel]
        return (k["fetch_bytes_per_update"] + k["write_bytes_per_update"]) * cells * launch["steps"]
    except (OSError, KeyError, ValueError):
        return None


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_workload(name: str):
    from paper_2502_20610_amd import workloads as wl
    if name == "c3":
        return wl.c3_large_dielectric()
    if name == "c2":
        return wl.c2_periodic_dielectric()
    if name == "c1":
        return wl.c1_cavity_pulse()
    if name.startswith("bare:"):
        return wl.bare_bones(int(name.split(":")[1]))
    raise SystemExit("unknown workload %r" % name)


def run_scheme(w, scheme: str, steps: int, warmup: int, options=None, sigma=None, storage="fp32",
               autotune=False, profile=True):
    """scheme: "systolic", "plain", "plain_fused", or "systolic_arrays" (the
    systolic scheme streaming the per-cell coefficient arrays instead of the
    material indices)."""
    import torch
    from paper_2502_20610_amd import fdtd
    stream = torch.cuda.current_stream()
    options = dict(options or {})
    if scheme == "systolic_arrays":
        scheme = "systolic"
        options[fdtd.OPT_MATERIAL_IDS] = 0
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme, stream=stream.cuda_stream,
                          storage=storage)
    try:
        for k, v in options.items():
            sim.set_option(k, v)
        dev = torch.device("cuda:0")
        if sigma is None:
            sim.set_materials(torch.from_numpy(w.eps).to(dev))
        else:
            sim.set_materials(torch.from_numpy(w.eps).to(dev), sigma=sigma)
        if w.fields is not None:
            sim.set_fields([torch.from_numpy(f).to(dev) for f in w.fields])
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"], s.get("first_step", 0))
        torch.cuda.synchronize()
        log("%s: warmup %d steps" % (scheme, warmup))
        if warmup:
            sim.step(warmup)
        if autotune and scheme == "systolic":
            tile, band = sim.autotune(steps)
            log("%s: autotune chose tile width %d, band %d" % (scheme, tile, band))
        # build what a call of `steps` steps needs (the systolic plan and face
        # rings, the fused step's second field set) outside the timed region
        sim.prepare(steps)
        sim.synchronize()
        # per-kernel HIP-event timing (the plain schemes then launch every
        # kernel directly instead of replaying their step graphs)
        if profile:
            sim.set_option(fdtd.OPT_PROFILE, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.synchronize()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        stats = {k: (sim.kernel_stats(k) if profile else (0, 0.0))
                 for k in (fdtd.KERNEL_PLAIN_E, fdtd.KERNEL_PLAIN_H, fdtd.KERNEL_SOURCES,
                           fdtd.KERNEL_SYSTOLIC, fdtd.KERNEL_PLAIN_FUSED)}
        if scheme == "systolic":
            stats["info"] = {"materials": sim.info(fdtd.INFO_MATERIALS) if options.get(
                                 fdtd.OPT_MATERIAL_IDS, 1) else 0,
                             "grid": sim.info(fdtd.INFO_SYSTOLIC_GRID),
                             "band_steps": sim.info(fdtd.INFO_SYSTOLIC_BAND),
                             "tickets": sim.info(fdtd.INFO_SYSTOLIC_TICKETS),
                             "ring_slots": sim.info(fdtd.INFO_RING_SLOTS),
                             "tile": [sim.info(fdtd.INFO_TILE_X), sim.info(fdtd.INFO_TILE_Y),
                                      sim.info(fdtd.INFO_TILE_Z)]}
        log("%s: %d steps in %.3f s" % (scheme, steps, t))
        return t, stats
    finally:
        sim.close()


def cpu_baseline(w, budget_s: float = 25.0):
    """The FP32 oracle, as it stands, on a bounded centre crop of the workload."""
    import oracle
    nx, ny, nz = w.shape
    cx, cy, cz = min(nx, 256), min(ny, 256), min(nz, 192)
    ox, oy, oz = (nx - cx) // 2, (ny - cy) // 2, (nz - cz) // 2
    eps = np.ascontiguousarray(w.eps[ox:ox + cx, oy:oy + cy, oz:oz + cz])
    shape = (cx, cy, cz)
    fields = tuple(np.zeros(shape, np.float32) for _ in range(6))
    fields[2][cx // 2, cy // 2, cz // 2] = 1.0
    cE = [oracle.round_f32(c) for c in oracle.coeff_E([eps] * 3, (0, 0, 0), w.dt, w.dx)]
    cH = np.float32(w.dt / w.dx)
    f = tuple(np.array(a) for a in fields)
    oracle.step(cE, cH, f, 1, dtype=np.float32)          # thread start-up
    t0 = time.perf_counter()
    oracle.step(cE, cH, f, 4, step0=1, dtype=np.float32)
    per = (time.perf_counter() - t0) / 4
    n = int(max(2, min(20000, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    oracle.step(cE, cH, f, n, step0=5, dtype=np.float32)
    t = time.perf_counter() - t0
    cells = cx * cy * cz
    threads = oracle.num_threads()
    # the same oracle on one thread, over a few steps
    oracle.set_threads(1)
    try:
        n1 = int(max(2, min(200, 4.0 / max(per * threads, 1e-6))))
        t1 = time.perf_counter()
        oracle.step(cE, cH, f, n1, step0=5 + n, dtype=np.float32)
        t1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(threads)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": cells * n / t, "unit": "cell updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "FP32 oracle, %dx%dx%d centre crop of the workload's permittivity, PEC, "
                      "%d steps (%.1f s)" % (cx, cy, cz, n, t),
            "cpu_model": model,
            "single_thread": {"value": cells * n1 / t1, "unit": "cell updates/s",
                              "sample": "the same crop, %d steps on one thread (%.1f s)" % (n1, t1)}}


def copy_bandwidth(gib: int = 2, reps: int = 5):
    """Achievable HBM bandwidth of a plain device copy (read + write), for the
    roofline beside the 8 TB/s peak: best of a few copies of `gib` GiB."""
    import torch
    n = gib * (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = 0.0
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = max(best, 2.0 * n * 4 / (a.elapsed_time(b) / 1e3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    return best


def sweep(args):
    """Fig. 1 analog: cell updates/s of the schemes against grid size, on the
    bare-bones workload (random boxes, fields U(-1, 1), PEC walls, no sources).
    Steps per point: the smallest multiple of the band above 100 that runs
    about 0.3 s at the expected rate, so small grids are timed long enough."""
    from paper_2502_20610_amd import fdtd
    from paper_2502_20610_amd import workloads as wl
    for n in [int(x) for x in args.sweep.split(",") if x]:
        w = wl.bare_bones(n)
        row = {"sweep": "bare_bones", "n": n, "cells": w.cells, "state_bytes_fp32": 24 * w.cells}
        for scheme in args.schemes.split(","):
            steps = max(128, int(0.3 * 5e10 / w.cells) // 32 * 32)
            steps = min(steps, 20000)
            opts = {}
            if scheme == "systolic" and args.band:
                opts[fdtd.OPT_BAND_STEPS] = args.band
            try:
                # wall clock only: no per-kernel events (the plain schemes replay graphs)
                t, _ = run_scheme(w, scheme, steps, 32, opts, profile=False)
            except fdtd.FdtdError as e:
                row[scheme] = None
                log("n=%d %s unavailable: %s" % (n, scheme, e))
                continue
            row[scheme] = {"cups": w.cells * steps / t, "steps": steps, "s": t}
        if row.get("systolic") and row.get("plain"):
            row["systolic_over_plain"] = row["systolic"]["cups"] / row["plain"]["cups"]
        if row.get("systolic") and row.get("plain_fused"):
            row["systolic_over_plain_fused"] = row["systolic"]["cups"] / row["plain_fused"]["cups"]
        print(json.dumps(row), flush=True)


def batch_bench(nsims: int, steps: int, dims=(64, 192)):
    """The batched sweep: nsims uneven PEC grids advanced by `steps` steps.
    Three ways, each after a warm-up band, with inputs resident: one
    fdtd_step_batch launch for all grids; one systolic launch per grid (queued
    back to back on one stream); the plain scheme per grid.  Value = aggregate
    cell updates/s of the batched launch."""
    import torch
    from paper_2502_20610_amd import fdtd
    from paper_2502_20610_amd import workloads as wl
    ws = wl.c4_batch(nsims, steps, dims=dims)
    cells = sum(w.cells for w in ws)
    # one stream for every context of every mode, so that per-grid launches
    # really run back to back (a null handle would give each context a
    # stream of its own, and their launches would overlap)
    stream = torch.cuda.Stream()
    dev = torch.device("cuda:0")

    def make(scheme):
        sims = []
        for w in ws:
            sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme=scheme, stream=stream.cuda_stream)
            sim.set_materials(torch.from_numpy(w.eps).to(dev))
            for s in w.sources:
                sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
            sims.append(sim)
        return sims

    res = {}
    for mode in ("batched", "per_grid", "plain"):
        sims = make("plain" if mode == "plain" else "systolic")
        try:
            def run(n):
                if mode == "batched":
                    fdtd.step_batch(sims, n)
                else:
                    for sim in sims:
                        sim.step(n)
            # warm-up: the same call once (it also builds and uploads the plans,
            # which the timed call then reuses)
            run(steps if mode != "plain" else 32)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(steps)
            torch.cuda.synchronize()
            res[mode] = time.perf_counter() - t0
            log("batch %s: %d grids x %d steps in %.3f s" % (mode, nsims, steps, res[mode]))
        finally:
            for sim in sims:
                sim.close()
    out = {"metric": "aggregate cell updates/s, %d uneven grids in one launch" % nsims,
           "value": cells * steps / res["batched"], "unit": "cell updates/s",
           "higher_is_better": True, "n_gpus": 1, "steps": steps, "cells": cells,
           "per_grid_launches_cups": cells * steps / res["per_grid"],
           "plain_cups": cells * steps / res["plain"],
           "batched_over_per_grid": res["per_grid"] / res["batched"],
           "batched_over_plain": res["plain"] / res["batched"],
           "config": {"workload": "c4_batch", "grids": nsims, "dims": list(dims),
                      "shapes": [list(w.shape) for w in ws]}}
    print(json.dumps(out), flush=True)


def host_io_bench(args):
    """A whole systolic run of the 1024x1024x512 workload from host (pageable
    numpy) arrays: set_materials, set_fields, add_source, the workload's 500
    steps, read_fields of all six components.  Reports the PCIe-inclusive rate
    and the share of each phase; the headline `value` never includes these
    transfers."""
    import torch
    from paper_2502_20610_amd import fdtd
    w = make_workload(args.workload)
    rng = np.random.default_rng(11)
    fields = [rng.uniform(-1e-3, 1e-3, w.shape).astype(np.float32) for _ in range(6)]
    nsteps = w.nsteps
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="systolic")
    try:
        torch.cuda.synchronize()
        t = [time.perf_counter()]
        sim.set_materials(w.eps)
        sim.set_fields(fields)
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"], s.get("first_step", 0))
        sim.synchronize()
        t.append(time.perf_counter())
        sim.step(nsteps)
        sim.synchronize()
        t.append(time.perf_counter())
        out = sim.read_fields()
        t.append(time.perf_counter())
    finally:
        sim.close()
    del out
    total = t[3] - t[0]
    up = 9 * w.cells * 4
    down = 6 * w.cells * 4
    res = {"metric": "cell updates/s of a whole run from host arrays (PCIe-inclusive), %dx%dx%d FP32"
                     % w.shape,
           "value": w.cells * nsteps / total, "unit": "cell updates/s", "higher_is_better": True,
           "n_gpus": 1, "steps": nsteps, "upload_s": t[1] - t[0], "step_s": t[2] - t[1],
           "download_s": t[3] - t[2], "upload_GBps": up / (t[1] - t[0]) / 1e9,
           "download_GBps": down / (t[3] - t[2]) / 1e9,
           "device_only_cups": w.cells * nsteps / (t[2] - t[1])}
    print(json.dumps(res), flush=True)


def adjoint_bench(checkpoint_every: int = 0):
    """One gradient of the 256x256x128 inverse-design objective: the forward
    run (N steps with the monitor transform, recording the last segment's
    design-box history and checkpointing the earlier ones), the recompute of
    the earlier segments and the reverse sweep, timed together.  With the
    automatic segment length (0) the whole history fits in HBM, so there is
    one segment and nothing is recomputed.  Reported as the gradient time and
    as cell updates/s over the full-grid passes actually run (N forward
    steps, the recomputed steps and N reverse steps)."""
    import torch
    from paper_2502_20610_amd import fdtd
    from paper_2502_20610_amd import workloads as wl
    w, a = wl.c5_adjoint()
    a["checkpoint_every"] = int(checkpoint_every)
    sim = fdtd.Simulation(w.shape, w.dt, w.dx, w.bc, scheme="plain")
    try:
        dev = torch.device("cuda:0")
        sim.set_materials(torch.from_numpy(w.eps).to(dev))
        for s in w.sources:
            sim.add_source(s["comp"], s["i"], s["j"], s["k"], s["waveform"])
        sim.synchronize()
        t0 = time.perf_counter()
        # all three components share the cell's permittivity
        J, gs = sim.adjoint(**a, isotropic=True)
        t = time.perf_counter() - t0
        recomputed = sim.adjoint_recomputed_steps
    finally:
        sim.close()
    passes = 2 * a["nsteps"] + recomputed
    out = {"metric": "adjoint gradient time, %dx%dx%d FP32, %d steps" % (w.shape + (a["nsteps"],)),
           "value": t, "unit": "s", "higher_is_better": False, "n_gpus": 1,
           "grid_passes": passes, "recomputed_steps": recomputed,
           "pass_cups": passes * w.cells / t, "objective": J,
           "grad_isotropic_absmax": float(np.abs(gs).max()),
           "grad_isotropic_l2": float(np.linalg.norm(gs)),
           "config": {"workload": w.name, "design_box": [a["des_lo"], a["des_hi"]],
                      "monitor_box": [a["mon_lo"], a["mon_hi"]], "omega": a["omega"],
                      "checkpoint_every": a["checkpoint_every"]}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=128)
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--schemes", default="systolic,systolic_arrays,plain,plain_fused")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--band", type=int, default=0, help="systolic band length (0 = default)")
    ap.add_argument("--tile-x", type=int, default=0, help="systolic tile width along x (0 = default, 11, 15, 19)")
    ap.add_argument("--autotune", action="store_true",
                    help="systolic: time the tile widths and band lengths first (fdtd_autotune) and "
                         "run the fastest")
    ap.add_argument("--workgroups", type=int, default=0, help="systolic grid size (0 = auto)")
    ap.add_argument("--sweep", default="",
                    help="comma-separated n: instead of the headline line, one JSON line per "
                         "bare-bones n^3 grid with both schemes (the Fig. 1 size sweep)")
    ap.add_argument("--host-io", action="store_true",
                    help="instead of the headline line, time a whole run from host arrays: "
                         "materials and fields uploaded, the workload's steps, fields read back "
                         "(the PCIe-inclusive rate)")
    ap.add_argument("--adjoint", action="store_true",
                    help="instead of the headline line, time the gradient of the 256x256x128 "
                         "inverse-design setup (forward, recompute of checkpointed segments, "
                         "reverse sweep)")
    ap.add_argument("--adjoint-checkpoint", type=int, default=0,
                    help="segment length of the --adjoint run (0 = automatic)")
    ap.add_argument("--batch", type=int, default=0,
                    help="instead of the headline line, advance this many uneven grids (the "
                         "batched sweep, 64 in its full form) in one launch, against one launch "
                         "per grid and the plain scheme")
    ap.add_argument("--batch-dims", default="64,192",
                    help="lo,hi: per-axis sizes of the batched grids (multiples of 16)")
    ap.add_argument("--storage", default="fp32", choices=("fp32", "fp16"),
                    help="field storage: fp32, or fp16 (binary16 arrays, FP32 arithmetic)")
    ap.add_argument("--sigma", type=float, default=0.0,
                    help="conductive variant: a graded absorbing shell (16 cells) with this peak "
                         "conductivity around the workload (0 = lossless)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run one plain device copy of this many MiB (read + write), the "
                         "reference dispatch for scaling HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2502_20610_amd import fdtd
    torch.cuda.set_device(0)
    if args.calibrate_copy_mb:
        n = args.calibrate_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)   # reads and writes exactly n*4 bytes each
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calibrate_copy_mb, args.calibrate_copy_mb))
        del src, dst
    if args.sweep:
        sweep(args)
        return
    if args.adjoint:
        adjoint_bench(args.adjoint_checkpoint)
        return
    if args.host_io:
        host_io_bench(args)
        return
    if args.batch:
        batch_bench(args.batch, args.steps if args.steps != 128 else 2000,
                    tuple(int(x) for x in args.batch_dims.split(",")))
        return
    log("building workload %s" % args.workload)
    w = make_workload(args.workload)
    cells = w.cells
    log("workload %s: %d cells, %d sources" % (w.name, cells, len(w.sources)))
    sigma = None
    if args.sigma > 0:
        from paper_2502_20610_amd import workloads as wl
        sigma = torch.from_numpy(wl.graded_shell(w.shape, 16, args.sigma)).to("cuda:0")
        log("conductive: graded shell of 16 cells, peak sigma %g" % args.sigma)

    results = {}
    for scheme in args.schemes.split(","):
        try:
            opts = {}
            if scheme in ("systolic", "systolic_arrays"):
                if args.band:
                    opts[fdtd.OPT_BAND_STEPS] = args.band
                if args.workgroups:
                    opts[fdtd.OPT_WORKGROUPS] = args.workgroups
                if args.tile_x:
                    opts[fdtd.OPT_TILE_X] = args.tile_x
            t, stats = run_scheme(w, scheme, args.steps, args.warmup, opts, sigma, args.storage,
                                  autotune=args.autotune and scheme == "systolic")
        except fdtd.FdtdError as e:
            if e.code == fdtd.FDTD_EUNSUPPORTED:
                log("%s unavailable: %s" % (scheme, e))
                continue
            raise
        results[scheme] = (t, stats)
    if not results:
        raise SystemExit("no scheme ran")
    head = "systolic" if "systolic" in results else next(iter(results))
    t, stats = results[head]
    cups = cells * args.steps / t

    if head == "systolic":
        n, ms = stats[fdtd.KERNEL_SYSTOLIC]
        avg_s = ms / 1e3 / max(n, 1)
        steps_per_launch = args.steps / max(n, 1)
        band = stats["info"]["band_steps"]
        mats = stats["info"]["materials"] > 0
        b_alg = systolic_alg_bytes_per_update(stats["info"]["tile"], band, sigma is not None,
                                              args.storage == "fp16", mats)
        b_design = systolic_bytes_per_update(stats["info"]["tile"], band, sigma is not None,
                                             args.storage == "fp16", mats)
        if band >= steps_per_launch and band < 64 and not args.band:
            log("systolic: the band (%d steps) is capped by the call length (--steps %d)"
                % (band, args.steps))
        updates = cells * steps_per_launch
        achieved = b_alg * updates / avg_s / 1e9
        flops = FLOPS_PER_CELL * updates / avg_s / 1e12
        launch = {"workload": w.name + ("_conductive" if sigma is not None else "")
                  + ("_fp16" if args.storage == "fp16" else ""),
                  "steps": int(round(steps_per_launch)), "band": band, "materials": int(mats),
                  "tile_x": stats["info"]["tile"][0]}
        traffic = counter_traffic("systolic_kernel", "paper_2502_20610_amd/csrc/systolic.hip",
                                  dict(launch, cells=cells))
        # arithmetic intensity 36 / b_alg flop/B is below the machine balance
        # (39.3 T op/s / 8 TB/s), so the roofline bound is HBM
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "kernel": "systolic_kernel", "launches": n, "avg_launch_ms": avg_s * 1e3,
                "alg_bytes_per_update": b_alg,
                "design_bytes_per_update": b_design,
                "band_steps": band,
                "band_capped_by_call": bool(band >= steps_per_launch and band < 64),
                "traffic_bytes_per_update": None if traffic is None else traffic / updates,
                "traffic_GBps": None if traffic is None else traffic / avg_s / 1e9,
                "alu_achieved_TFLOPs": flops, "alu_peak_TFLOPs": VALU_FP32_PEAK_TFLOPS,
                "alu_frac": flops / VALU_FP32_PEAK_TFLOPS}
    else:
        n, ms = stats[fdtd.KERNEL_PLAIN_E]
        avg_s = ms / 1e3 / max(n, 1)
        e_bytes = PLAIN_E_BYTES + (12 if sigma is not None else 0)
        if args.storage == "fp16":
            e_bytes //= 2
        achieved = e_bytes * cells / avg_s / 1e9
        traffic = counter_traffic("plain_E_kernel", "paper_2502_20610_amd/csrc/plain.hip",
                                  {"workload": w.name + ("_conductive" if sigma is not None else "")
                                   + ("_fp16" if args.storage == "fp16" else ""),
                                   "steps": 1, "cells": cells})
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": "plain_E_kernel",
                "launches": n, "avg_launch_ms": avg_s * 1e3}

    copy_gbps = copy_bandwidth()
    roof["copy_GBps"] = copy_gbps
    roof["frac_of_copy"] = roof["achieved"] / copy_gbps
    out = {
        "metric": "cell updates/s, systolic vs plain Yee FDTD, %dx%dx%d FP32" % w.shape
                  + (", conductive" if sigma is not None else "")
                  + (", FP16 storage" if args.storage == "fp16" else ""),
        "value": cups, "unit": "cell updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w.name, "shape": list(w.shape), "bc": list(w.bc),
                   "sources": len(w.sources), "scheme": head},
        "roofline": roof,
    }
    for scheme, (ts, st) in results.items():
        c = cells * args.steps / ts
        entry = {"cups": c, "ms_per_step": ts / args.steps * 1e3}
        if scheme in ("systolic", "systolic_arrays"):
            entry.update(st["info"])
            mats = st["info"]["materials"] > 0
            b = systolic_alg_bytes_per_update(st["info"]["tile"], st["info"]["band_steps"],
                                              sigma is not None, args.storage == "fp16", mats)
            entry["alg_bytes_per_update"] = b
            entry["design_bytes_per_update"] = systolic_bytes_per_update(
                st["info"]["tile"], st["info"]["band_steps"], sigma is not None, args.storage == "fp16",
                mats)
            entry["alg_roofline_frac"] = c * b / (HBM_PEAK_GBS * 1e9)
            entry["effective_bw_frac_84B"] = c * PLAIN_BYTES_PER_UPDATE / (HBM_PEAK_GBS * 1e9)
        if scheme == "plain":
            ne, mse = st[fdtd.KERNEL_PLAIN_E]
            nh, msh = st[fdtd.KERNEL_PLAIN_H]
            entry["E_avg_ms"] = mse / max(ne, 1)
            entry["H_avg_ms"] = msh / max(nh, 1)
            pb = PLAIN_BYTES_PER_UPDATE + (12 if sigma is not None else 0)
            if args.storage == "fp16":
                pb //= 2
            entry["alg_bytes_per_update"] = pb
            entry["alg_roofline_frac"] = c * pb / (HBM_PEAK_GBS * 1e9)
        if scheme == "plain_fused":
            nf, msf = st[fdtd.KERNEL_PLAIN_FUSED]
            entry["avg_ms"] = msf / max(nf, 1)
            pb = PLAIN_FUSED_BYTES_PER_UPDATE + (12 if sigma is not None else 0)
            entry["alg_bytes_per_update"] = pb
            entry["alg_roofline_frac"] = c * pb / (HBM_PEAK_GBS * 1e9)
        out[scheme] = entry
    if "plain" in results and "systolic" in results:
        out["systolic_over_plain"] = out["systolic"]["cups"] / out["plain"]["cups"]
    if "plain_fused" in results and "systolic" in results:
        out["systolic_over_plain_fused"] = out["systolic"]["cups"] / out["plain_fused"]["cups"]
    if "plain_fused" in results and "systolic_arrays" in results:
        out["systolic_arrays_over_plain_fused"] = (out["systolic_arrays"]["cups"]
                                                   / out["plain_fused"]["cups"])
    if sigma is not None:
        out["config"]["conductive"] = {"shell_cells": 16, "sigma_max": args.sigma}
    if args.storage == "fp16":
        out["config"]["storage"] = "fp16"   # arithmetic stays FP32
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
