#!/usr/bin/env python
"""Benchmark of the two-grid sweeping preconditioner on one MI355X.

Workload (default): the 2-D seeded smooth layered medium, 1023 x 1023
interior nodes + 16 PML cells per side, h = 10 m, 8 points per wavelength at
c_min = 1.5 km/s (f = 18.75 Hz), two-grid sweeping preconditioner (5-point
fine level, optimized 9-point FE coarse level, X-sweep over J = 32 slabs,
w_dd = 4, nu = 3, omega_jac = 0.8) inside FGMRES, point source at the centre,
solved to a 1e-6 relative residual.

One step = one complete batched solve: 64 point sources at seeded random
interior positions on that medium, every one solved to 1e-6 by its own FGMRES
process (FGMRES + every preconditioner application), with the medium,
factors and right-hand sides resident in HBM.  The metric is
dof * iterations / solve time summed over the batch, with dof the interior
nodes (absorbing layers excluded).  The reported value is the FP32-batched
form (complex64 smoother, slab factors and sweeps; complex128 Arnoldi
basis, orthogonalisation, residual, coarse-grid correction and solution; all
sources in one batch); the plain FP64 form (complex128 throughout, one source
at a time) is timed beside it at the same final residual, as are the
single-source mixed form and the batched form with the Arnoldi basis stored
in complex64 as well (the opt-in krylov_fp32 option).  Each form runs with
its own chunk length of the slab substitutions (an evaluation-order
setting): 34 tangential blocks per chunk for the batched solves (fewer,
longer chunks keep one workgroup per CU at 64 sources), the automatic
choice (about the square root of the tangential nodes) for the
single-source ones.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# HBM traffic of the roofline kernels, measured with rocprofv3 counters
# (a FETCH_SIZE and a WRITE_SIZE run, scaled by the same counters on a copy of
# known size); a record is valid only for the kernel sources it was taken on
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_layered1023_64src.md")
KERNEL_SOURCES = {
    "stage": ["batch.hip", "sweep_dev.h", "internal.h", "common.h"],
    "project": ["blas.hip", "internal.h", "common.h"],
    "update": ["blas.hip", "internal.h", "common.h"],
    "matvec": ["stencil.hip", "internal.h", "common.h"],
    "nd_stage": ["nd3d.hip", "slab3d.hip", "d3.h", "internal.h", "common.h"],
}
# the 3-D nested-dissection stage's record (per stage of the 3-D workload)
ND_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k3_nd_stage_factor_smooth127cubed.md")
# kernel names in the counter files: the batched stage (two launches per
# stage, for the tile in use) and the projection and update passes over the
# complex128 Arnoldi basis
KERNEL_PATTERNS = {
    "stage": r"k_bstage_(fwd|bwd)<float, (\d+), (\d+)",
    "project": r"k_bmultidot2<double>",
    "update": r"k_bdcgs_update<double>",
    "matvec": r"k_stencil_multi<5, double, float, double, double>",
}
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector peak
CLASSES = ("stage", "smooth", "coarse", "transfer", "krylov", "project", "update")
COPY_BYTES = 256 << 20

# tangential blocks per chunk of the slab substitutions in the batched solves
AUTOTUNE = -1  # --chunk value that asks the autotuner for the chunk length and tile

METRIC = "dof·iter/s and solve time to 1e-6 rel. residual: FP32-batched vs plain FP64"
UNIT = "dof·iter/s"
HBM_PEAK_GBS = 8000.0


def sources_digest(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1412_0464_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel, tile, nsrc, chunk=0, path=None):
    """Measured HBM bytes per launch (per stage for "stage") from the counter
    record, or None when there is none for this kernel, tile, chunk length
    and batch size or the kernel's sources changed since it was taken (tile
    and chunk length matter for the stage only)."""
    import re
    try:
        with open(path or TRAFFIC_RECORD) as fh:
            txt = fh.read()
    except OSError:
        return None
    for m in re.finditer(r"traffic-record: kernel=(\w+) bytes_per_launch=(\S+) tile=(\d+) chunk=(\d+) "
                         r"sources=(\d+) digest=(\w+)", txt):
        if m.group(1) != kernel or int(m.group(5)) != nsrc or m.group(6) != sources_digest(kernel):
            continue
        if kernel == "stage" and (int(m.group(3)) != tile or int(m.group(4)) != chunk):
            continue
        return float(m.group(2))
    return None


def copy_calibration():
    """A plain streaming kernel of known size (torch's elementwise negation
    of COPY_BYTES of float32: reads and writes COPY_BYTES each), run three
    times so that counter runs can scale FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.ones(COPY_BYTES // 4, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(f"[bench] copy calibration: 3 x neg over {COPY_BYTES} bytes", file=sys.stderr, flush=True)


def reduce_counters(fetch_csv, write_csv, tile, nsrc, chunk=0):
    """Per-kernel averages of the rocprofv3 counter files of a FETCH_SIZE run
    and a WRITE_SIZE run (KiB per dispatch), the copy scale factors, and the
    traffic records of the batched stage (per stage, for ``tile``), of the
    projection and update passes and of the batched FGMRES matvec (per
    launch)."""
    import csv
    import re
    from collections import defaultdict

    def load_csv(path):
        tot, disp = defaultdict(float), defaultdict(set)
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                name = row["Kernel_Name"]
                tot[name] += float(row["Counter_Value"])
                disp[name].add(row["Dispatch_Id"])
        return {k: (len(disp[k]), tot[k]) for k in tot}

    per = {"stage": {}, "project": {}, "update": {}, "matvec": {}}
    for label, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        d = load_csv(path)
        print(f"{label} (KiB per dispatch)")
        for k, (n, v) in sorted(d.items(), key=lambda kv: -kv[1][1])[:14]:
            print(f"  {n:7d} x {v / n:14.1f}  {k[:110]}")
        copy = [(n, v) for k, (n, v) in d.items() if "neg_kernel" in k]
        if not copy:
            raise SystemExit(f"{path}: no copy calibration kernel")
        copy_kib = copy[0][1] / copy[0][0]
        scale = (COPY_BYTES / 1024) / copy_kib
        print(f"  copy: {copy_kib:.1f} KiB per dispatch for {COPY_BYTES // 1024} KiB -> scale {scale:.4f}")
        stage_kib, stages = 0.0, 0
        pass_kib = {"project": 0.0, "update": 0.0, "matvec": 0.0}
        passes = {"project": 0, "update": 0, "matvec": 0}
        for k, (n, v) in d.items():
            m = re.search(KERNEL_PATTERNS["stage"], k)
            if m and int(m.group(3)) == tile:
                stage_kib += v
                if m.group(1) == "fwd":
                    stages += n
            for kern in pass_kib:
                if re.search(KERNEL_PATTERNS[kern], k):
                    pass_kib[kern] += v
                    passes[kern] += n
        print(f"  stage (tile {tile}): {stages} stages, {stage_kib / max(stages, 1):.1f} KiB per stage raw")
        per["stage"][label] = stage_kib / max(stages, 1) * 1024 * scale
        for kern in pass_kib:
            print(f"  {kern}: {passes[kern]} launches, {pass_kib[kern] / max(passes[kern], 1):.1f} KiB per launch raw")
            per[kern][label] = pass_kib[kern] / max(passes[kern], 1) * 1024 * scale
    for kernel, t in (("stage", tile), ("project", 0), ("update", 0), ("matvec", 0)):
        f, w = per[kernel]["FETCH_SIZE"], per[kernel]["WRITE_SIZE"]
        print(f"{kernel}: fetch {f:.4e} B + write {w:.4e} B per launch (scaled)")
        ch = chunk if kernel == "stage" else 0
        print(f"traffic-record: kernel={kernel} bytes_per_launch={f + w:.5e} tile={t} chunk={ch} sources={nsrc} "
              f"digest={sources_digest(kernel)}")


def config(name):
    if name == "c2":
        n, w, h, ppw, J = 1023, 16, 0.01, 8.0, 32
        return dict(n=n, w=w, h=h, omega=2 * np.pi * 1.5 / (ppw * h), J=J, two_grid=True,
                    workload="2D layered 1023^2 + 16 PML, 8 ppw, TGSP (5-pt fine, opt 9-pt FE coarse), "
                             "X-sweep J=32, w_dd=4, point source")
    if name == "c1":
        n, w, h = 127, 10, 1.0 / 128
        return dict(n=n, w=w, h=h, omega=2 * np.pi * 12.8, J=4, two_grid=False, S_outer=50.0, c_pml=1.0,
                    workload="2D constant 127^2 + 10 PML, 10 ppw, 5-pt, X-sweep J=4, point source")
    raise SystemExit(f"unknown config {name}")


def medium(cfg):
    from synth.media import layered_medium_2d, extend_into_pml
    n, w = cfg["n"], cfg["w"]
    if "c_pml" in cfg:
        return np.ones((n + 2 * w, n + 2 * w))
    return extend_into_pml(layered_medium_2d(n, n, 1412046), w)


def sources(cfg, shape, nsrc, seed=1412048):
    """Point sources at seeded random interior positions (1/h^2 at one node)."""
    from synth.media import point_source
    rng = np.random.default_rng(seed)
    w = cfg["w"]
    out = []
    for _ in range(nsrc):
        i = int(rng.integers(w + 1, shape[0] - w - 1))
        k = int(rng.integers(w + 1, shape[1] - w - 1))
        out.append(point_source(shape, (i, k), cfg["h"]))
    return out


def autotune_batch(cfg, c, nsrc, precision):
    """Chunk length and tile for the batched solves of this problem from the
    library's autotuner (one setup and four timed tile choices per candidate
    chunk length); not part of any timed region."""
    import torch
    from paper_1412_0464_amd import hsp
    ct = torch.tensor(c, device=torch.device("cuda:0"))
    t0 = time.perf_counter()
    chunk, tile, ms, table = hsp.autotune(ct, cfg["omega"], cfg["h"], cfg["w"], cfg["J"], nsrc, restart=1,
                                          S_outer=cfg.get("S_outer", 0.0), c_pml=cfg.get("c_pml", 0.0),
                                          two_grid=cfg["two_grid"], precision=precision)
    torch.cuda.synchronize()
    return {"chunk": chunk, "tile": tile, "ms": ms, "s": time.perf_counter() - t0,
            "candidates": [{"chunk": m, "tile": t, "ms": x} for m, t, x in table]}


def gpu_run_batch(cfg, c, fs, precision, steps, warmup, tol, restart=40, profile=False, tile=0, **opts):
    """Setup once, tune the right-hand-side tile (unless ``tile`` fixes it),
    then time ``steps`` batched solves of all sources after ``warmup`` ones.
    ``opts`` are further solver options (krylov_fp32)."""
    import torch
    from paper_1412_0464_amd import Helmholtz
    dev = torch.device("cuda:0")
    ct = torch.tensor(c, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs = Helmholtz(ct, cfg["omega"], cfg["h"], cfg["w"], cfg["J"], S_outer=cfg.get("S_outer", 0.0),
                   c_pml=cfg.get("c_pml", 0.0), two_grid=cfg["two_grid"], precision=precision, restart=restart,
                   **opts)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    B = torch.stack([hs.rhs(torch.tensor(f, dtype=torch.complex128, device=dev)) for f in fs])
    U = torch.empty_like(B)
    if tile:
        tile_ms = None
    else:
        tile, tile_ms = hs.tune_batch(len(fs), restart)
    for _ in range(warmup):
        hs.solve_batch(B, tol=tol, maxit=200, restart=restart, tile=tile, out=U)
    torch.cuda.synchronize()
    tot = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        _, its, rrs = hs.solve_batch(B, tol=tol, maxit=200, restart=restart, tile=tile, out=U)
        tot += sum(its)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = dict(setup_s=setup_s, solve_s=dt / steps, iters=its, relres=rrs, total_iters=tot, time_s=dt,
               tile=tile, tile_ms=tile_ms, hs=hs, U=U)
    if profile:
        # the same steps again with an event pair around every kernel class
        # launch (the records add a little time, so they stay out of the
        # steps timed above)
        hs.profile(True)
        for cls in CLASSES:
            hs.profile_read(cls)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(steps):
            hs.solve_batch(B, tol=tol, maxit=200, restart=restart, tile=tile, out=U)
        torch.cuda.synchronize()
        res["profiled_solve_s"] = (time.perf_counter() - t1) / steps
        res["classes"] = {cls: hs.profile_read(cls) for cls in CLASSES}
        hs.profile(False)
    return res


# (n, points per wavelength at 1.5 km/s, J): higher frequencies on finer
# grids; below 8 points per wavelength the coarse level of the two-grid
# method is too coarse for it to converge
C3_GRIDS = [(255, 12.0, 8), (511, 10.0, 16), (767, 9.0, 24), (1023, 8.0, 32)]


def c3_inputs(nsrc=64):
    """The batched multi-frequency workload's inputs: one seeded layered
    medium on a 10.24 km square sampled on four grids (255^2 .. 1023^2
    interior nodes + 16 PML cells), one frequency per grid (8-12 points per
    wavelength at 1.5 km/s, higher frequencies on finer grids), nsrc point
    sources per grid at seeded interior positions.  Returns a list of dicts
    (n, w, h, omega, J, c, sources)."""
    from synth.media import layered_medium_2d, extend_into_pml, resample_nodes
    L, w = 10.24, 16
    base = layered_medium_2d(1023, 1023, 1412046)
    out = []
    for n, ppw, J in C3_GRIDS:
        h = L / (n + 1)
        c = extend_into_pml(resample_nodes(base, n), w)
        om = 2 * np.pi * 1.5 / (ppw * h)
        fs = sources(dict(w=w, h=h), c.shape, nsrc, seed=1412049 + n)
        out.append(dict(n=n, w=w, h=h, omega=om, J=J, ppw=ppw, c=c, sources=fs))
    return out


_C3_TUNED = {}


def c3_tune(nsrc=64):
    """Chunk length per grid and the group's tile from the library's
    autotuner (run once per process, outside the timed solves): each grid is
    tuned for its own batch; the group takes the tile of the largest grid,
    whose stages dominate the aligned launches."""
    if nsrc in _C3_TUNED:
        return _C3_TUNED[nsrc]
    import torch
    from paper_1412_0464_amd import hsp
    dev = torch.device("cuda:0")
    per = []
    t0 = time.perf_counter()
    for q in c3_inputs(nsrc):
        chunk, tile, ms, _ = hsp.autotune(torch.tensor(q["c"], device=dev), q["omega"], q["h"], q["w"], q["J"], nsrc,
                                          restart=1, two_grid=True, precision="mixed")
        per.append({"n": q["n"], "chunk": chunk, "tile": tile, "ms": ms})
    torch.cuda.synchronize()
    _C3_TUNED[nsrc] = {"grids": per, "tile": per[-1]["tile"], "s": time.perf_counter() - t0}
    return _C3_TUNED[nsrc]


def c3_run(steps, warmup, tol, nsrc=64, graph=False, tuned=None):
    """All 4 x nsrc right-hand sides of c3_inputs solved to tol in one group
    (every aligned sweep step is one launch pair over all grids); with
    ``tuned`` (c3_tune) the autotuner's chunk lengths and tile."""
    import torch
    from paper_1412_0464_amd import Group, Helmholtz
    dev = torch.device("cuda:0")
    probs, Bs, dofs = [], [], []
    for k, q in enumerate(c3_inputs(nsrc)):
        chunk = tuned["grids"][k]["chunk"] if tuned else 0
        hs = Helmholtz(torch.tensor(q["c"], device=dev), q["omega"], q["h"], q["w"], q["J"], two_grid=True,
                       precision="mixed", restart=40, chunk=chunk)
        Bs.append(torch.stack([hs.rhs(torch.tensor(f, dtype=torch.complex128, device=dev)) for f in q["sources"]]))
        probs.append(hs)
        dofs.append(q["n"] * q["n"])
    w = 16
    grp = Group(probs, restart=40)
    tile = tuned["tile"] if tuned else 0
    for _ in range(warmup):
        grp.solve(Bs, tol=tol, maxit=200, graph=graph, tile=tile)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    work = 0
    for _ in range(steps):
        _, its, rrs = grp.solve(Bs, tol=tol, maxit=200, graph=graph, tile=tile)
        work += sum(d * sum(it) for d, it in zip(dofs, its))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"value": work / dt, "unit": UNIT, "solve_s": dt / steps, "sources_per_grid": nsrc,
            "grids": [f"{n}^2 + {w} PML, ppw {ppw}, J={J}" for n, ppw, J in C3_GRIDS],
            "iterations": [[min(it), max(it)] for it in its], "relres_max": max(max(r) for r in rrs),
            "graph": bool(graph), "autotune": tuned}


def c4_config():
    """The 3-D workload: a seeded smooth random medium (linear depth trend
    1.5 -> 4.5 km/s times 1 + 5 % Gaussian random field, correlation length
    10 cells) on 127^3 interior nodes + 8 PML cells per side, h = 20 m,
    10 points per wavelength at 1.5 km/s (7.5 Hz), two-grid sweeping
    preconditioner with the 7-point fine level and the optimized 27-point
    FE coarse level (79^3), X-sweep over J = 16 coarse slabs of 4 layers
    plus 3 DD-PML layers per side, nu = 3, omega_jac = 0.6."""
    n, w, h, ppw, J = 127, 8, 0.02, 10.0, 16
    return dict(n=n, w=w, h=h, omega=2 * np.pi * 1.5 / (ppw * h), J=J, w_dd=3, omega_jac=0.6,
                workload="3D smooth random 127^3 + 8 PML, 10 ppw, TGSP (7-pt fine, opt 27-pt FE coarse 79^3), "
                         "X-sweep J=16, w_dd=3, point source")


def c4_medium(cfg, seed=1412047):
    from synth.media import smooth_medium_3d
    n, w = cfg["n"], cfg["w"]
    return np.pad(smooth_medium_3d(n, n, n, seed, corr_len=10.0), w, mode="edge")


def c4_run(steps, warmup, tol, profile=True, slab_factor="nd"):
    """Setup (timed alone), then ``steps`` solves of a point source at the
    centre to ``tol``; optionally a profiled repeat with event pairs around
    every kernel class.  ``slab_factor``: 'nd' (nested dissection of the
    slab planes, the default) or 'block' (block tridiagonal along y);
    ``steps`` = 0 stops after the setup."""
    import torch
    from paper_1412_0464_amd import Helmholtz
    from synth.media import point_source
    cfg = c4_config()
    dev = torch.device("cuda:0")
    c = c4_medium(cfg)
    ct = torch.tensor(c, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs = Helmholtz(ct, cfg["omega"], cfg["h"], cfg["w"], cfg["J"], two_grid=True, w_dd=cfg["w_dd"],
                   omega_jac=cfg["omega_jac"], restart=60, slab_factor=slab_factor)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"[bench] c4 ({slab_factor}) setup {setup_s:.3f} s, pivot growth {hs.pivot_growth:.3f}", file=sys.stderr,
          flush=True)
    if steps == 0:
        return {"setup_s": setup_s, "slab_factor": slab_factor, "u": None, "hs": hs}
    f = point_source(c.shape, tuple(s // 2 for s in c.shape), cfg["h"])
    b = hs.rhs(torch.tensor(f, dtype=torch.complex128, device=dev))
    u = torch.empty_like(b)
    for _ in range(warmup):
        hs.solve(b, tol=tol, maxit=200, out=u)
    torch.cuda.synchronize()
    its = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        _, it, rr = hs.solve(b, tol=tol, maxit=200, out=u)
        its += it
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dof = cfg["n"] ** 3
    out = {"workload": cfg["workload"], "value": dof * its / dt, "unit": UNIT, "solve_s": dt / steps,
           "setup_s": setup_s, "iterations": it, "relres": rr, "dof_interior": dof, "unknowns": int(c.size),
           "pivot_growth": hs.pivot_growth, "precision": "mixed (complex64 factors on FP32 MFMA, complex128 FGMRES)",
           "slab_factor": slab_factor}
    if profile:
        hs.profile(True)
        for cls in CLASSES:
            hs.profile_read(cls)
        for _ in range(steps):
            hs.solve(b, tol=tol, maxit=200, out=u)
        torch.cuda.synchronize()
        cl = {cls: hs.profile_read(cls) for cls in CLASSES}
        hs.profile(False)
        out["kernel_ms_per_solve"] = {k: v[0] / steps for k, v in cl.items()}
        ms, n, by = cl["stage"]
        out["stage"] = {"launch_groups": n, "avg_us": ms * 1e3 / max(n, 1), "alg_bytes_per_stage": by / max(n, 1),
                        "achieved_gbs": (by / max(n, 1)) / (ms * 1e-3 / max(n, 1)) / 1e9 if n else 0.0}
        ach = out["stage"]["achieved_gbs"]
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS,
                           "traffic": recorded_traffic("nd_stage", 0, 1, 0, ND_TRAFFIC_RECORD)
                           if slab_factor == "nd" else None,
                           "kernel": "3-D SubdomSolve stage (" + ("kn_fwd / kn_bwd per dissection level"
                                                                  if slab_factor == "nd" else "k3s_step per y-block")
                                     + ", k3s_prep, k3s_fin)"}
    out["u"] = u
    out["hs"] = hs
    return out


def c4_report(args, slab_factor, setup_only=False):
    r4 = c4_run(0 if setup_only else args.steps, args.warmup, args.tol, slab_factor=slab_factor)
    r4.pop("u")
    hs = r4.pop("hs")
    hs.close()
    if setup_only:
        return r4
    print(f"[bench] c4 ({slab_factor}): setup {r4['setup_s']:.2f} s, solve {r4['solve_s'] * 1e3:.1f} ms, "
          f"{r4['iterations']} iterations, {r4['value']:.3e} dof*iter/s", file=sys.stderr, flush=True)
    return r4


def gpu_run(cfg, c, f, precision, steps, warmup, tol, profile=False):
    """Setup once, then time ``steps`` complete solves after ``warmup`` ones.
    With ``profile`` the same solves are repeated with the library bracketing
    every kernel launch of each class with HIP events on the solve's stream."""
    import torch
    from paper_1412_0464_amd import Helmholtz
    dev = torch.device("cuda:0")
    ct = torch.tensor(c, device=dev)
    ft = torch.tensor(f, dtype=torch.complex128, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hs = Helmholtz(ct, cfg["omega"], cfg["h"], cfg["w"], cfg["J"], S_outer=cfg.get("S_outer", 0.0),
                   c_pml=cfg.get("c_pml", 0.0), two_grid=cfg["two_grid"], precision=precision, restart=60)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    b = hs.rhs(ft)
    u = torch.empty_like(b)
    for _ in range(warmup):
        hs.solve(b, tol=tol, maxit=200, out=u)
    torch.cuda.synchronize()
    its = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, it, rr = hs.solve(b, tol=tol, maxit=200, out=u)
        its.append(it)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = dict(setup_s=setup_s, solve_s=dt / steps, iters=its[-1], relres=rr, total_iters=sum(its), time_s=dt)
    if profile:
        hs.profile(True)
        for cls in CLASSES:
            hs.profile_read(cls)
        for _ in range(steps):
            hs.solve(b, tol=tol, maxit=200, out=u)
        torch.cuda.synchronize()
        res["classes"] = {cls: hs.profile_read(cls) for cls in CLASSES}
        hs.profile(False)
    res["u"] = u
    res["hs"] = hs
    return res


def _host_info():
    """Host facts for the CPU baseline: logical CPUs, the CPUs this process
    may run on, the CPU model and the BLAS thread pools."""
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        info["blas_threads"] = {d.get("internal_api", "?"): d.get("num_threads") for d in threadpool_info()}
    except Exception:  # noqa: BLE001 - informational only
        pass
    return info


def cpu_baseline(cfg, c, f, iters, tol):
    """The CPU reference implementation (oracle), untuned, on a bounded
    sample of the same workload: its full setup, then ``iters`` FGMRES
    iterations of the same solve.  The thread pools are left at their
    defaults; SciPy's sparse products and SuperLU run on one thread, so the
    threads actually used are measured as CPU time / wall time."""
    from oracle.problem import Problem2D
    dof = cfg["n"] ** 2
    c0 = time.process_time()
    t0 = time.perf_counter()
    P = Problem2D(c, cfg["omega"], cfg["h"], cfg["w"], S_outer=cfg.get("S_outer"), c_pml=cfg.get("c_pml"),
                  J=cfg["J"], w_dd=4, two_grid=cfg["two_grid"])
    t1 = time.perf_counter()
    c1 = time.process_time()
    _, it, hist, _ = P.solve(f, tol=tol, maxit=iters)
    t2 = time.perf_counter()
    c2 = time.process_time()
    used = (c2 - c1) / max(t2 - t1, 1e-9)
    out = {"value": dof * it / (t2 - t1), "unit": UNIT, "cores": max(1, int(round(used))), "kind": "oracle",
           "sample": f"full setup ({t1 - t0:.1f} s) + {it} FGMRES iterations of the same solve "
                     f"({t2 - t1:.1f} s); value = interior dof x iterations / iteration time",
           "setup_s": t1 - t0, "s_per_iter": (t2 - t1) / max(it, 1),
           "threads_used_cpu_over_wall": {"setup": (c1 - c0) / max(t1 - t0, 1e-9), "iterations": used}}
    out.update(_host_info())
    return out


def cpu_c3_sample(per_grid=1, seed=1412050):
    """The oracle on a seeded subset of the multi-frequency workload:
    ``per_grid`` of the 64 sources on each of the four grids (4 of the 256
    systems by default), each grid's full FP64 setup and complete solves to
    1e-6.  ``value`` is the subset's interior dof x iterations / solve time;
    the whole group's oracle time is extrapolated as each grid's setup plus
    64 times its mean solve time."""
    from oracle.problem import Problem2D
    rng = np.random.default_rng(seed)
    work, solve_s, extra, grids = 0, 0.0, 0.0, []
    c0 = time.process_time()
    w0 = time.perf_counter()
    for q in c3_inputs():
        t0 = time.perf_counter()
        P = Problem2D(q["c"], q["omega"], q["h"], q["w"], J=q["J"], w_dd=4, two_grid=True)
        t1 = time.perf_counter()
        picks = sorted(int(i) for i in rng.choice(len(q["sources"]), per_grid, replace=False))
        its, ts = [], []
        for i in picks:
            s0 = time.perf_counter()
            _, it, _, _ = P.solve(q["sources"][i], tol=1e-6, maxit=200)
            ts.append(time.perf_counter() - s0)
            its.append(it)
        dof = q["n"] * q["n"]
        work += dof * sum(its)
        solve_s += sum(ts)
        extra += (t1 - t0) + len(q["sources"]) * float(np.mean(ts))
        grids.append({"n": q["n"], "setup_s": t1 - t0, "sources": picks, "iterations": its, "solve_s": ts})
        del P
    used = (time.process_time() - c0) / max(time.perf_counter() - w0, 1e-9)
    return {"value": work / solve_s, "unit": UNIT, "cores": max(1, int(round(used))), "kind": "oracle",
            "sample": f"{per_grid} seeded source{'s' if per_grid > 1 else ''} per grid ({4 * per_grid} of 256 systems): FP64 setup per grid and "
                      f"complete solves to 1e-6; value = interior dof x iterations / solve time",
            "extrapolated_group_s": extra, "grids": grids}


def cpu_c4_sample():
    """The oracle on a bounded part of the 3-D workload, whose full FP64
    setup (16 SuperLU slab factorizations of about 69 k unknowns each) does
    not fit a benchmark run: one middle slab of the 79^3 coarse level
    assembled and factored, one solve with it, and the product with the
    fine 7-point operator.  An X-sweep applies 2 J slab solves and the
    two-grid cycle 2 nu + 2 fine products (smoothing, residual, FGMRES
    product), which gives the extrapolated time per iteration; the setup is
    extrapolated as J middle-slab factorizations (the two end slabs are
    wider by their PML)."""
    import scipy.sparse.linalg as spla
    from oracle import discretization as D, dd as DD, problem3d as P3, twogrid as TG
    cfg = c4_config()
    c = c4_medium(cfg)
    n, w, h, om, J = cfg["n"], cfg["w"], cfg["h"], cfg["omega"], cfg["J"]
    N = n + 1 + 2 * w
    cp = float(c.mean())
    c0 = time.process_time()
    w0 = time.perf_counter()
    axes = [D.uniform_axis(N, h, w, 5.0 * w, cp) for _ in range(3)]
    k2n = om ** 2 / c ** 2
    A = P3.Level3D(*axes, om, "fd7", k2_nodes=k2n).matrix().tocsr()
    cax, Ws = [], []
    for a in axes:
        ca, ifp, ref = TG.coarsen_axis(a, w)
        cax.append(ca)
        Ws.append(TG.cell_average_1d(ifp, ref, N))
    lev = P3.Level3D(*cax, om, "fe27", k2_cells=P3.cell_average_3d(*Ws, P3.pad_nodes_edge_3d(k2n)))
    beta = DD.partition(lev.n1, w, J)
    j = J // 2
    t0 = time.perf_counter()
    As = lev.slab_level(beta, j, cfg["w_dd"], 5.0 * cfg["w_dd"], cp).matrix().tocsc()
    t1 = time.perf_counter()
    lu = spla.splu(As)
    t2 = time.perf_counter()
    rng = np.random.default_rng(1412051)
    x = lu.solve(rng.standard_normal(As.shape[0]) + 1j * rng.standard_normal(As.shape[0]))
    t3 = time.perf_counter()
    v = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    y = A @ v
    t4 = time.perf_counter()
    del x, y
    used = (time.process_time() - c0) / max(time.perf_counter() - w0, 1e-9)
    nu = 3
    per_iter = 2 * J * (t3 - t2) + (2 * nu + 2) * (t4 - t3)
    return {"value": n ** 3 / per_iter, "unit": UNIT, "cores": max(1, int(round(used))), "kind": "oracle",
            "sample": f"coarse slab {j} of {J} ({As.shape[0]} unknowns): assembly {t1 - t0:.1f} s, SuperLU "
                      f"{t2 - t1:.1f} s, one solve {t3 - t2:.2f} s; fine 7-point product {t4 - t3:.3f} s; value = "
                      f"interior dof / ({2 * J} slab solves + {2 * nu + 2} fine products), extrapolated",
            "extrapolated_s_per_iter": per_iter, "extrapolated_setup_s": J * (t2 - t0),
            "slab_unknowns": int(As.shape[0]), "slab_factor_nnz": int(lu.L.nnz + lu.U.nnz)}


def oracle_check(cfg, c, fs, U, sampled):
    """Relative L2 error of sampled GPU solutions (batched, mixed precision)
    against the oracle's direct solution of the same FP64 system (sparse LU
    of the fine operator), computed outside the timed region."""
    import scipy.sparse.linalg as spla
    from oracle import discretization as D
    N = cfg["n"] + 1 + 2 * cfg["w"]
    cp = float(c.mean()) if not cfg.get("c_pml") else cfg["c_pml"]
    S_o = cfg.get("S_outer") or 5.0 * cfg["w"]
    ax = D.uniform_axis(N, cfg["h"], cfg["w"], S_o, cp)
    t0 = time.perf_counter()
    lu = spla.splu(D.fd5_matrix(ax, ax, cfg["omega"] ** 2 / c ** 2, cfg["omega"]).tocsc())
    scale = D.fd5_rhs_scale(ax, ax, cfg["omega"])
    errs = {}
    for j in sampled:
        x = lu.solve((scale * fs[j]).ravel())
        errs[str(j)] = float(np.linalg.norm(U[j].ravel() - x) / np.linalg.norm(x))
    return {"kind": "oracle direct solve (SuperLU of the FP64 fine operator)", "sources": list(sampled),
            "rel_l2_error": errs, "max_rel_l2_error": max(errs.values()), "oracle_s": time.perf_counter() - t0}


def c3_report(args, graph):
    tuned = c3_tune(args.c3_sources)
    r3 = c3_run(max(1, args.steps - 1), 1, args.tol, nsrc=args.c3_sources, graph=graph, tuned=tuned)
    print(f"[bench] c3 group (graph={graph}): {r3['solve_s'] * 1e3:.1f} ms, {r3['value']:.3e} dof*iter/s",
          file=sys.stderr, flush=True)
    return r3


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--sources", type=int, default=64, help="right-hand sides of the batched solve")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-single", action="store_true", help="skip the single-source mixed run")
    ap.add_argument("--no-krylov-fp32", action="store_true",
                    help="skip the batched run with the Arnoldi basis in complex64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=10)
    ap.add_argument("--no-cpu-samples", action="store_true",
                    help="skip the oracle's timed samples of the multi-frequency and 3-D workloads")
    ap.add_argument("--no-c3", action="store_true", help="skip the batched multi-frequency group workload")
    ap.add_argument("--no-c4", action="store_true", help="skip the 3-D workload")
    ap.add_argument("--no-fp64-batched", action="store_true",
                    help="skip the plain FP64 batched run (same batch, restart, tile and chunk)")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the batched runs with the NX-sweep and with sponge layers")
    ap.add_argument("--no-oracle-check", action="store_true",
                    help="skip the error of sampled solutions against the oracle's direct solve")
    ap.add_argument("--c3-sources", type=int, default=64)
    ap.add_argument("--c3-only", action="store_true",
                    help="time only the group workload (no config-2 runs, no CPU baseline)")
    ap.add_argument("--c4-only", action="store_true", help="time only the 3-D workload")
    ap.add_argument("--c4-slab-factor", nargs="+", choices=("nd", "block"), default=["nd", "block"],
                    help="3-D slab factorizations to time (nested dissection, block tridiagonal)")
    ap.add_argument("--c4-setup-only", action="store_true", help="with --c4-only: stop after the setups")
    ap.add_argument("--c3-graph", choices=("both", "off", "on"), default="both",
                    help="group solves eager (off), with the preconditioner captured in a graph (on), or both")
    ap.add_argument("--tile", type=int, default=0, help="right-hand-side tile (0: tuned)")
    ap.add_argument("--chunk", type=int, default=AUTOTUNE,
                    help="tangential blocks per chunk of the slab substitutions in the batched solves "
                         "(-1: chosen with the tile by the library's autotuner, hsp_autotune; 0: about sqrt of "
                         "the tangential nodes, the single-source choice)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a streaming kernel of known size (for counter scaling)")
    ap.add_argument("--reduce-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="summarise rocprofv3 counter files of the batched stage and exit (no GPU)")
    args = ap.parse_args()
    if args.reduce_counters:
        reduce_counters(*args.reduce_counters, tile=args.tile or 4, nsrc=args.sources, chunk=args.chunk)
        return
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design, not a measured path", file=sys.stderr)
        sys.exit(2)

    c3_graphs = {"both": (False, True), "off": (False,), "on": (True,)}[args.c3_graph]
    if args.c4_only:
        out = {}
        for sf in args.c4_slab_factor:
            r4 = c4_report(args, sf, args.c4_setup_only)
            out["c4" if sf == "nd" else "c4_" + sf] = r4
        print(json.dumps(out))
        return
    if args.c3_only:
        out = {}
        for graph in c3_graphs:
            out["c3_graph" if graph else "c3"] = c3_report(args, graph)
        print(json.dumps(out))
        return

    cfg = config(args.config)
    c = medium(cfg)
    fs = sources(cfg, c.shape, args.sources)
    dof = cfg["n"] ** 2
    print(f"[bench] {cfg['workload']}: {dof} interior dof, {c.size} unknowns, {len(fs)} sources",
          file=sys.stderr, flush=True)

    tuned = None
    if args.chunk == AUTOTUNE:
        tuned = autotune_batch(cfg, c, len(fs), "mixed")
        args.chunk = tuned["chunk"]
        if not args.tile:
            args.tile = tuned["tile"]
        print(f"[bench] autotuner: chunk {tuned['chunk']}, tile {tuned['tile']} ({tuned['ms']:.2f} ms per batched "
              f"preconditioner application; {tuned['s']:.1f} s)", file=sys.stderr, flush=True)
    if args.copy_calibration:
        copy_calibration()
    bat = gpu_run_batch(cfg, c, fs, "mixed", args.steps, args.warmup, args.tol, profile=True, tile=args.tile,
                        chunk=args.chunk)
    its = bat["iters"]
    print(f"[bench] batched mixed: setup {bat['setup_s']:.3f} s, tile {bat['tile']}, solve {bat['solve_s'] * 1e3:.1f} ms "
          f"for {len(fs)} sources, iterations {min(its)}..{max(its)}, max relres {max(bat['relres']):.2e}",
          file=sys.stderr, flush=True)
    value = dof * bat["total_iters"] / bat["time_s"]
    workload = cfg["workload"].replace("point source", f"{len(fs)} point sources in one batch")
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": bat["solve_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "c64+c128", "data": "synthetic",
        "config": {"workload": workload, "dof_interior": dof, "unknowns": int(c.size), "sources": len(fs),
                   "iterations_min": min(its), "iterations_max": max(its), "relres_max": max(bat["relres"]),
                   "setup_s": bat["setup_s"], "solve_s": bat["solve_s"],
                   "solve_s_per_source": bat["solve_s"] / len(fs), "precision": "mixed",
                   "rhs_tile": bat["tile"], "chunk": args.chunk},
    }
    if tuned is not None:
        out["config"]["autotune"] = tuned
    # rooflines from the event-timed classes of the profiled repeat:
    # algorithmic bytes per launch / average launch time.  The dominant kernel
    # class is the SubdomSolve stage (two dependent launches timed as one,
    # about 40 % of a solve); the two HBM-bound passes of the complex128
    # Gram-Schmidt follow: the update pass (k_bdcgs_update: k basis vectors,
    # u_k and w read, v_k and u_{k+1} written; the kernel with the largest
    # total time) as roofline_update and the projection pass (k_bmultidot2:
    # every basis vector and w once per Arnoldi step; its event pair also
    # covers two small reductions) as roofline_project.  roofline_matvec is the
    # batched 5-point FGMRES matvec (k_stencil_multi: z read and w written per
    # source, k^2 read once).
    cls = bat["classes"]

    def roofline(name, kernel, traffic):
        ms, n, by = cls[name]
        per_launch_bytes = by / max(n, 1)
        per_launch_s = ms * 1e-3 / max(n, 1)
        achieved = per_launch_bytes / per_launch_s / 1e9 if n else 0.0
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel, "launches": n,
                "avg_launch_us": per_launch_s * 1e6, "alg_bytes_per_launch": per_launch_bytes}

    out["roofline"] = roofline("stage", "batched SubdomSolve stage (k_bstage_fwd + k_bstage_bwd)",
                               recorded_traffic("stage", bat["tile"], len(fs), args.chunk))
    out["roofline_project"] = roofline("project", "FGMRES projection pass k_bmultidot2<double> (complex128 basis)",
                                       recorded_traffic("project", bat["tile"], len(fs)))
    out["roofline_update"] = roofline("update", "FGMRES update pass k_bdcgs_update<double> (complex128 basis)",
                                      recorded_traffic("update", bat["tile"], len(fs)))
    out["roofline_matvec"] = roofline("krylov", "FGMRES matvec k_stencil_multi<5> (batched 5-point operator)",
                                      recorded_traffic("matvec", bat["tile"], len(fs)))
    # the same stage against the FP32 vector ALU by the method's flops: per
    # slab solve and source, forward y_t = G_t (f_t - A_t y_{t-1}) and
    # backward x_t = y_t - E_t x_{t+1} take 2 nl^2 + 3 nl complex multiply-adds
    # (8 real flops each) per tangential node; an X-sweep solves every slab
    # twice, and each FGMRES iteration of a source applies the preconditioner
    # once (the chunked evaluation's extra fix-up products are not counted)
    hs_b = bat["hs"]
    n2c = hs_b.n_coarse[1] if hs_b.two_grid else hs_b.n_fine[1]
    flops_app = sum(2.0 * n2c * 8.0 * (2.0 * nl * nl + 3.0 * nl)
                    for nl in (x1 - x0 + 1 for x0, x1 in zip(hs_b.x0, hs_b.x1)))
    st_ms, st_n, _ = cls["stage"]
    achieved_tf = (bat["total_iters"] / args.steps) * flops_app / (st_ms * 1e-3 / args.steps) / 1e12
    out["roofline_stage_flops"] = {"bound": "alu", "achieved": achieved_tf, "peak": FP32_PEAK_TFLOPS,
                                   "unit": "TFLOP/s", "frac": achieved_tf / FP32_PEAK_TFLOPS, "traffic": None,
                                   "kernel": "batched SubdomSolve stage (k_bstage_fwd + k_bstage_bwd), complex64",
                                   "flop_per_application_per_source": flops_app}
    out["config"]["kernel_ms_per_solve"] = {k: v[0] / args.steps for k, v in cls.items()}
    out["config"]["profiled_solve_s"] = bat["profiled_solve_s"]
    samp = [0, len(fs) // 2, len(fs) - 1]
    Ub = {j: bat["U"][j].cpu().numpy() for j in samp}
    bat_tile = bat["tile"]
    del bat
    if not args.no_krylov_fp32:
        bk = gpu_run_batch(cfg, c, fs, "mixed", args.steps, args.warmup, args.tol, tile=bat_tile, krylov_fp32=True,
                           chunk=args.chunk)
        kits = bk["iters"]
        print(f"[bench] batched mixed, complex64 basis: solve {bk['solve_s'] * 1e3:.1f} ms, iterations "
              f"{min(kits)}..{max(kits)}, max relres {max(bk['relres']):.2e}", file=sys.stderr, flush=True)
        out["batched_krylov_fp32"] = {"value": dof * bk["total_iters"] / bk["time_s"], "solve_s": bk["solve_s"],
                                      "iterations_min": min(kits), "iterations_max": max(kits),
                                      "relres_max": max(bk["relres"]), "rhs_tile": bk["tile"]}
        del bk
    if not args.no_fp64_batched:
        bf = gpu_run_batch(cfg, c, fs, "fp64", args.steps, args.warmup, args.tol, tile=bat_tile, chunk=args.chunk)
        fits = bf["iters"]
        print(f"[bench] batched fp64: solve {bf['solve_s'] * 1e3:.1f} ms, iterations {min(fits)}..{max(fits)}, "
              f"max relres {max(bf['relres']):.2e}", file=sys.stderr, flush=True)
        out["fp64_batched"] = {"value": dof * bf["total_iters"] / bf["time_s"], "solve_s": bf["solve_s"],
                               "setup_s": bf["setup_s"], "iterations_min": min(fits), "iterations_max": max(fits),
                               "relres_max": max(bf["relres"]), "rhs_tile": bf["tile"], "chunk": args.chunk,
                               "speedup_mixed_over_fp64_same_batch": bf["solve_s"] / out["config"]["solve_s"]}
        del bf
    if not args.no_variants:
        # the same batch with the partial sweeps over two groups (SweepingPrecNX)
        # and with the outer PML cells replaced by sponge layers (the two-grid
        # method then coarsens every cell)
        for key, label, extra in (("c2_nx", "NX-sweep, 2 groups", dict(sweep="nx", ncell=2)),
                                  ("c2_sponge", "sponge layers (16 cells)", dict(sponge=True))):
            bv = gpu_run_batch(cfg, c, fs, "mixed", args.steps, args.warmup, args.tol, tile=bat_tile,
                               chunk=args.chunk, profile=True, **extra)
            vits = bv["iters"]
            ms_st, n_st, by_st = bv["classes"]["stage"]
            print(f"[bench] batched mixed, {label}: solve {bv['solve_s'] * 1e3:.1f} ms, iterations "
                  f"{min(vits)}..{max(vits)}, max relres {max(bv['relres']):.2e}", file=sys.stderr, flush=True)
            out[key] = {"variant": label, "value": dof * bv["total_iters"] / bv["time_s"], "solve_s": bv["solve_s"],
                        "setup_s": bv["setup_s"], "iterations_min": min(vits), "iterations_max": max(vits),
                        "relres_max": max(bv["relres"]), "rhs_tile": bv["tile"], "chunk": args.chunk,
                        "stage": {"avg_us": ms_st * 1e3 / max(n_st, 1),
                                  "achieved_gbs": (by_st / max(n_st, 1)) / (ms_st * 1e-3 / max(n_st, 1)) / 1e9
                                  if n_st else 0.0},
                        "kernel_ms_per_solve": {k: v[0] / args.steps for k, v in bv["classes"].items()}}
            del bv
    if not args.no_fp64:
        fp = gpu_run(cfg, c, fs[0], "fp64", args.steps, args.warmup, args.tol)
        print(f"[bench] plain fp64, one source: setup {fp['setup_s']:.3f} s, solve {fp['solve_s'] * 1e3:.2f} ms, "
              f"{fp['iters']} iters", file=sys.stderr, flush=True)
        uf = fp["u"].cpu().numpy()
        out["fp64"] = {"value": dof * fp["total_iters"] / fp["time_s"], "solve_s": fp["solve_s"],
                       "setup_s": fp["setup_s"], "iterations": fp["iters"], "relres": fp["relres"],
                       "batched_mixed_vs_fp64_rel_l2_source0": float(np.linalg.norm(Ub[0] - uf) / np.linalg.norm(uf))}
        del fp
    if not args.no_single:
        sm = gpu_run(cfg, c, fs[0], "mixed", args.steps, args.warmup, args.tol, profile=True)
        print(f"[bench] mixed, one source: solve {sm['solve_s'] * 1e3:.2f} ms, {sm['iters']} iters",
              file=sys.stderr, flush=True)
        scl = sm["classes"]
        s_ms, s_n, s_b = scl["stage"]
        out["single_mixed"] = {"value": dof * sm["total_iters"] / sm["time_s"], "solve_s": sm["solve_s"],
                               "iterations": sm["iters"], "relres": sm["relres"],
                               "stage_avg_us": s_ms * 1e3 / max(s_n, 1),
                               "stage_frac_hbm": (s_b / max(s_n, 1)) / (s_ms * 1e-3 / max(s_n, 1)) / 1e9
                               / HBM_PEAK_GBS,
                               "kernel_ms_per_solve": {k: v[0] / args.steps for k, v in scl.items()}}
        if "fp64" in out:
            out["fp64"]["speedup_single_mixed_over_fp64"] = out["fp64"]["solve_s"] / sm["solve_s"]
        del sm
    if not args.no_c3:
        for graph in c3_graphs:
            out["c3_graph" if graph else "c3"] = c3_report(args, graph)
    if not args.no_c4:
        for sf in args.c4_slab_factor:
            out["c4" if sf == "nd" else "c4_" + sf] = c4_report(args, sf)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(cfg, c, fs[0], args.cpu_iters, args.tol)
        if Ub is not None and not args.no_oracle_check:
            print("[bench] sampled batched solutions against the oracle's direct solve ...", file=sys.stderr,
                  flush=True)
            out["cpu_baseline"]["oracle_check"] = oracle_check(cfg, c, fs, Ub, [0, len(fs) // 2, len(fs) - 1])
        if not args.no_cpu_samples and "c3" in out:
            print("[bench] oracle sample of the multi-frequency group ...", file=sys.stderr, flush=True)
            out["c3"]["cpu_baseline"] = cpu_c3_sample()
        if not args.no_cpu_samples and "c4" in out:
            print("[bench] oracle sample of the 3-D workload ...", file=sys.stderr, flush=True)
            out["c4"]["cpu_baseline"] = cpu_c4_sample()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
