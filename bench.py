#!/usr/bin/env python3
"""Benchmark: ms per solve to rtol 1e-6 on the 1,048,576-cell Jacobian.

Workload: the seeded 128x128x64 synthetic fully implicit Jacobian (3x3
blocks, 7-point stencil, log-normal permeability, seed 2), 256 subdomains
(16x16 of 8x8x64) with overlap 1, GMRES(30) to rtol 1e-6 from x0 = 0.
The headline is the two-level coarsened-overlap preconditioner (near boxes
4^3, far boxes 16^3) with FP64 factors; the same line carries the FP32-factor
variant and the classical (restricted) form.

A step is one complete solve (asm_solve) with A, the factors and b already
resident in HBM; setup is timed separately.  Kernel-phase durations come from
HIP events recorded by the library on the solve stream inside the timed
region; the dominant kernel's algorithmic bytes per launch divided by its
mean launch time give the roofline figure (HBM peak 8 TB/s).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GRID, SEED = (128, 128, 64), 2
SPLIT = dict(sx=16, sy=16, overlap=1)
NEAR, FAR = (4, 4, 4), (16, 16, 16)
HBM_PEAK_GBS = 8000.0
RESTART = 30
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "ilu_apply_two_level_1M_traffic.json")
# Sources that decide what the sweep kernel reads and writes: the kernel
# itself and the host code that lays out its records.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1401_7227_amd", "csrc", f)
                  for f in ("kernels.hip", "kernels.hpp", "plan.hpp", "setup.hpp", "setup.cpp")]
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written per launch


def kernel_source_sha():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per sweep launch from the committed counter runs (FETCH_SIZE
    and WRITE_SIZE per dispatch, each scaled by what the same counter reads
    for a copy of known size), or None if the kernel source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != kernel_source_sha():
        return None
    return (t["fetch_kib_per_dispatch"] * t["copy_fetch_factor"]
            + t["write_kib_per_dispatch"] * t["copy_write_factor"]) * 1024.0


def ilu_apply_bytes(st, N, fp32=False):
    """Algorithmic bytes of one preconditioner application (sweeps kernel):
    every factor block once (L, U, D^-1: 72 B in FP64, 36 B in FP32 for fine
    rows), one 4-byte column index per off-diagonal block, 16 B of per-row
    metadata (row order, right-hand side source, output cell, row start),
    the gathered right-hand side (24 B per extended row) and the written
    solution (24 B per cell)."""
    blocks, rows = st["factor_blocks"], st["ext_rows"]
    fine_blocks = st["fine_row_blocks"]
    vbytes = (fine_blocks * 36 + (blocks - fine_blocks) * 72) if fp32 else blocks * 72
    return vbytes + (blocks - rows) * 4 + rows * 16 + rows * 24 + N * 24


def spmv_bytes(nnzb, N):
    """Blocks (72 B) + column indices (4 B) + row starts + x read + y write."""
    return nnzb * 76 + N * 4 + 2 * 24 * N


def krylov_vector_bytes(n, iters, cycles, restart):
    """Dots and update passes: step j of a cycle reads j+1 basis vectors and
    w in each pass and writes one vector in the update."""
    js = []
    left = iters
    for _ in range(cycles):
        k = min(restart, left)
        js += list(range(k))
        left -= k
    dots = sum((j + 2) * 8 * n for j in js)
    update = sum((j + 3) * 8 * n for j in js)
    return dots, update, len(js)


def timed_solves(P, torch, G, B, b, steps, warmup, profile):
    """Times `steps` solves; `profile` names the phases timed by HIP events
    inside the timed region (None: none)."""
    x = torch.zeros_like(b)
    info = None
    for _ in range(warmup):
        x.zero_()
        _, info = P.solve(G, B, b, out=x, restart=RESTART, rtol=1e-6, max_iters=5000)
    G.profile(profile is not None, phases=profile)
    G.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        _, info = P.solve(G, B, b, out=x, restart=RESTART, rtol=1e-6, max_iters=5000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = G.profile_read(reset=True)
    G.profile(False)
    return (t1 - t0) / steps * 1e3, info, prof, x


def cpu_baseline(s, gpu_iters, budget_steps):
    """The CPU oracle (single thread, FP64) on a bounded sample of the same
    workload: the oracle's setup of the same preconditioner, then a fixed
    number of GMRES steps, scaled to one solve of the GPU's iteration count."""
    import oracle as O
    A = O.Matrix.from_system(s)
    t0 = time.perf_counter()
    Bo = O.Precond(A, kind=O.KIND_TWO_LEVEL, combine=O.RESTRICTED, near=NEAR, far=FAR, **SPLIT)
    t1 = time.perf_counter()
    res = O.gmres(A, Bo, s.b, restart=RESTART, fixed_iters=budget_steps)
    t2 = time.perf_counter()
    per_step = (t2 - t1) / budget_steps
    return {"value": round(per_step * gpu_iters * 1e3, 1), "unit": "ms/solve", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup ({t1 - t0:.1f} s, not in the metric) plus {budget_steps} GMRES steps "
                      f"({t2 - t1:.1f} s) of the same 1M-cell two-level solve, scaled to {gpu_iters} steps",
            "setup_s": round(t1 - t0, 2), "s_per_step": round(per_step, 3)}


def batch_systems(gen, np, count=256):
    """256 systems: nx, ny uniform in 16..96, nz uniform in 8..32 (seed 1000+s
    for system s), subdomains clamp(round(cells/4096), 16, 64) split in
    proportion to nx:ny; two-level RAS, overlap 1, near 4^3, far 16^3."""
    rng = np.random.default_rng(77)
    out = []
    for k in range(count):
        nx, ny = int(rng.integers(16, 97)), int(rng.integers(16, 97))
        nz = int(rng.integers(8, 33))
        cells = nx * ny * nz
        nsub = int(min(64, max(16, round(cells / 4096))))
        sx = max(1, min(nx, int(round((nsub * nx / ny) ** 0.5))))
        sy = max(1, min(ny, int(round(nsub / sx))))
        out.append(((nx, ny, nz), 1000 + k, dict(sx=sx, sy=sy, overlap=1)))
    return out


def bench_batch(P, gen, torch, np, args):
    specs = batch_systems(gen, np)
    systems, preconds, bs = [], [], []
    t0 = time.perf_counter()
    cells = 0
    for grid, seed, split in specs:
        s = gen.generate(*grid, seed=seed)
        cells += s.N
        G = P.System.from_generated(s)
        systems.append(G)
        preconds.append(P.Precond(G, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, near=NEAR, far=FAR,
                                  precision=P.FP32, **split))
        bs.append(torch.from_numpy(s.b).cuda())
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    kw = dict(restart=RESTART, rtol=1e-6, max_iters=5000)
    # warm-up, then one timed batched solve and one timed sequential pass
    P.solve_batch(systems, preconds, bs, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos = P.solve_batch(systems, preconds, bs, **kw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    t0 = time.perf_counter()
    seq = [P.solve(G, B, b, **kw) for G, B, b in zip(systems, preconds, bs)]
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    identical = all(bool(torch.equal(x, x1)) and i.iters == i1.iters for x, i, (x1, i1) in zip(xs, infos, seq))
    iters = [i.iters for i in infos]
    return {
        "metric": "batch of 256 independent solves to rtol 1e-6 (FP32 preconditioner, FP64 GMRES(30))",
        "value": round(t_batch * 1e3, 1), "unit": "ms/batch", "higher_is_better": False, "n_gpus": 1,
        "dtype": "f64 (FP32 factors)", "data": "synthetic (seeded generator, no external dataset)",
        "config": {"workload": "256 systems, nx, ny in 16..96, nz in 8..32 (seeds 1000+s), 16-64 subdomains "
                               "each, two-level RAS, overlap 1, near 4^3, far 16^3, FP32 factors",
                   "cells": cells, "systems": len(specs)},
        "systems_per_s": round(len(specs) / t_batch, 1),
        "sequential_ms": round(t_seq * 1e3, 1), "speedup_vs_sequential": round(t_seq / t_batch, 2),
        "identical_to_sequential": identical, "converged": sum(i.status == P.OK for i in infos),
        "iters": {"min": min(iters), "median": int(np.median(iters)), "max": max(iters)},
        "setup_s": round(t_setup, 1),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-variants", action="store_true", help="headline only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--workload", choices=["solve1m", "batch256"], default="solve1m",
                    help="solve1m: the 1M-cell solve (default); batch256: 256 independent systems of "
                         "2k-295k cells solved as one batch, against solving them one after another")
    ap.add_argument("--counter-workload", choices=["apply", "copy"], default=None,
                    help="run only a short workload for hardware-counter collection: five preconditioner "
                         "applications of the benchmark configuration, or a plain 1 GiB device copy")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the solve of one "
                                   "system is not sharded across GPUs)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import gen
    import paper_1401_7227_amd as P

    torch.cuda.set_device(0)
    if args.workload == "batch256":
        print(json.dumps(bench_batch(P, gen, torch, np, args)))
        return
    if args.counter_workload == "copy":
        a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        for _ in range(5):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"counter_workload": "copy", "bytes_read_per_launch": COPY_BYTES,
                          "bytes_written_per_launch": COPY_BYTES, "launches": 5}))
        return
    s = gen.generate(*GRID, seed=SEED)
    N, n = s.N, s.n
    t0 = time.perf_counter()
    G = P.System.from_generated(s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    B = P.Precond(G, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, near=NEAR, far=FAR, **SPLIT)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st = B.stats()
    b = torch.from_numpy(s.b).cuda()
    if args.counter_workload == "apply":
        z = torch.empty_like(b)
        for _ in range(5):
            B.apply(b, out=z)
        torch.cuda.synchronize()
        print(json.dumps({"counter_workload": "apply", "launches": 5,
                          "alg_bytes_per_launch": ilu_apply_bytes(st, N)}))
        return

    # the sweep kernel (the dominant one) is timed by HIP events inside the
    # timed region; a further solve with every phase timed gives the
    # breakdown (events add a little time per launch)
    ms, info, prof, x = timed_solves(P, torch, G, B, b, args.steps, args.warmup, profile=["ilu_apply"])
    _, _, prof_all, _ = timed_solves(P, torch, G, B, b, 1, 0, profile=P.PHASES)
    phase = {k: {"launches": v[0], "ms_total": v[1], "ms_avg": v[1] / v[0] if v[0] else 0.0}
             for k, v in prof_all.items()}
    phase["ilu_apply"] = {"launches": prof["ilu_apply"][0], "ms_total": prof["ilu_apply"][1] / args.steps,
                          "ms_avg": prof["ilu_apply"][1] / max(prof["ilu_apply"][0], 1)}
    per_solve_launch = {k: float(v["launches"]) for k, v in phase.items()}
    per_solve_launch["ilu_apply"] = phase["ilu_apply"]["launches"] / args.steps
    dots_b, upd_b, nsteps = krylov_vector_bytes(n, info.iters, info.cycles, RESTART)
    alg = {
        "ilu_apply": ilu_apply_bytes(st, N),
        "spmv": spmv_bytes(s.nnzb, N),
        "dots": dots_b / nsteps,
        "update": upd_b / nsteps,
        "residual": spmv_bytes(s.nnzb, N) + 24 * N,
    }
    dominant = max(alg, key=lambda k: phase[k]["ms_total"])
    avg_ms = phase[dominant]["ms_avg"]
    achieved = alg[dominant] / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic() if dominant == "ilu_apply" else None
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else int(traffic),
                "alg_bytes_per_launch": int(alg[dominant]), "avg_launch_ms": round(avg_ms, 4)}
    # algorithmic bytes of the whole solve over the wall time
    total_bytes = (alg["ilu_apply"] * per_solve_launch["ilu_apply"] + alg["spmv"] * per_solve_launch["spmv"]
                   + dots_b + upd_b + alg["residual"] * per_solve_launch["residual"])

    out = {
        "metric": "ms/solve to rtol 1e-6 (1M cells), FP64 vs FP32-precond; served p50/p99 ms",
        "value": round(ms, 3), "unit": "ms/solve", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic (seeded generator, no external dataset)",
        "config": {"workload": "128x128x64 fully implicit 3x3-block Jacobian (1,048,576 cells, 3,145,728 "
                               "unknowns), two-level Schwarz RAS, 16x16 subdomains, overlap 1, near 4^3, far 16^3, "
                               "block ILU(0), GMRES(30) to rtol 1e-6",
                   "grid": list(GRID), "seed": SEED, "nnzb": s.nnzb, "parallelism": "single GPU"},
        "iters": info.iters, "rel_res_true": info.rel_res_true,
        "setup_ms": {"create_system": round((t1 - t0) * 1e3, 1), "setup_precond": round((t2 - t1) * 1e3, 1)},
        "precond": st,
        "phases": {k: {"launches_per_solve": per_solve_launch[k], "ms_avg": round(v["ms_avg"], 4),
                       "ms_per_solve": round(v["ms_total"], 3)} for k, v in phase.items()},
        "phases_note": "ilu_apply timed inside the timed region; other phases from one further solve "
                       "with every phase timed",
        "solve_alg_GBs": round(total_bytes / (ms * 1e-3) / 1e9, 1),
        "roofline": roofline,
    }
    if not args.no_variants:
        variants = {}
        x64 = x.cpu().numpy()
        B32 = P.Precond(G, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, near=NEAR, far=FAR, precision=P.FP32,
                        **SPLIT)
        ms32, info32, prof32, x32 = timed_solves(P, torch, G, B32, b, args.steps, args.warmup, profile=None)
        variants["two_level_fp32_factors"] = {
            "ms_per_solve": round(ms32, 3), "iters": info32.iters, "rel_res_true": info32.rel_res_true,
            "speedup_vs_fp64": round(ms / ms32, 3),
            "rel_err_vs_fp64_solution": float(np.linalg.norm(x32.cpu().numpy() - x64) / np.linalg.norm(x64))}
        del B32
        Bc = P.Precond(G, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, **SPLIT)
        msc, infoc, _, _ = timed_solves(P, torch, G, Bc, b, max(1, args.steps // 2), 1, profile=None)
        variants["classical_ras_fp64"] = {"ms_per_solve": round(msc, 3), "iters": infoc.iters,
                                          "rel_res_true": infoc.rel_res_true}
        del Bc
        out["variants"] = variants
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, info.iters, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
