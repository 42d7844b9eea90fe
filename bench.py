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
import re
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
TRAFFIC_FILE_FP32 = os.path.join(ROOT, "profiles", "ilu_apply_two_level_fp32_1M_traffic.json")
# Sources that decide what the sweep kernel reads and writes: the kernel
# itself and the host code that lays out its records.
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1401_7227_amd", "csrc", f)
                  for f in ("kernels.hip", "kernels.hpp", "plan.hpp", "setup.hpp", "setup.cpp")]
COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written per launch


def _code_only(text):
    """Source text without comments, trailing blanks and empty lines: an
    edit of the comments leaves the measured kernel what it was."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*$", "", line).rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line.strip())


def kernel_source_sha():
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per sweep launch from the committed counter runs (FETCH_SIZE
    and WRITE_SIZE per dispatch, each scaled by what the same counter reads
    for a copy of known size), or None if the kernel source changed since."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
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


def timed_solves(P, torch, G, B, b, steps, warmup, profile, graph=False):
    """Times `steps` solves; `profile` names the phases timed by HIP events
    inside the timed region (None: none); graph: restart cycles run as
    captured graphs (asm_solve_graph)."""
    x = torch.zeros_like(b)
    info = None
    for _ in range(warmup):
        x.zero_()
        _, info = P.solve(G, B, b, out=x, restart=RESTART, rtol=1e-6, max_iters=5000, graph=graph)
    G.profile(profile is not None, phases=profile)
    G.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    per = []
    for _ in range(steps):
        ts = time.perf_counter()
        x.zero_()
        _, info = P.solve(G, B, b, out=x, restart=RESTART, rtol=1e-6, max_iters=5000, graph=graph)  # synchronises
        per.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = G.profile_read(reset=True)
    G.profile(False)
    timed_solves.last_per_solve_ms = per
    return (t1 - t0) / steps * 1e3, info, prof, x


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, gpu_iters, budget_steps):
    """The CPU oracle (single thread, FP64) on a bounded sample of the same
    workload: the oracle's setup of the same preconditioner, then a fixed
    number of GMRES steps, scaled to one solve of the GPU's iteration count.
    The calling thread (the one the oracle runs on) is pinned to one core for
    the leg and released afterwards."""
    import oracle as O
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    os.sched_setaffinity(0, {core})
    try:
        A = O.Matrix.from_system(s)
        t0 = time.perf_counter()
        Bo = O.Precond(A, kind=O.KIND_TWO_LEVEL, combine=O.RESTRICTED, near=NEAR, far=FAR, **SPLIT)
        t1 = time.perf_counter()
        O.gmres(A, Bo, s.b, restart=RESTART, fixed_iters=budget_steps)
        t2 = time.perf_counter()
    finally:
        os.sched_setaffinity(0, set(allowed))
    per_step = (t2 - t1) / budget_steps
    return {"value": round(per_step * gpu_iters * 1e3, 1), "unit": "ms/solve", "cores": 1, "kind": "oracle",
            "sample": f"oracle setup ({t1 - t0:.1f} s, not in the metric) plus {budget_steps} GMRES steps "
                      f"({t2 - t1:.1f} s) of the same 1M-cell two-level solve, scaled to {gpu_iters} steps",
            "setup_s": round(t1 - t0, 2), "s_per_step": round(per_step, 3),
            "cpu_model": cpu_model(), "pinned_core": core, "host_cores": os.cpu_count(),
            "host_cores_allowed": len(allowed),
            "note": "single-threaded plain C (gcc -O2), pinned to one core with sched_setaffinity"}


def oracle_reference():
    """The FP64 oracle's two-level solution of the benchmark system, stored by
    tests/golden/make_config2_golden.py (which calls only the oracle): the
    iteration count and the solution on a fixed sample of unknowns."""
    path = os.path.join(ROOT, "tests", "golden", "config2_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    return d if "two_level_ras" in d else None


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
    order = P.batch_tuning_last()
    if args.batch_no_sequential:  # (a traced run: the batched solves only)
        seq, t_seq = None, float("nan")
        identical = None
    else:
        t0 = time.perf_counter()
        seq = [P.solve(G, B, b, **kw) for G, B, b in zip(systems, preconds, bs)]
        torch.cuda.synchronize()
        t_seq = time.perf_counter() - t0
        identical = all(bool(torch.equal(x, x1)) and i.iters == i1.iters
                        for x, i, (x1, i1) in zip(xs, infos, seq))
    iters = [i.iters for i in infos]
    return {
        "metric": "batch of 256 independent solves to rtol 1e-6 (FP32 preconditioner, FP64 GMRES(30))",
        "value": round(t_batch * 1e3, 1), "unit": "ms/batch", "higher_is_better": False, "n_gpus": 1,
        "dtype": "f64 (FP32 factors)", "data": "synthetic (seeded generator, no external dataset)",
        "config": {"workload": "256 systems, nx, ny in 16..96, nz in 8..32 (seeds 1000+s), 16-64 subdomains "
                               "each, two-level RAS, overlap 1, near 4^3, far 16^3, FP32 factors",
                   "cells": cells, "systems": len(specs)},
        "systems_per_s": round(len(specs) / t_batch, 1),
        "sequential_ms": None if seq is None else round(t_seq * 1e3, 1),
        "speedup_vs_sequential": None if seq is None else round(t_seq / t_batch, 2),
        "identical_to_sequential": identical, "converged": sum(i.status == P.OK for i in infos),
        "iters": {"min": min(iters), "median": int(np.median(iters)), "max": max(iters)},
        "setup_s": round(t_setup, 1),
        "batch_order": order,
        "tuning_by_size_class": tuning_classes(systems),
    }


def tuning_classes(systems):
    """The launch-shape choice of each size class among the systems (one
    representative per class)."""
    out = {}
    for G in systems:
        t = G.tuning()
        k = f"N<={1 << max(0, int(G.N - 1).bit_length())}"
        if k not in out:
            out[k] = {"spmv_rows": t["spmv_rows"], "red_blocks": t["red_blocks"], "source": t["source"]}
    return dict(sorted(out.items(), key=lambda kv: int(kv[0][3:])))


def bench_tuning(P, gen, torch, np, args):
    """The tuner's choice per size class: one system per class (grid 2nz x
    2nz x nz, classical RAS), timed on its first solve."""
    rows = []
    for nz in (6, 10, 16, 25, 40, 64):
        grid = (2 * nz, 2 * nz, nz)
        s = gen.generate(*grid, seed=7)
        G = P.System.from_generated(s)
        B = P.Precond(G, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, sx=4, sy=4, overlap=1)
        P.solve(G, B, torch.from_numpy(s.b).cuda(), restart=RESTART, fixed_iters=2)
        t = G.tuning()
        rows.append({"grid": list(grid), "block_rows": s.N, **t})
        del B, G
    return {"metric": "launch-shape tuner choices by size class", "restart": RESTART, "classes": rows}


def serve_trace(np, count=1000, rate=200.0, seed=5):
    """Requests of the serving workload: Poisson arrivals at `rate` per
    second; cells log-uniform in [1e4, 1e6], nz = round((cells/4)^(1/3)),
    nx = ny = 2 nz; 1-3 solves each (the Newton iterations of one time step:
    new values on the same pattern); seed 5 for the trace, request r draws
    its system from seed 50000 + r."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    cells = np.exp(rng.uniform(np.log(1e4), np.log(1e6), count))
    nsolves = rng.integers(1, 4, count)
    out = []
    for r in range(count):
        nz = int(round((cells[r] / 4.0) ** (1.0 / 3.0)))
        out.append({"t": float(t[r]), "grid": (2 * nz, 2 * nz, nz), "nsolves": int(nsolves[r]),
                    "seed": 50000 + r})
    return out


def serve_split(nx, ny, nz):
    """Subdomains: clamp(round(cells/4096), 16, 64), split in proportion to nx:ny."""
    cells = nx * ny * nz
    nsub = int(min(64, max(16, round(cells / 4096))))
    sx = max(1, min(nx, int(round((nsub * nx / ny) ** 0.5))))
    sy = max(1, min(ny, int(round(nsub / sx))))
    return sx, sy


class ServeInputs:
    """Draws a request's systems on the device when it arrives (the
    Jacobian assembly of the simulator that sends it).  Patterns are shared
    per grid."""

    def __init__(self, torch):
        from gen import device as gd
        self.gd, self.torch, self.patterns = gd, torch, {}

    def pattern(self, grid):
        if grid not in self.patterns:
            self.patterns[grid] = self.gd.pattern(*grid, "cuda")
        return self.patterns[grid]

    def draw(self, req):
        grid = req["grid"]
        rp, ci = self.pattern(grid)
        perm = self.gd.draw_perm(*grid, req["seed"], "cuda")
        vals, bs, xs = [], [], []
        for k in range(req["nsolves"]):
            v, b, _ = self.gd.draw_values(*grid, perm, req["seed"] * 10 + k)
            vals.append(v.reshape(-1))
            bs.append(b)
            xs.append(self.torch.zeros_like(b))
        return rp, ci, vals, bs, xs


def serve_popts(P, grid, precision):
    sx, sy = serve_split(*grid)
    return dict(kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, sx=sx, sy=sy, overlap=1, near=NEAR, far=FAR,
                precision=precision)


def percentiles(np, lat):
    a = np.asarray(lat) * 1e3
    return {"p50_ms": round(float(np.percentile(a, 50)), 1), "p99_ms": round(float(np.percentile(a, 99)), 1),
            "mean_ms": round(float(a.mean()), 1), "max_ms": round(float(a.max()), 1)}


def run_server(P, torch, np, trace, precision, budget, max_active, label):
    """Replays the trace in real time against the library's request server.
    Arrived requests wait in a front queue and are drawn and submitted while
    the server's own queue is short (inputs of queued requests are not held
    on the device for long); latency counts from the arrival time."""
    from collections import deque
    inputs = ServeInputs(torch)
    srv = P.Server(restart=RESTART, rtol=1e-6, max_iters=5000, budget_bytes=budget, max_active=max_active)
    n = len(trace)
    front, done, arrived = deque(), {}, 0
    running_sum, polls, status = 0, 0, {}
    busy_s, tprev, busy = 0.0, 0.0, False  # time with a request queued or in flight
    t0 = time.perf_counter()
    last = t0
    while len(done) < n:
        now = time.perf_counter() - t0
        if busy:
            busy_s += now - tprev
        tprev = now
        while arrived < n and trace[arrived]["t"] <= now:
            front.append(arrived)
            arrived += 1
        st = srv.state()
        while front and st["queued"] < 4:
            r = front.popleft()
            rp, ci, vals, bs, xs = inputs.draw(trace[r])
            srv.submit(r, trace[r]["grid"], rp, ci, P.precond_opts(**serve_popts(P, trace[r]["grid"], precision)),
                       vals, bs, xs)
            st["queued"] += 1
        if st["running"] == 0 and st["queued"] == 0 and not front and arrived < n:
            busy = False
            time.sleep(max(0.0, trace[arrived]["t"] - (time.perf_counter() - t0)))
            continue
        for c in srv.poll():
            done[c["tag"]] = (time.perf_counter() - t0, c)
            status[c["status"]] = status.get(c["status"], 0) + 1
        st = srv.state()
        running_sum += st["running"]
        busy = st["running"] > 0 or st["queued"] > 0 or bool(front)
        polls += 1
        if time.perf_counter() - last > 15.0:
            last = time.perf_counter()
            print(f"[serve {label}] t={last - t0:.1f}s done {len(done)}/{n} arrived {arrived} "
                  f"state {srv.state()}", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
    wall = time.perf_counter() - t0
    st = srv.state()
    srv.close()
    lat = [done[r][0] - trace[r]["t"] for r in range(n)]
    cells = sum(trace[r]["grid"][0] * trace[r]["grid"][1] * trace[r]["grid"][2] * trace[r]["nsolves"]
                for r in range(n))
    out = percentiles(np, lat)
    out.update({"requests": n, "wall_s": round(wall, 2), "requests_per_s": round(n / wall, 2),
                "solves_per_s": round(sum(t["nsolves"] for t in trace) / wall, 2),
                "cell_solves_per_s": round(cells / wall, 0),
                "mean_running": round(running_sum / max(polls, 1), 1), "polls": polls,
                "busy_frac": round(busy_s / wall, 3),
                "plan_builds": st["plan_builds"], "plan_hits": st["plan_hits"],
                "statuses": {str(k): v for k, v in status.items()},
                "iters_total": sum(done[r][1]["iters"] for r in range(n))})
    return out


def run_fifo(P, torch, np, trace, label):
    """The same trace served one request at a time, in arrival order, with
    the plain calls and an FP64 preconditioner set up for each request."""
    inputs = ServeInputs(torch)
    n = len(trace)
    lat, status, iters = [], {}, 0
    t0 = time.perf_counter()
    last = t0
    for r in range(n):
        now = time.perf_counter() - t0
        if trace[r]["t"] > now:
            time.sleep(trace[r]["t"] - now)
        rp, ci, vals, bs, xs = inputs.draw(trace[r])
        grid = trace[r]["grid"]
        st = P.OK
        try:
            G = P.System(*grid, rp, ci, vals[0])
            B = P.Precond(G, **serve_popts(P, grid, P.FP64))
            for k in range(trace[r]["nsolves"]):
                if k > 0:
                    G.update_values(vals[k])
                    B.refactor()
                _, info = P.solve(G, B, bs[k], restart=RESTART, rtol=1e-6, max_iters=5000, out=xs[k])
                iters += info.iters
                st = min(st, info.status) if info.status < 0 else max(st, info.status)
            B.close()
            G.close()
        except P.AsmError as e:
            st = e.status
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - trace[r]["t"])
        status[st] = status.get(st, 0) + 1
        if time.perf_counter() - last > 15.0:
            last = time.perf_counter()
            print(f"[fifo {label}] t={last - t0:.1f}s done {r + 1}/{n}", file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    out = percentiles(np, lat)
    out.update({"requests": n, "wall_s": round(wall, 2), "requests_per_s": round(n / wall, 2),
                "statuses": {str(k): v for k, v in status.items()}, "iters_total": iters})
    return out


def bench_serve(P, gen, torch, np, args):
    trace = serve_trace(np, count=args.serve_requests, rate=args.serve_rate)
    budget = int(args.serve_budget_gib * (1 << 30))
    prefix = trace[:args.serve_compare]
    # warm-up: one small request through both paths (library load, kernels)
    warm = [{"t": 0.0, "grid": (28, 28, 14), "nsolves": 1, "seed": 1}]
    run_server(P, torch, np, warm, P.FP32, budget, args.serve_max_active, "warm-up")
    run_fifo(P, torch, np, warm, "warm-up")
    full = run_server(P, torch, np, trace, P.FP32, budget, args.serve_max_active, "full")
    torch.cuda.empty_cache()
    if len(prefix) < len(trace):
        srv_prefix = run_server(P, torch, np, prefix, P.FP32, budget, args.serve_max_active, "prefix")
        torch.cuda.empty_cache()
    else:  # the comparison covers the whole trace
        srv_prefix = full
    fifo_prefix = run_fifo(P, torch, np, prefix, "prefix" if len(prefix) < len(trace) else "full")
    cells = np.array([t["grid"][0] * t["grid"][1] * t["grid"][2] for t in trace])
    offered = float(np.sum(cells * np.array([t["nsolves"] for t in trace]))) / trace[-1]["t"]
    return {
        "metric": f"served latency p50/p99 ms (Poisson arrivals {args.serve_rate:g}/s, 1e4-1e6 cells, 1-3 solves "
                  "per request)",
        "value": full["p99_ms"], "unit": "ms (p99)", "higher_is_better": False, "n_gpus": 1,
        "dtype": "f64 (FP32 factors)", "data": "synthetic (seeded generator drawn on the device at arrival)",
        "config": {"workload": f"{len(trace)} requests, Poisson arrivals at {args.serve_rate:g}/s (trace seed 5), cells "
                               "log-uniform in [1e4, 1e6], grid 2nz x 2nz x nz, 1-3 solves each with new values "
                               "on the same pattern; two-level RAS, overlap 1, near 4^3, far 16^3, 16-64 "
                               "subdomains, FP32 factors, GMRES(30) to rtol 1e-6",
                   "hbm_budget_gib": args.serve_budget_gib, "max_active": args.serve_max_active},
        "p50_ms": full["p50_ms"], "p99_ms": full["p99_ms"],
        "offered_cell_solves_per_s": round(offered, 0),
        "offered_over_served": round(offered / full["cell_solves_per_s"], 3),
        "arrival_span_s": round(trace[-1]["t"], 2),
        "server_full_trace": full,
        "utilisation": {"server_busy_frac": full["busy_frac"],
                        "offered_over_saturated_capacity": round(offered / args.serve_capacity, 3),
                        "saturated_capacity_cell_solves_per_s": args.serve_capacity,
                        "run_length_s": full["wall_s"]},
        "prefix_comparison": {"requests": len(prefix), "server_fp32": srv_prefix, "fifo_fp64": fifo_prefix,
                              "p50_speedup": round(fifo_prefix["p50_ms"] / srv_prefix["p50_ms"], 2),
                              "p99_speedup": round(fifo_prefix["p99_ms"] / srv_prefix["p99_ms"], 2)},
    }


def bench_serve_leg(P, torch, np, args):
    """The served form inside the default benchmark: a prefix of the serving
    trace (same seed and mix: 1e4-1e6 cells, 1-3 solves per request) at an
    arrival rate one GPU sustains, through the request server with FP32
    factors, against the same requests solved one at a time with FP64
    factors and the plain calls."""
    trace = serve_trace(np, count=args.serve_leg_requests, rate=args.serve_leg_rate)
    budget = int(args.serve_budget_gib * (1 << 30))
    warm = [{"t": 0.0, "grid": (28, 28, 14), "nsolves": 1, "seed": 1}]
    run_server(P, torch, np, warm, P.FP32, budget, args.serve_max_active, "warm-up")
    run_fifo(P, torch, np, warm, "warm-up")
    srv = run_server(P, torch, np, trace, P.FP32, budget, args.serve_max_active, "leg")
    torch.cuda.empty_cache()
    fifo = run_fifo(P, torch, np, trace, "leg")
    torch.cuda.empty_cache()
    cells = np.array([t["grid"][0] * t["grid"][1] * t["grid"][2] * t["nsolves"] for t in trace], dtype=float)
    span = trace[-1]["t"]
    return {"workload": f"first {len(trace)} requests of the serving trace (seed 5) at {args.serve_leg_rate}/s "
                        "Poisson arrivals",
            "offered_cell_solves_per_s": round(float(cells.sum()) / span, 0),
            "server_fp32": {k: srv[k] for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "wall_s",
                                                "requests_per_s", "cell_solves_per_s", "mean_running",
                                                "busy_frac", "statuses")},
            "fifo_fp64": {k: fifo[k] for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "wall_s", "requests_per_s",
                                               "statuses")},
            "p50_speedup": round(fifo["p50_ms"] / srv["p50_ms"], 2),
            "p99_speedup": round(fifo["p99_ms"] / srv["p99_ms"], 2)}


def bench_comparators(P, gen, torch, np, args):
    """The comparisons of Section 5 on synthetic stand-ins: iteration counts
    against the number of subdomains K and the coarsening size C for the
    near field only, the far field only and both (near boxes C, far boxes
    2C), the far field against the classical two-level Schwarz method
    (eq. (3.5)) and the two-stage method (eq. (3.8)) with coarse boxes C,
    and the far field with one- and two-dimensional splits.  No overlap,
    exact (dense) or ILU(0) local solves, GMRES(30) to rtol 1e-6."""
    def run(s, G, b, **o):
        try:
            B = P.Precond(G, **o)
        except P.AsmError as e:
            return {"error": str(e).split(":")[0]}
        st = B.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = P.solve(G, B, b, restart=RESTART, rtol=1e-6, max_iters=3000)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        return {"iters": info.iters if info.status == P.OK else None, "ms": round(ms, 2),
                "rows_per_sub": round(st["ext_rows"] / st["nsub"], 1),
                "blocks_per_sub": round(st["factor_blocks"] / st["nsub"], 1)}

    out = {"metric": "GMRES iterations to rtol 1e-6 for the preconditioners compared in Section 5",
           "unit": "iterations", "higher_is_better": False, "n_gpus": 1, "dtype": "f64",
           "data": "synthetic (seeded generator, no external dataset)"}
    # Figs. 5 and 6: 21x21x5 (the grid size of the ORSREG1 benchmark), x split
    s = gen.generate(21, 21, 5, seed=1)
    G = P.System.from_generated(s)
    b = torch.from_numpy(s.b).cuda()
    fields = {"near": P.FIELD_NEAR, "far": P.FIELD_FAR, "near_far": P.FIELD_NEAR_FAR}
    fig5, fig6 = [], []
    for local_name, local in [("exact", P.LOCAL_EXACT), ("ilu0", P.LOCAL_ILU0)]:
        for K in (2, 3, 5, 7):
            for C in (2, 3, 4, 5):
                row = {"local": local_name, "K": K, "C": C}
                for name, f in fields.items():
                    row[name] = run(s, G, b, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, sx=K, sy=1, overlap=0,
                                    near=(C, C, C), far=(2 * C, 2 * C, 2 * C) if f == P.FIELD_NEAR_FAR else (C, C, C),
                                    field=f, local=local)
                fig5.append(row)
                row6 = {"local": local_name, "K": K, "C": C, "far": row["far"]}
                row6["two_level_3_5"] = run(s, G, b, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, sx=K, sy=1,
                                            overlap=0, coarse=P.COARSE_ADDITIVE, cbox=(C, C, C), local=local)
                row6["two_stage_3_8"] = run(s, G, b, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, sx=K, sy=1,
                                            overlap=0, coarse=P.COARSE_TWO_STAGE, cbox=(C, C, C), local=local)
                fig6.append(row6)
            row0 = run(s, G, b, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, sx=K, sy=1, overlap=0, local=local)
            fig5.append({"local": local_name, "K": K, "C": None, "classical_ras": row0})
            print(f"[comparators] 21x21x5 {local_name} K={K} done", file=sys.stderr, flush=True)
    out["fig5_near_far_21x21x5"] = fig5
    out["fig6_coarse_21x21x5"] = fig6
    # Fig. 9: 30x30x9, far field, 1-D (K x 1) against 2-D splits
    s = gen.generate(30, 30, 9, seed=2)
    G = P.System.from_generated(s)
    b = torch.from_numpy(s.b).cuda()
    fig9 = []
    for K, split2 in ((4, (2, 2)), (9, (3, 3)), (16, (4, 4))):
        for C in (2, 3, 5):
            for local_name, local in [("exact", P.LOCAL_EXACT), ("ilu0", P.LOCAL_ILU0)]:
                common = dict(kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, overlap=0, near=(C, C, C), far=(C, C, C),
                              field=P.FIELD_FAR, local=local)
                fig9.append({"local": local_name, "K": K, "C": C,
                             "split_1d": run(s, G, b, sx=K, sy=1, **common),
                             "split_2d": run(s, G, b, sx=split2[0], sy=split2[1], **common)})
        print(f"[comparators] 30x30x9 K={K} done", file=sys.stderr, flush=True)
    out["fig9_splits_30x30x9"] = fig9
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-variants", action="store_true", help="headline only")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--workload", choices=["solve1m", "batch256", "serve", "comparators", "tuning"],
                    default="solve1m",
                    help="solve1m: the 1M-cell solve (default); batch256: 256 independent systems of "
                         "2k-295k cells solved as one batch, against solving them one after another; "
                         "serve: a Poisson request trace against the request server, and a prefix of it "
                         "against one-at-a-time FP64 solves; comparators: the iteration-count studies of "
                         "the paper's Section 5 on synthetic systems")
    ap.add_argument("--no-serve", action="store_true", help="no served leg in the default benchmark")
    ap.add_argument("--batch-no-sequential", action="store_true",
                    help="batch256: skip the one-after-another comparison (for traced runs)")
    ap.add_argument("--serve-leg-requests", type=int, default=40)
    ap.add_argument("--serve-leg-rate", type=float, default=4.0,
                    help="arrivals per second of the served leg (one GPU sustains the trace's mix at this rate)")
    ap.add_argument("--serve-rate", type=float, default=200.0, help="arrival rate of --workload serve")
    ap.add_argument("--serve-capacity", type=float, default=5.26e6,
                    help="saturated server throughput (cell-solves/s, from the 200/s run) the offered load is "
                         "stated against")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--serve-compare", type=int, default=100, help="trace prefix for the FIFO comparison")
    ap.add_argument("--serve-budget-gib", type=float, default=128.0)
    ap.add_argument("--serve-max-active", type=int, default=256)
    ap.add_argument("--counter-precision", choices=["fp64", "fp32"], default="fp64",
                    help="factor precision of --counter-workload apply")
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
    if args.workload == "tuning":
        print(json.dumps(bench_tuning(P, gen, torch, np, args)))
        return
    if args.workload == "batch256":
        print(json.dumps(bench_batch(P, gen, torch, np, args)))
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(P, gen, torch, np, args)))
        return
    if args.workload == "comparators":
        print(json.dumps(bench_comparators(P, gen, torch, np, args)))
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
        fp32 = args.counter_precision == "fp32"
        if fp32:
            del B
            B = P.Precond(G, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, near=NEAR, far=FAR, precision=P.FP32,
                          **SPLIT)
            st = B.stats()
        z = torch.empty_like(b)
        for _ in range(5):
            B.apply(b, out=z)
        torch.cuda.synchronize()
        print(json.dumps({"counter_workload": "apply", "precision": args.counter_precision, "launches": 5,
                          "alg_bytes_per_launch": ilu_apply_bytes(st, N, fp32=fp32)}))
        return

    # the headline: solves with nothing else on the stream.  The sweep kernel
    # (the dominant one) is then timed by HIP events on its stream over
    # further timed solves (each event pair adds a few microseconds per
    # launch, so those solves are reported beside the headline, not as it),
    # and one more solve with every phase timed gives the breakdown.
    ms, info, _, x = timed_solves(P, torch, G, B, b, args.steps, args.warmup, profile=None)
    per_solve = list(timed_solves.last_per_solve_ms)
    psteps = max(2, args.steps // 2)
    ms_ev, _, prof, _ = timed_solves(P, torch, G, B, b, psteps, 0, profile=["ilu_apply"])
    _, _, prof_all, _ = timed_solves(P, torch, G, B, b, 1, 0, profile=P.PHASES)
    phase = {k: {"launches": v[0], "ms_total": v[1], "ms_avg": v[1] / v[0] if v[0] else 0.0}
             for k, v in prof_all.items()}
    phase["ilu_apply"] = {"launches": prof["ilu_apply"][0], "ms_total": prof["ilu_apply"][1] / psteps,
                          "ms_avg": prof["ilu_apply"][1] / max(prof["ilu_apply"][0], 1)}
    per_solve_launch = {k: float(v["launches"]) for k, v in phase.items()}
    per_solve_launch["ilu_apply"] = phase["ilu_apply"]["launches"] / psteps
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
        "ms_median": round(float(np.median(per_solve)), 3),
        "ms_per_solve_each": [round(v, 3) for v in per_solve],
        "iters": info.iters, "rel_res_true": info.rel_res_true,
        "setup_ms": {"create_system": round((t1 - t0) * 1e3, 1), "setup_precond": round((t2 - t1) * 1e3, 1)},
        "precond": st,
        "phases": {k: {"launches_per_solve": per_solve_launch[k], "ms_avg": round(v["ms_avg"], 4),
                       "ms_per_solve": round(v["ms_total"], 3)} for k, v in phase.items()},
        "phases_note": f"ilu_apply timed by HIP events on its stream over {psteps} further timed solves "
                       f"({round(ms_ev, 3)} ms per solve with those events); other phases from one more solve "
                       "with every phase timed",
        "solve_alg_GBs": round(total_bytes / (ms * 1e-3) / 1e9, 1),
        "roofline": roofline,
        "tuning": G.tuning(),
    }
    if not args.no_variants:
        variants = {}
        x64 = x.cpu().numpy()
        # the same solve with every restart cycle one captured graph
        msg, infog, _, xg = timed_solves(P, torch, G, B, b, max(1, args.steps // 2), 1, profile=None, graph=True)
        variants["two_level_fp64_graph_cycles"] = {
            "ms_per_solve": round(msg, 3), "iters": infog.iters, "rel_res_true": infog.rel_res_true,
            "rel_diff_vs_host_loop_solution": float(np.linalg.norm(xg.cpu().numpy() - x64) / np.linalg.norm(x64))}
        B32 = P.Precond(G, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, near=NEAR, far=FAR, precision=P.FP32,
                        **SPLIT)
        st32 = B32.stats()
        ms32, info32, _, x32 = timed_solves(P, torch, G, B32, b, args.steps, args.warmup, profile=None)
        _, _, prof32, _ = timed_solves(P, torch, G, B32, b, psteps, 0, profile=["ilu_apply"])
        a32 = prof32["ilu_apply"][1] / max(prof32["ilu_apply"][0], 1)
        alg32 = ilu_apply_bytes(st32, N, fp32=True)
        v32 = {
            "ms_per_solve": round(ms32, 3), "iters": info32.iters, "rel_res_true": info32.rel_res_true,
            "speedup_vs_fp64": round(ms / ms32, 3),
            "rel_err_vs_fp64_solution": float(np.linalg.norm(x32.cpu().numpy() - x64) / np.linalg.norm(x64)),
            "roofline": {"bound": "hbm", "kernel": "ilu_apply (FP32 fine-row factors)",
                         "achieved": round(alg32 / (a32 * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(alg32 / (a32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "traffic": (lambda t: None if t is None else int(t))(measured_traffic(TRAFFIC_FILE_FP32)),
                         "alg_bytes_per_launch": int(alg32), "avg_launch_ms": round(a32, 4)}}
        ref = oracle_reference()
        if ref is not None:
            # against the FP64 oracle at the oracle's own iteration count
            g = ref["two_level_ras"]
            xf, _ = P.solve(G, B32, b, restart=RESTART, fixed_iters=g["iters"])
            idx = np.array(ref["sample"])
            xs, xr = xf.cpu().numpy()[idx], np.array(g["x_sample"])
            v32["rel_err_vs_oracle"] = float(np.linalg.norm(xs - xr) / np.linalg.norm(xr))
            v32["oracle_iters"] = g["iters"]
            v32["rel_err_vs_oracle_note"] = (f"at the oracle's {g['iters']} iterations, on its stored sample of "
                                             f"{len(idx)} unknowns (tests/golden/config2_oracle.json)")
            del xf
        variants["two_level_fp32_factors"] = v32
        del B32
        Bc = P.Precond(G, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, **SPLIT)
        msc, infoc, _, _ = timed_solves(P, torch, G, Bc, b, max(1, args.steps // 2), 1, profile=None)
        variants["classical_ras_fp64"] = {"ms_per_solve": round(msc, 3), "iters": infoc.iters,
                                          "rel_res_true": infoc.rel_res_true}
        del Bc
        # classical additive Schwarz (eq. (3.3): overlapping contributions summed)
        Ba = P.Precond(G, kind=P.KIND_CLASSICAL, combine=P.ADDITIVE, **SPLIT)
        msa, infoa, _, _ = timed_solves(P, torch, G, Ba, b, max(1, args.steps // 4), 1, profile=None)
        variants["classical_additive_fp64"] = {"ms_per_solve": round(msa, 3), "iters": infoa.iters,
                                               "rel_res_true": infoa.rel_res_true}
        del Ba
        # the two-stage global coarse-grid comparator (eq. (3.8)), coarse boxes 16^3
        Bt = P.Precond(G, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, coarse=P.COARSE_TWO_STAGE,
                       cbox=(16, 16, 16), **SPLIT)
        mst, infot, _, _ = timed_solves(P, torch, G, Bt, b, max(1, args.steps // 2), 1, profile=None)
        variants["classical_ras_two_stage_coarse16_fp64"] = {"ms_per_solve": round(mst, 3), "iters": infot.iters,
                                                             "rel_res_true": infot.rel_res_true}
        del Bt
        out["variants"] = variants
    if not args.no_serve:
        del G, B
        torch.cuda.empty_cache()
        out["served"] = bench_serve_leg(P, torch, np, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, info.iters, args.cpu_steps)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
