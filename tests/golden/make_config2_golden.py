"""Writes oracle results for the 128x128x64 (1,048,576-cell) system.

Calls only the CPU oracle on the seeded generator's input (seed 2, 16x16
subdomains of 8x8x64, overlap 1, GMRES(30) to rtol 1e-6).  For each
preconditioner it stores the iteration count, the true relative residual,
the solution at a fixed sample of unknowns and its per-subdomain
fingerprint (fingerprint.py: norm, component sums and seeded projections of
every owned 8x8x64 column block), so that the GPU tests can compare every
subdomain at equal iteration counts without re-running the oracle.  With
--apply it stores instead, for every variant, one application z = B^-1 b of
the preconditioner (the same sample of z, its norm and its fingerprint): the check of the
Schwarz apply alone at full size, additive combine included.

Usage: python tests/golden/make_config2_golden.py [--apply] [variant ...]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle as O  # noqa: E402
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from fingerprint import fingerprint  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_oracle.json")
GRID, SEED = (128, 128, 64), 2
SPLIT = dict(sx=16, sy=16, overlap=1)
NEAR, FAR = (4, 4, 4), (16, 16, 16)
VARIANTS = {
    "classical_ras": dict(kind=O.KIND_CLASSICAL, combine=O.RESTRICTED),
    "two_level_ras": dict(kind=O.KIND_TWO_LEVEL, combine=O.RESTRICTED),
    "classical_additive": dict(kind=O.KIND_CLASSICAL, combine=O.ADDITIVE),
}
NSAMPLE = 512


def main(names):
    s = gen.generate(*GRID, seed=SEED)
    A = O.Matrix.from_system(s)
    sample = np.sort(np.random.default_rng(12345).choice(s.n, NSAMPLE, replace=False))
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    data["grid"], data["seed"], data["sample"] = list(GRID), SEED, sample.tolist()
    for name in names:
        kw = VARIANTS[name]
        t0 = time.perf_counter()
        P = O.Precond(A, near=NEAR, far=FAR, **SPLIT, **kw)
        t1 = time.perf_counter()
        res = O.gmres(A, P, s.b, restart=30, rtol=1e-6, max_iters=3000)
        t2 = time.perf_counter()
        data[name] = dict(status=res.status, iters=res.iters, cycles=res.cycles,
                          rel_res_true=res.rel_res_true, x_norm=float(np.linalg.norm(res.x)),
                          x_sample=res.x[sample].tolist(),
                          x_fp=fingerprint(res.x, GRID, SPLIT["sx"], SPLIT["sy"]),
                          setup_s=t1 - t0, solve_s=t2 - t1,
                          near=list(NEAR), far=list(FAR), **SPLIT)
        print(name, res.status, res.iters, res.rel_res_true, f"setup {t1 - t0:.1f}s solve {t2 - t1:.1f}s",
              flush=True)
        json.dump(data, open(OUT, "w"), indent=1)


def main_apply(names):
    s = gen.generate(*GRID, seed=SEED)
    A = O.Matrix.from_system(s)
    data = json.load(open(OUT))
    sample = np.array(data["sample"])
    app = data.setdefault("apply", {})
    for name in names:
        t0 = time.perf_counter()
        P = O.Precond(A, near=NEAR, far=FAR, **SPLIT, **VARIANTS[name])
        z = P.apply(s.b)
        app[name] = dict(r="b", z_norm=float(np.linalg.norm(z)), z_sample=z[sample].tolist(),
                         z_fp=fingerprint(z, GRID, SPLIT["sx"], SPLIT["sy"]))
        print(name, "apply", f"{time.perf_counter() - t0:.1f}s", flush=True)
        json.dump(data, open(OUT, "w"), indent=1)


if __name__ == "__main__":
    args = sys.argv[1:]
    if args and args[0] == "--apply":
        main_apply(args[1:] or list(VARIANTS))
    else:
        main(args or list(VARIANTS))
