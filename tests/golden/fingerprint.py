"""Per-subdomain fingerprints of a solution vector (test infrastructure).

A full 128x128x64 vector (3,145,728 doubles) is too large to store beside
the tests, and a sample of unknowns misses an error confined to a few
subdomains.  This file condenses a vector into, for each owned column block
of the sx x sy split (the cells a subdomain owns: its x-y tile, all of z):

  * norm  - the 2-norm of the block's unknowns,
  * sum   - the sum of each of the three components (p, So, Sg),
  * proj  - two projections on seeded N(0, 1) weight vectors.

If v and v_ref differ by d, the differences of these numbers are bounded by
the block's ||d||: |dnorm| <= ||d||, |dsum_k| <= sqrt(cells) ||d||, and each
projection difference is N(0, ||d||^2)-distributed over the weights, so a
check of all of them at a tolerance of tol * ||v_ref block|| (times the
stated factor) fails when any block's relative error is much above tol.
It computes nothing of the method: no oracle or library code is used.
"""
from __future__ import annotations

import numpy as np

WEIGHT_SEED = 7001
NPROJ = 4


def _split(n: int, k: int) -> np.ndarray:
    """Owner part of each of n columns in a balanced split into k parts
    (the first n mod k parts get one extra column)."""
    base, extra = divmod(n, k)
    sizes = [base + (1 if i < extra else 0) for i in range(k)]
    return np.repeat(np.arange(k), sizes)


def groups(grid, sx: int, sy: int) -> np.ndarray:
    """Block index (bx * sy + by) of every cell, cell c = (ix*ny + iy)*nz + iz."""
    nx, ny, nz = grid
    gx, gy = _split(nx, sx), _split(ny, sy)
    g2 = gx[:, None] * sy + gy[None, :]
    return np.repeat(g2.reshape(-1), nz)


def weights(n: int) -> np.ndarray:
    return np.random.default_rng(WEIGHT_SEED).standard_normal((NPROJ, n))


def fingerprint(v: np.ndarray, grid, sx: int, sy: int, W: np.ndarray | None = None) -> dict:
    v = np.asarray(v, dtype=np.float64)
    g = groups(grid, sx, sy)
    ng = sx * sy
    gu = np.repeat(g, 3)  # group of every unknown
    if W is None:
        W = weights(v.size)
    norm = np.sqrt(np.bincount(gu, weights=v * v, minlength=ng))
    v3 = v.reshape(-1, 3)
    sums = np.stack([np.bincount(g, weights=v3[:, k], minlength=ng) for k in range(3)], axis=1)
    proj = np.stack([np.bincount(gu, weights=W[p] * v, minlength=ng) for p in range(W.shape[0])], axis=1)
    cells = np.bincount(g, minlength=ng)
    return dict(norm=norm.tolist(), sum=sums.tolist(), proj=proj.tolist(), cells=cells.tolist())


def compare(fp: dict, ref: dict, tol: float) -> tuple[float, int]:
    """Largest violation ratio (> 1 means a failure) and the block it is in.
    Each difference is divided by its bound at relative error tol."""
    nr = np.asarray(ref["norm"])
    cells = np.asarray(ref["cells"], dtype=np.float64)
    bound = tol * np.maximum(nr, 1e-300)
    r_norm = np.abs(np.asarray(fp["norm"]) - nr) / bound
    r_sum = (np.abs(np.asarray(fp["sum"]) - np.asarray(ref["sum"])).max(axis=1)
             / (np.sqrt(cells) * bound))
    # a projection difference is N(0, ||d||^2): 8 standard deviations
    r_proj = np.abs(np.asarray(fp["proj"]) - np.asarray(ref["proj"])).max(axis=1) / (8.0 * bound)
    worst = np.maximum(np.maximum(r_norm, r_sum), r_proj)
    i = int(np.argmax(worst))
    return float(worst[i]), i
