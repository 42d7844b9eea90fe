"""Seeded synthetic fully implicit black-oil Jacobians (test and benchmark input).

This module only *draws inputs*: a block-sparse matrix A (= -J, the sign
convention of the linear problem r = b - Ax stated in Section 2) with dense
3x3 blocks on a Cartesian grid, and a right-hand side b.  It contains none of
the solver's arithmetic (no partitioning, no lumping, no factorisation, no
Krylov step) and is shared by the CPU oracle and the GPU path as their common
input.

The paper's own matrices (ORSREG1, the SPE1 variants of Table 1) are not
available; this generator stands in for them with the same traits: a
7-point finite-volume stencil, 3 unknowns per cell (pressure, oil saturation,
gas saturation; Section 1 describes the 3-component sub-vectors and 3x3
sub-matrices), and the strong vertical coupling described in Section 2.

Recipe (fixed draw order from one ``numpy.random.Generator(PCG64(seed))``):

1. permeability ``k[N] = exp(mu + sigma * N(0,1))``;
2. upwind potential ``phi[N] ~ N(0,1)``;
3. face mobilities ``M[F,3,3] ~ U(0.1, 1)``; faces are listed as x-faces,
   then y-faces, then z-faces, each in increasing order of the lower cell;
4. accumulation ``U(1e-3,1e-2)`` for p, then ``U(1,2)`` for So, then
   ``U(1,2)`` for Sg, each an [N] array;
5. right-hand side ``b[3N] ~ N(0,1)``.

Face transmissibility is the harmonic mean ``2 k_i k_j / (k_i + k_j)``,
multiplied by 10 on z-faces (vertical transmissibility 10x horizontal).
Each mobility matrix gets a dominant pressure column
(``M[r,0] += M[r,1] + M[r,2]``).  Upwinding: the cell with the larger
potential is upstream u (ties go to the lower cell), the other is downstream
d; then ``A[d,u] = -T M`` and ``A[u,d] = -T M`` with its saturation columns
zeroed (the upstream equation sees only the downstream pressure).

Diagonal blocks: the pressure column is minus the block column sum of the
off-diagonal pressure columns, each saturation diagonal entry is minus the
scalar column sum of that saturation column over the off-diagonal blocks,
other saturation entries are zero, and ``diag(acc)`` is added.  Hence every
scalar column sum of A equals the accumulation of that unknown, the
material-balance structure that Section 2 ties to zero column sums of the
error matrix.

Cell ordering: ``c = (ix*ny + iy)*nz + iz`` (z fastest), unknown ``3c + v``
with v = 0 (p), 1 (So), 2 (Sg).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Neighbour slots of a block row, in increasing column order.
SLOT_XM, SLOT_YM, SLOT_ZM, SLOT_DIAG, SLOT_ZP, SLOT_YP, SLOT_XP = range(7)


@dataclass
class System:
    """A generated linear system A x = b in BSR form (3x3 blocks)."""

    nx: int
    ny: int
    nz: int
    row_ptr: np.ndarray  # int32 [N+1]
    col_idx: np.ndarray  # int32 [nnzb]
    vals: np.ndarray  # float64 [nnzb, 3, 3], row-major blocks
    b: np.ndarray  # float64 [3N]
    acc: np.ndarray  # float64 [N, 3] accumulation per unknown
    perm: np.ndarray  # float64 [N] permeability
    seed: int

    @property
    def N(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n(self) -> int:
        return 3 * self.N

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def contrast_decades(self) -> float:
        return float(np.log10(self.perm.max() / self.perm.min()))

    def dense(self) -> np.ndarray:
        """Dense scalar matrix (small systems only)."""
        n = self.n
        if n > 20000:
            raise ValueError("dense() is for small systems")
        A = np.zeros((n, n))
        for r in range(self.N):
            for e in range(self.row_ptr[r], self.row_ptr[r + 1]):
                c = self.col_idx[e]
                A[3 * r:3 * r + 3, 3 * c:3 * c + 3] = self.vals[e]
        return A


def _faces(nx: int, ny: int, nz: int):
    """Face lists (lower cell, upper cell, direction 0=x 1=y 2=z)."""
    c = np.arange(nx * ny * nz, dtype=np.int64).reshape(nx, ny, nz)
    lo_x, hi_x = c[:-1, :, :].ravel(), c[1:, :, :].ravel()
    lo_y, hi_y = c[:, :-1, :].ravel(), c[:, 1:, :].ravel()
    lo_z, hi_z = c[:, :, :-1].ravel(), c[:, :, 1:].ravel()
    lo = np.concatenate([lo_x, lo_y, lo_z])
    hi = np.concatenate([hi_x, hi_y, hi_z])
    d = np.concatenate([
        np.zeros(lo_x.size, np.int8),
        np.ones(lo_y.size, np.int8),
        np.full(lo_z.size, 2, np.int8),
    ])
    return lo, hi, d


def generate(nx: int, ny: int, nz: int, seed: int, *, mu: float = 0.0,
             sigma: float = 1.0, vertical_factor: float = 10.0) -> System:
    """Draw one synthetic Jacobian system on an nx x ny x nz grid."""
    if min(nx, ny, nz) < 1:
        raise ValueError("grid dimensions must be positive")
    N = nx * ny * nz
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = np.exp(mu + sigma * rng.standard_normal(N))
    return _assemble_with(nx, ny, nz, perm, rng, seed, vertical_factor)


def redraw_values(sys: System, seed: int) -> System:
    """Same grid and pattern, new potentials/mobilities/accumulation/b.

    Stands in for the next Newton iteration's linear system: the rock
    permeability is kept, every other draw is taken again from ``seed`` in
    the same order as :func:`generate` (the permeability draw is consumed and
    discarded so that the remaining draws line up).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    rng.standard_normal(sys.N)
    return _assemble_with(sys.nx, sys.ny, sys.nz, sys.perm, rng, seed)


def _assemble_with(nx, ny, nz, perm, rng, seed, vertical_factor=10.0):
    """Draws 2-5 of the recipe, then the block assembly."""
    N = nx * ny * nz
    phi = rng.standard_normal(N)
    lo, hi, direction = _faces(nx, ny, nz)
    M = rng.uniform(0.1, 1.0, size=(lo.size, 3, 3))
    acc = np.empty((N, 3))
    acc[:, 0] = rng.uniform(1e-3, 1e-2, size=N)
    acc[:, 1] = rng.uniform(1.0, 2.0, size=N)
    acc[:, 2] = rng.uniform(1.0, 2.0, size=N)
    b = rng.standard_normal(3 * N)
    T = 2.0 * perm[lo] * perm[hi] / (perm[lo] + perm[hi])
    T = np.where(direction == 2, T * vertical_factor, T)
    M[:, :, 0] += M[:, :, 1] + M[:, :, 2]
    full = -T[:, None, None] * M
    press_only = full.copy()
    press_only[:, :, 1:] = 0.0
    lo_up = phi[lo] >= phi[hi]
    blk_hi_lo = np.where(lo_up[:, None, None], full, press_only)
    blk_lo_hi = np.where(lo_up[:, None, None], press_only, full)
    S = np.zeros((N, 7, 3, 3))
    present = np.zeros((N, 7), dtype=bool)
    plus_slot = np.array([SLOT_XP, SLOT_YP, SLOT_ZP])[direction]
    minus_slot = np.array([SLOT_XM, SLOT_YM, SLOT_ZM])[direction]
    S[lo, plus_slot] = blk_lo_hi
    S[hi, minus_slot] = blk_hi_lo
    present[lo, plus_slot] = True
    present[hi, minus_slot] = True
    colsum_p = np.zeros((N, 3))
    colsum_s = np.zeros((N, 3))
    for comp in range(3):
        colsum_p[:, comp] += np.bincount(hi, weights=blk_lo_hi[:, comp, 0], minlength=N)
        colsum_p[:, comp] += np.bincount(lo, weights=blk_hi_lo[:, comp, 0], minlength=N)
        colsum_s[:, comp] += np.bincount(hi, weights=blk_lo_hi[:, :, comp].sum(axis=1), minlength=N)
        colsum_s[:, comp] += np.bincount(lo, weights=blk_hi_lo[:, :, comp].sum(axis=1), minlength=N)
    D = np.zeros((N, 3, 3))
    D[:, :, 0] = -colsum_p
    D[:, 1, 1] = -colsum_s[:, 1]
    D[:, 2, 2] = -colsum_s[:, 2]
    D[:, 0, 0] += acc[:, 0]
    D[:, 1, 1] += acc[:, 1]
    D[:, 2, 2] += acc[:, 2]
    S[:, SLOT_DIAG] = D
    present[:, SLOT_DIAG] = True
    counts = present.sum(axis=1)
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    offsets = np.array([-ny * nz, -nz, -1, 0, 1, nz, ny * nz], dtype=np.int64)
    cols_full = np.arange(N, dtype=np.int64)[:, None] + offsets[None, :]
    return System(nx, ny, nz, row_ptr.astype(np.int32),
                  cols_full[present].astype(np.int32),
                  np.ascontiguousarray(S[present]), b, acc, perm, seed)
