"""The Jacobian recipe of :mod:`gen.jacobian`, drawn with torch on a device.

Serving workloads need thousands of systems of up to a million cells; drawing
them on the host is far slower than solving them.  This module draws the same
recipe (steps 1-5 of :mod:`gen.jacobian`: permeability, upwind potential, face
mobilities, accumulation, right-hand side; harmonic transmissibility, x10 on
z-faces; dominant pressure column; upwinding; diagonal from the column sums
plus accumulation) with ``torch.Generator`` on the target device.  The draws
come from torch's generator, not from PCG64, so the values differ from
:func:`gen.jacobian.generate` for the same seed; the block pattern, the
distributions and the column-sum structure are the same.  Like
:mod:`gen.jacobian` it holds none of the solver's arithmetic.

All sums are taken in a fixed order (no atomics), so a seed gives the same
values on every run.
"""
from __future__ import annotations

import torch


def _shift(t: torch.Tensor, axis: int, front: bool) -> torch.Tensor:
    """Pads a face array [..] along a grid axis by one zero slab, at the front
    (face k -> cell k+1) or at the back (face k -> cell k)."""
    shape = list(t.shape)
    shape[axis] = 1
    z = torch.zeros(shape, dtype=t.dtype, device=t.device)
    return torch.cat([z, t], axis) if front else torch.cat([t, z], axis)


def pattern(nx: int, ny: int, nz: int, device) -> tuple[torch.Tensor, torch.Tensor]:
    """Block pattern of the 7-point grid (row_ptr, col_idx, int32), the same
    as :func:`gen.jacobian.generate` gives."""
    N = nx * ny * nz
    present = _present(nx, ny, nz, device)
    counts = present.sum(1)
    row_ptr = torch.zeros(N + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    offsets = torch.tensor([-ny * nz, -nz, -1, 0, 1, nz, ny * nz], dtype=torch.int64, device=device)
    cols = torch.arange(N, dtype=torch.int64, device=device)[:, None] + offsets[None, :]
    return row_ptr.to(torch.int32), cols[present].to(torch.int32)


def _present(nx, ny, nz, device) -> torch.Tensor:
    ix = torch.arange(nx, device=device)[:, None, None].expand(nx, ny, nz)
    iy = torch.arange(ny, device=device)[None, :, None].expand(nx, ny, nz)
    iz = torch.arange(nz, device=device)[None, None, :].expand(nx, ny, nz)
    p = torch.stack([ix > 0, iy > 0, iz > 0, torch.ones_like(ix, dtype=torch.bool),
                     iz < nz - 1, iy < ny - 1, ix < nx - 1], -1)
    return p.reshape(-1, 7)


def draw_perm(nx: int, ny: int, nz: int, seed: int, device, *, sigma: float = 1.0) -> torch.Tensor:
    """Step 1: permeability exp(sigma * N(0,1)) per cell."""
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return torch.exp(sigma * torch.randn(nx * ny * nz, generator=g, device=device, dtype=torch.float64))


def draw_values(nx: int, ny: int, nz: int, perm: torch.Tensor, seed: int,
                vertical_factor: float = 10.0):
    """Steps 2-5 and the assembly on the grid's pattern: returns the block
    values [nnzb, 3, 3] (float64, the order of :func:`pattern`), b [3N] and
    the accumulation [N, 3]."""
    dev = perm.device
    f64 = torch.float64
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    N = nx * ny * nz
    phi = torch.randn(N, generator=g, device=dev, dtype=f64).reshape(nx, ny, nz)
    K = perm.reshape(nx, ny, nz)
    nfx, nfy, nfz = (nx - 1) * ny * nz, nx * (ny - 1) * nz, nx * ny * (nz - 1)
    M = torch.rand(nfx + nfy + nfz, 3, 3, generator=g, device=dev, dtype=f64) * 0.9 + 0.1
    acc = torch.empty(N, 3, device=dev, dtype=f64)
    acc[:, 0] = torch.rand(N, generator=g, device=dev, dtype=f64) * 9e-3 + 1e-3
    acc[:, 1] = torch.rand(N, generator=g, device=dev, dtype=f64) + 1.0
    acc[:, 2] = torch.rand(N, generator=g, device=dev, dtype=f64) + 1.0
    b = torch.randn(3 * N, generator=g, device=dev, dtype=f64)
    M[:, :, 0] += M[:, :, 1] + M[:, :, 2]
    S = torch.zeros(nx, ny, nz, 7, 3, 3, device=dev, dtype=f64)
    colsum_p = torch.zeros(nx, ny, nz, 3, device=dev, dtype=f64)
    colsum_s = torch.zeros(nx, ny, nz, 3, device=dev, dtype=f64)
    shapes = [(nx - 1, ny, nz), (nx, ny - 1, nz), (nx, ny, nz - 1)]
    plus_slot, minus_slot = [6, 5, 4], [0, 1, 2]
    start = 0
    for axis in range(3):
        sh = shapes[axis]
        cnt = sh[0] * sh[1] * sh[2]
        Mf = M[start:start + cnt].reshape(*sh, 3, 3)
        start += cnt
        lo_sl = [slice(None)] * 3
        hi_sl = [slice(None)] * 3
        lo_sl[axis] = slice(0, -1)
        hi_sl[axis] = slice(1, None)
        klo, khi = K[tuple(lo_sl)], K[tuple(hi_sl)]
        T = 2.0 * klo * khi / (klo + khi)
        if axis == 2:
            T = T * vertical_factor
        full = -T[..., None, None] * Mf
        press = full.clone()
        press[..., :, 1:] = 0.0
        lo_up = (phi[tuple(lo_sl)] >= phi[tuple(hi_sl)])[..., None, None]
        blk_hi_lo = torch.where(lo_up, full, press)  # row hi, column lo
        blk_lo_hi = torch.where(lo_up, press, full)  # row lo, column hi
        S[..., plus_slot[axis], :, :] += _shift(blk_lo_hi, axis, front=False)
        S[..., minus_slot[axis], :, :] += _shift(blk_hi_lo, axis, front=True)
        # column sums: blk_lo_hi sits in column hi, blk_hi_lo in column lo
        colsum_p += _shift(blk_lo_hi[..., :, 0], axis, front=True)
        colsum_p += _shift(blk_hi_lo[..., :, 0], axis, front=False)
        colsum_s += _shift(blk_lo_hi.sum(-2), axis, front=True)
        colsum_s += _shift(blk_hi_lo.sum(-2), axis, front=False)
    colsum_p = colsum_p.reshape(N, 3)
    colsum_s = colsum_s.reshape(N, 3)
    D = torch.zeros(N, 3, 3, device=dev, dtype=f64)
    D[:, :, 0] = -colsum_p
    D[:, 1, 1] = -colsum_s[:, 1]
    D[:, 2, 2] = -colsum_s[:, 2]
    D[:, 0, 0] += acc[:, 0]
    D[:, 1, 1] += acc[:, 1]
    D[:, 2, 2] += acc[:, 2]
    S = S.reshape(N, 7, 3, 3)
    S[:, 3] = D
    present = _present(nx, ny, nz, dev)
    return S[present].contiguous(), b, acc
