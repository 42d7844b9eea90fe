"""The device-side input generator (torch) against the host recipe.

It draws from torch's generator, so values differ from the host generator;
what must agree is the block pattern, the structure of the blocks and the
column-sum invariant of the recipe (every scalar column sum of A equals the
accumulation of that unknown)."""
import numpy as np
import pytest
import torch

import gen
from gen import device as gd


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 1, 1), (1, 1, 4), (4, 3, 2), (6, 5, 7)])
def test_pattern_equals_host_generator(shape):
    rp, ci = gd.pattern(*shape, "cpu")
    s = gen.generate(*shape, seed=3)
    assert np.array_equal(rp.numpy(), s.row_ptr)
    assert np.array_equal(ci.numpy(), s.col_idx)


@pytest.mark.parametrize("shape", [(2, 2, 2), (5, 4, 3), (7, 6, 5)])
def test_column_sums_equal_accumulation(shape):
    nx, ny, nz = shape
    N = nx * ny * nz
    perm = gd.draw_perm(nx, ny, nz, 11, "cpu")
    vals, b, acc = gd.draw_values(nx, ny, nz, perm, 12)
    rp, ci = gd.pattern(nx, ny, nz, "cpu")
    A = np.zeros((3 * N, 3 * N))
    v = vals.numpy()
    for r in range(N):
        for e in range(int(rp[r]), int(rp[r + 1])):
            c = int(ci[e])
            A[3 * r:3 * r + 3, 3 * c:3 * c + 3] = v[e]
    scale = np.abs(A).max()
    assert np.abs(A.sum(axis=0) - acc.numpy().ravel()).max() <= 1e-12 * scale
    assert b.shape == (3 * N,)
    # off-diagonal blocks: minus a transmissibility times a mobility matrix,
    # with a dominant pressure column; one direction of each face sees the
    # neighbour's pressure only
    for r in range(N):
        for e in range(int(rp[r]), int(rp[r + 1])):
            c = int(ci[e])
            if c == r:
                # saturation columns of the diagonal block: one entry each
                assert v[e][0, 1] == 0 and v[e][2, 1] == 0 and v[e][0, 2] == 0 and v[e][1, 2] == 0
                continue
            blk = -v[e]
            assert (blk[:, 0] > 0).all()
            sat = blk[:, 1:]
            assert (sat == 0).all() or ((sat > 0).all() and (blk[:, 0] >= sat.sum(1) * 0.999).all())
        # exactly one of the two blocks of each face has zero saturation columns
        for e in range(int(rp[r]), int(rp[r + 1])):
            c = int(ci[e])
            if c <= r:
                continue
            back = [q for q in range(int(rp[c]), int(rp[c + 1])) if int(ci[q]) == r][0]
            z1 = (v[e][:, 1:] == 0).all()
            z2 = (v[back][:, 1:] == 0).all()
            assert z1 != z2


def test_same_seed_same_values():
    perm = gd.draw_perm(4, 4, 3, 5, "cpu")
    a = gd.draw_values(4, 4, 3, perm, 9)
    b = gd.draw_values(4, 4, 3, perm, 9)
    c = gd.draw_values(4, 4, 3, perm, 10)
    assert all(torch.equal(x, y) for x, y in zip(a, b))
    assert not torch.equal(a[0], c[0])
