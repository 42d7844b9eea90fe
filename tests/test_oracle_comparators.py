"""Pins of the oracle's comparator preconditioners (Section 3 and Section 5).

* Field variants of the two-level form compared in Section 5: near field
  only, far field only, near and far fields.
* Global coarse-grid correction: eq. (3.5)-(3.6), added to the Schwarz
  local solves, and the two-stage form of eq. (3.7)-(3.8).

Each is checked against dense numpy linear algebra built here from the
definitions (brute-force restriction operators), or against an invariant.
"""
import numpy as np
import pytest

import gen
import oracle as O
from test_oracle_pins import brute_labels, dense_local, mat, owners, restriction


def field_labels(s, own, sub, sx, sy, delta, near, far, field):
    """Labels for the field variants, from the near+far brute force: near
    only drops far cells; far only lumps every outside cell in far boxes."""
    if field == O.FIELD_NEAR_FAR:
        return brute_labels(s, own, sub, sx, sy, delta, near, far, True)
    lab, nf, _ = brute_labels(s, own, sub, sx, sy, delta, near, far, False)
    px, py = divmod(sub, sy)
    keys = {}
    for c in range(s.N):
        if lab[c] >= 0:
            continue
        ox, oy = divmod(int(own[c]), sy)
        x, y, z = c // (s.ny * s.nz), (c // s.nz) % s.ny, c % s.nz
        is_near = abs(ox - px) + abs(oy - py) == 1
        if field == O.FIELD_NEAR and is_near:
            keys.setdefault((x // near[0], y // near[1], z // near[2]), []).append(c)
        elif field == O.FIELD_FAR:
            keys.setdefault((x // far[0], y // far[1], z // far[2]), []).append(c)
    nxt = nf
    for key in sorted(keys):
        for c in keys[key]:
            lab[c] = nxt
        nxt += 1
    return lab, nf, nxt - nf


FIELD_CASES = [
    ((6, 5, 4), 3, 2, 1, (2, 2, 2), (3, 3, 2)),
    ((7, 3, 3), 4, 1, 0, (2, 2, 2), (5, 5, 5)),
    ((6, 6, 2), 3, 3, 2, (1, 2, 1), (4, 4, 2)),
]


@pytest.mark.parametrize("field", [O.FIELD_NEAR, O.FIELD_FAR, O.FIELD_NEAR_FAR])
@pytest.mark.parametrize("grid,sx,sy,delta,near,far", FIELD_CASES)
def test_field_variants_labels_and_assembly(grid, sx, sy, delta, near, far, field):
    s = gen.generate(*grid, seed=4)
    Ad = s.dense()
    own = owners(*grid, sx, sy)
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=sx, sy=sy, overlap=delta, near=near, far=far,
                  field=field)
    for i in range(sx * sy):
        lab, nf, nc = field_labels(s, own, i, sx, sy, delta, near, far, field)
        sub = P.sub(i)
        assert (sub.nfine, sub.ncoarse) == (nf, nc)
        assert np.array_equal(sub.label, lab)
        R = restriction(lab, nf + nc)
        ref = R @ Ad @ R.T
        assert np.allclose(dense_local(sub), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_near_field_with_unit_boxes_is_schwarz_on_the_neighbourhood():
    """Near field only with 1x1x1 boxes keeps every cell of the face
    neighbours at full resolution and drops the rest: exact local solves then
    give restricted Schwarz on the set (subdomain + overlap + face neighbours)."""
    grid, sx, sy = (6, 6, 3), 3, 3
    s = gen.generate(*grid, seed=8)
    Ad = s.dense()
    own = owners(*grid, sx, sy)
    r = np.random.default_rng(2).standard_normal(s.n)
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, combine=O.RESTRICTED, sx=sx, sy=sy, overlap=1,
                  near=(1, 1, 1), far=(2, 2, 2), field=O.FIELD_NEAR, local=O.LOCAL_EXACT)
    z_ref = np.zeros(s.n)
    for i in range(sx * sy):
        px, py = divmod(i, sy)
        S = [c for c in range(s.N)
             if own[c] == i or abs(own[c] // sy - px) + abs(own[c] % sy - py) == 1]
        lab_fine, _, _ = brute_labels(s, own, i, sx, sy, 1, (1, 1, 1), (1, 1, 1), False)
        S = sorted(set(S) | set(np.flatnonzero(lab_fine >= 0)))
        idx = np.concatenate([[3 * c, 3 * c + 1, 3 * c + 2] for c in S])
        x = np.linalg.solve(Ad[np.ix_(idx, idx)], r[idx])
        for k, c in enumerate(S):
            if own[c] == i:
                z_ref[3 * c:3 * c + 3] = x[3 * k:3 * k + 3]
    assert np.allclose(P.apply(r), z_ref, rtol=1e-8, atol=1e-9 * np.abs(z_ref).max())


def test_far_field_column_sums_are_lumped_accumulation():
    """Far field only still labels every cell, so 1^T R_i = 1^T and the
    scalar column sums of A_i are the lumped accumulations."""
    s = gen.generate(6, 5, 4, seed=21)
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=3, sy=2, overlap=1, near=(2, 2, 2), far=(3, 3, 2),
                  field=O.FIELD_FAR)
    for i in range(P.nsub):
        sub = P.sub(i)
        assert np.all(sub.label >= 0)
        M = dense_local(sub)
        lumped = np.zeros((sub.n, 3))
        np.add.at(lumped, sub.label, s.acc)
        scale = np.abs(M).sum(axis=0).reshape(-1, 3)
        assert np.all(np.abs(M.sum(axis=0).reshape(-1, 3) - lumped) <= 1e-12 * scale + 1e-14)


def coarse_restriction(s, cbox):
    """R_C by brute force: box (x // Cx, y // Cy, z // Cz) of each cell,
    boxes numbered in lexicographic (x, y, z) order of the global box grid."""
    nbx, nby, nbz = [-(-n // c) for n, c in zip((s.nx, s.ny, s.nz), cbox)]
    R = np.zeros((3 * nbx * nby * nbz, s.n))
    for c in range(s.N):
        x, y, z = c // (s.ny * s.nz), (c // s.nz) % s.ny, c % s.nz
        b = ((x // cbox[0]) * nby + y // cbox[1]) * nbz + z // cbox[2]
        R[3 * b:3 * b + 3, 3 * c:3 * c + 3] += np.eye(3)
    return R


COARSE_CASES = [
    ((6, 5, 4), O.KIND_CLASSICAL, 3, 2, 1, (2, 2, 2)),
    ((7, 4, 3), O.KIND_TWO_LEVEL, 2, 2, 0, (3, 2, 3)),
    ((8, 3, 2), O.KIND_CLASSICAL, 4, 1, 0, (4, 3, 2)),
]


@pytest.mark.parametrize("local", [O.LOCAL_ILU0, O.LOCAL_EXACT])
@pytest.mark.parametrize("grid,kind,sx,sy,delta,cbox", COARSE_CASES)
def test_global_coarse_correction_matches_definitions(grid, kind, sx, sy, delta, cbox, local):
    """eq. (3.5): B^-1 r = B_AS^-1 r + R_C^T A_C^-1 R_C r;
    eq. (3.8): B^-1 r = B_AS^-1 r + R_C^T A_C^-1 R_C (r - A B_AS^-1 r);
    A_C = R_C A R_C^T (eq. (3.6)), R_C the box sums built here."""
    s = gen.generate(*grid, seed=12)
    Ad = s.dense()
    RC = coarse_restriction(s, cbox)
    AC = RC @ Ad @ RC.T
    r = np.random.default_rng(4).standard_normal(s.n)
    kw = dict(kind=kind, combine=O.RESTRICTED, sx=sx, sy=sy, overlap=delta, near=(2, 2, 2), far=(3, 3, 3),
              local=local)
    z_as = O.Precond(mat(s), **kw).apply(r)
    add = O.Precond(mat(s), coarse=O.COARSE_ADDITIVE, cbox=cbox, **kw).apply(r)
    ref_add = z_as + RC.T @ np.linalg.solve(AC, RC @ r)
    assert np.allclose(add, ref_add, rtol=1e-9, atol=1e-10 * np.abs(ref_add).max())
    two = O.Precond(mat(s), coarse=O.COARSE_TWO_STAGE, cbox=cbox, **kw).apply(r)
    ref_two = z_as + RC.T @ np.linalg.solve(AC, RC @ (r - Ad @ z_as))
    assert np.allclose(two, ref_two, rtol=1e-9, atol=1e-10 * np.abs(ref_two).max())


@pytest.mark.parametrize("grid,kind,sx,sy,delta,cbox", COARSE_CASES)
def test_two_stage_leaves_no_coarse_residual(grid, kind, sx, sy, delta, cbox):
    """After the two-stage application the box sums of the residual vanish:
    R_C (r - A B^-1 r) = R_C r2 - A_C A_C^-1 R_C r2 = 0 (the conservation of
    App. B on the global coarse grid)."""
    s = gen.generate(*grid, seed=13)
    Ad = s.dense()
    RC = coarse_restriction(s, cbox)
    P = O.Precond(mat(s), kind=kind, sx=sx, sy=sy, overlap=delta, near=(2, 2, 2), far=(3, 3, 3),
                  coarse=O.COARSE_TWO_STAGE, cbox=cbox)
    r = np.random.default_rng(5).standard_normal(s.n)
    res = RC @ (r - Ad @ P.apply(r))
    assert np.abs(res).max() <= 1e-9 * np.abs(r).max() * np.abs(Ad).max()


def test_two_stage_with_unit_boxes_is_the_exact_inverse():
    """1x1x1 coarse boxes make R_C the identity and A_C = A, so (3.8) gives
    B^-1 = B_AS^-1 + A^-1 (I - A B_AS^-1) = A^-1: GMRES takes one step."""
    s = gen.generate(5, 4, 3, seed=17)
    P = O.Precond(mat(s), kind=O.KIND_CLASSICAL, sx=2, sy=2, overlap=1, coarse=O.COARSE_TWO_STAGE,
                  cbox=(1, 1, 1))
    r = np.random.default_rng(6).standard_normal(s.n)
    ref = np.linalg.solve(s.dense(), r)
    assert np.allclose(P.apply(r), ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
    res = O.gmres(mat(s), P, s.b, rtol=1e-10)
    assert res.status == O.OK and res.iters == 1


def test_comparator_option_errors():
    s = gen.generate(4, 4, 2, seed=1)
    with pytest.raises(O.OracleError):
        O.Precond(mat(s), kind=O.KIND_NONE, coarse=O.COARSE_ADDITIVE, cbox=(2, 2, 2))
    with pytest.raises(O.OracleError):
        O.Precond(mat(s), kind=O.KIND_CLASSICAL, sx=2, coarse=O.COARSE_TWO_STAGE, cbox=(0, 2, 2))
    with pytest.raises(O.OracleError):
        O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=2, field=3)
