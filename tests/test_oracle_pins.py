"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: dense
linear algebra from numpy, closed forms, invariants of the definitions, or
brute force written independently here on tiny inputs.
"""
import itertools

import numpy as np
import pytest

import gen
import oracle as O


# ---------------------------------------------------------------- helpers
def mat(s):
    return O.Matrix.from_system(s)


def widths(n, k):
    base, rem = divmod(n, k)
    return [base + 1] * rem + [base] * (k - rem)


def owners(nx, ny, nz, sx, sy):
    px = np.repeat(np.arange(sx), widths(nx, sx))
    py = np.repeat(np.arange(sy), widths(ny, sy))
    own = np.empty(nx * ny * nz, int)
    for ix, iy, iz in itertools.product(range(nx), range(ny), range(nz)):
        own[(ix * ny + iy) * nz + iz] = px[ix] * sy + py[iy]
    return own


def cell_xyz(c, ny, nz):
    return c // (ny * nz), (c // nz) % ny, c % nz


def fine_set(Ad, own, s, delta):
    """Cells within graph distance delta of subdomain s (brute force on the
    dense scalar matrix: cells a, b adjacent if any entry of block (a,b) or
    (b,a) is structurally present)."""
    N = own.size
    blk = np.abs(Ad).reshape(N, 3, N, 3).sum(axis=(1, 3)) > 0
    adj = blk | blk.T
    np.fill_diagonal(adj, False)
    cur = set(np.flatnonzero(own == s))
    for _ in range(delta):
        nxt = set(cur)
        for c in cur:
            nxt.update(np.flatnonzero(adj[c]))
        cur = nxt
    return sorted(cur)


def brute_labels(s, own, sub, sx, sy, delta, near, far, two_level):
    """Row of A_i for every cell, by direct use of the set definitions."""
    nx, ny, nz = s.nx, s.ny, s.nz
    Ad = s.dense()
    F = fine_set(Ad, own, sub, delta)
    label = -np.ones(s.N, int)
    for k, c in enumerate(F):
        label[c] = k
    if not two_level:
        return label, len(F), 0
    px, py = divmod(sub, sy)
    near_keys, far_keys = {}, {}
    for c in range(s.N):
        if label[c] >= 0:
            continue
        ox, oy = divmod(int(own[c]), sy)
        x, y, z = cell_xyz(c, ny, nz)
        if abs(ox - px) + abs(oy - py) == 1:
            key = (x // near[0], y // near[1], z // near[2])
            near_keys.setdefault(key, []).append(c)
        else:
            key = (x // far[0], y // far[1], z // far[2])
            far_keys.setdefault(key, []).append(c)
    nxt = len(F)
    for key in sorted(near_keys):
        for c in near_keys[key]:
            label[c] = nxt
        nxt += 1
    for key in sorted(far_keys):
        for c in far_keys[key]:
            label[c] = nxt
        nxt += 1
    return label, len(F), nxt - len(F)


def restriction(label, n_rows):
    """Scalar restriction matrix R_i (3 n_rows x 3N) from a label array."""
    N = label.size
    R = np.zeros((3 * n_rows, 3 * N))
    for c in range(N):
        u = label[c]
        if u >= 0:
            R[3 * u:3 * u + 3, 3 * c:3 * c + 3] += np.eye(3)
    return R


def dense_local(sub):
    """Dense scalar matrix of an exported A_i."""
    n = sub.n
    M = np.zeros((3 * n, 3 * n))
    for u in range(n):
        for e in range(sub.rp[u], sub.rp[u + 1]):
            v = sub.ci[e]
            M[3 * u:3 * u + 3, 3 * v:3 * v + 3] = sub.a[e]
    return M


def dense_factors(sub):
    """Dense unit-lower L and upper U (pivots D_i = inverse of the stored
    D_i^-1 on the diagonal) from exported ILU(0) factors."""
    n = sub.n
    L = np.eye(3 * n)
    U = np.zeros((3 * n, 3 * n))
    for u in range(n):
        for e in range(sub.rp[u], sub.rp[u + 1]):
            v = sub.ci[e]
            blk = sub.f[e]
            if v < u:
                L[3 * u:3 * u + 3, 3 * v:3 * v + 3] = blk
            elif v == u:
                U[3 * u:3 * u + 3, 3 * u:3 * u + 3] = np.linalg.inv(blk)
            else:
                U[3 * u:3 * u + 3, 3 * v:3 * v + 3] = blk
    return L, U


def pattern_mask(sub):
    n = sub.n
    m = np.zeros((3 * n, 3 * n), bool)
    for u in range(n):
        for e in range(sub.rp[u], sub.rp[u + 1]):
            v = sub.ci[e]
            m[3 * u:3 * u + 3, 3 * v:3 * v + 3] = True
    return m


def precond_matrix(P, n):
    """Dense B^-1 by applying the oracle preconditioner to unit vectors."""
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = P.apply(e)
    return M


# ---------------------------------------------------------------- SpMV
@pytest.mark.parametrize("grid", [(10, 10, 5), (3, 1, 4), (1, 1, 1)])
def test_spmv_equals_dense_product(grid):
    s = gen.generate(*grid, seed=1)
    x = np.random.default_rng(2).standard_normal(s.n)
    Ad = s.dense()
    y = O.spmv(mat(s), x)
    assert np.allclose(y, Ad @ x, rtol=0, atol=1e-14 * np.abs(Ad).sum(axis=1).max() * np.abs(x).max())


# ---------------------------------------------------------------- block ILU(0)
@pytest.mark.parametrize("kind,sx,sy,grid", [
    (O.KIND_CLASSICAL, 1, 1, (5, 4, 3)),
    (O.KIND_CLASSICAL, 3, 2, (6, 5, 4)),
    (O.KIND_TWO_LEVEL, 3, 2, (6, 5, 4)),
])
def test_ilu0_pattern_identity(kind, sx, sy, grid):
    """ILU(0): (L U)_ij = (A_i)_ij for every (i, j) in the pattern of A_i."""
    s = gen.generate(*grid, seed=4)
    P = O.Precond(mat(s), kind=kind, combine=O.RESTRICTED, sx=sx, sy=sy, overlap=1,
                  near=(2, 2, 2), far=(3, 3, 2))
    for i in range(P.nsub):
        sub = P.sub(i)
        L, U = dense_factors(sub)
        Ai = dense_local(sub)
        mask = pattern_mask(sub)
        scale = np.abs(Ai).max()
        err = np.abs((L @ U - Ai)[mask]).max()
        assert err <= 1e-12 * scale, (i, err, scale)


def test_ilu0_triangular_solves_match_dense_factors():
    s = gen.generate(6, 5, 4, seed=8)
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=2, sy=2, overlap=1, near=(2, 2, 2), far=(3, 3, 3))
    rng = np.random.default_rng(0)
    for i in range(P.nsub):
        sub = P.sub(i)
        L, U = dense_factors(sub)
        rh = rng.standard_normal(3 * sub.n)
        xh = P.sub_solve(i, rh)
        ref = np.linalg.solve(U, np.linalg.solve(L, rh))
        assert np.allclose(xh, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("grid", [(1, 1, 9), (8, 1, 1), (1, 6, 1)])
def test_ilu0_is_exact_on_block_tridiagonal(grid):
    """On a chain of cells A is block tridiagonal: ILU(0) drops nothing, so
    one-subdomain Schwarz with ILU(0) equals a dense solve."""
    s = gen.generate(*grid, seed=3)
    P = O.Precond(mat(s), kind=O.KIND_CLASSICAL, sx=1, sy=1, overlap=0)
    r = np.random.default_rng(1).standard_normal(s.n)
    z = P.apply(r)
    ref = np.linalg.solve(s.dense(), r)
    assert np.allclose(z, ref, rtol=1e-10, atol=1e-10 * np.abs(ref).max())


def test_ilu0_closed_form_without_triangles():
    """The 7-point grid graph has no triangles, so ILU(0) only modifies the
    pivots: D_i = A_ii - sum_{k<i, k~i} A_ik D_k^-1 A_ki, L_ik = A_ik D_k^-1,
    U_ij = A_ij."""
    s = gen.generate(5, 4, 6, seed=12)
    P = O.Precond(mat(s), kind=O.KIND_CLASSICAL, sx=2, sy=1, overlap=1)
    for i in range(P.nsub):
        sub = P.sub(i)
        blocks = {}
        for u in range(sub.n):
            for e in range(sub.rp[u], sub.rp[u + 1]):
                blocks[(u, int(sub.ci[e]))] = e
        D = {}
        for u in range(sub.n):
            d = sub.a[blocks[(u, u)]].copy()
            for (r, k), e in blocks.items():
                if r == u and k < u:
                    d -= sub.a[e] @ np.linalg.inv(D[k]) @ sub.a[blocks[(k, u)]]
            D[u] = d
        for (r, k), e in blocks.items():
            if k < r:
                ref = sub.a[e] @ np.linalg.inv(D[k])
            elif k == r:
                ref = np.linalg.inv(D[r])
            else:
                ref = sub.a[e]
            assert np.allclose(sub.f[e], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


# ---------------------------------------------------------------- Schwarz (classical)
@pytest.mark.parametrize("combine", [O.ADDITIVE, O.RESTRICTED])
@pytest.mark.parametrize("delta", [0, 1, 2])
def test_classical_exact_matches_brute_force(combine, delta):
    """(3.3)-(3.4) with exact local solves, written out densely here."""
    nx, ny, nz, sx, sy = 5, 4, 3, 2, 2
    s = gen.generate(nx, ny, nz, seed=6)
    Ad = s.dense()
    own = owners(nx, ny, nz, sx, sy)
    r = np.random.default_rng(3).standard_normal(s.n)
    z_ref = np.zeros(s.n)
    for i in range(sx * sy):
        F = fine_set(Ad, own, i, delta)
        idx = np.array([3 * c + k for c in F for k in range(3)])
        xi = np.linalg.solve(Ad[np.ix_(idx, idx)], r[idx])
        for j, c in enumerate(F):
            if combine == O.RESTRICTED and own[c] != i:
                continue
            z_ref[3 * c:3 * c + 3] += xi[3 * j:3 * j + 3]
    P = O.Precond(mat(s), kind=O.KIND_CLASSICAL, combine=combine, sx=sx, sy=sy,
                  overlap=delta, local=O.LOCAL_EXACT)
    z = P.apply(r)
    assert np.allclose(z, z_ref, rtol=1e-9, atol=1e-9 * np.abs(z_ref).max())


def test_one_subdomain_equals_global_ilu0_and_large_overlap_ras_too():
    s = gen.generate(6, 5, 4, seed=13)
    A = mat(s)
    r = np.random.default_rng(4).standard_normal(s.n)
    z1 = O.Precond(A, kind=O.KIND_CLASSICAL, sx=1, sy=1, overlap=1).apply(r)
    zbig = O.Precond(A, kind=O.KIND_CLASSICAL, combine=O.RESTRICTED, sx=3, sy=2,
                     overlap=6 + 5 + 4).apply(r)
    assert np.array_equal(z1, zbig)
    z2l = O.Precond(A, kind=O.KIND_TWO_LEVEL, sx=1, sy=1, overlap=1).apply(r)
    assert np.array_equal(z1, z2l)


def test_block_jacobi_special_case():
    """Additive Schwarz with no overlap and exact local solves is block
    Jacobi over the subdomains."""
    nx, ny, nz = 6, 4, 2
    s = gen.generate(nx, ny, nz, seed=14)
    Ad = s.dense()
    own = owners(nx, ny, nz, 3, 2)
    r = np.random.default_rng(5).standard_normal(s.n)
    z_ref = np.zeros(s.n)
    for i in range(6):
        idx = np.array([3 * c + k for c in np.flatnonzero(own == i) for k in range(3)])
        z_ref[idx] = np.linalg.solve(Ad[np.ix_(idx, idx)], r[idx])
    z = O.Precond(mat(s), kind=O.KIND_CLASSICAL, combine=O.ADDITIVE, sx=3, sy=2, overlap=0,
                  local=O.LOCAL_EXACT).apply(r)
    assert np.allclose(z, z_ref, rtol=1e-10, atol=1e-10 * np.abs(z_ref).max())


# ---------------------------------------------------------------- two-level (Section 4)
TL_CASES = [
    # grid, sx, sy, overlap, near, far
    ((6, 5, 4), 3, 2, 1, (2, 2, 2), (3, 3, 2)),
    ((7, 3, 3), 4, 1, 1, (2, 2, 2), (5, 5, 5)),
    ((5, 5, 3), 2, 2, 0, (2, 1, 3), (2, 3, 2)),
    ((6, 6, 2), 3, 3, 2, (1, 2, 1), (4, 4, 2)),
]


@pytest.mark.parametrize("grid,sx,sy,delta,near,far", TL_CASES)
def test_two_level_labels_brute_force(grid, sx, sy, delta, near, far):
    s = gen.generate(*grid, seed=2)
    own = owners(*grid, sx, sy)
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=sx, sy=sy, overlap=delta, near=near, far=far)
    for i in range(sx * sy):
        lab, nf, nc = brute_labels(s, own, i, sx, sy, delta, near, far, True)
        sub = P.sub(i)
        assert (sub.nfine, sub.ncoarse) == (nf, nc)
        assert np.array_equal(sub.label, lab)
        assert np.array_equal(sub.owned.astype(bool), own[sub.cell] == i)


@pytest.mark.parametrize("grid,sx,sy,delta,near,far", TL_CASES)
def test_two_level_assembly_is_RART(grid, sx, sy, delta, near, far):
    """A_i = R_i A R_i^T with R_i of (4.1): selection on the fine cells and
    summation (App. B, (B.3)) on each coarse group, per unknown."""
    s = gen.generate(*grid, seed=2)
    Ad = s.dense()
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=sx, sy=sy, overlap=delta, near=near, far=far)
    for i in range(sx * sy):
        sub = P.sub(i)
        R = restriction(sub.label, sub.n)
        ref = R @ Ad @ R.T
        got = dense_local(sub)
        assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
        # the stored pattern is exactly the block pattern reached by A's
        # structural blocks
        Sb = np.zeros((s.N, s.N))
        for a in range(s.N):
            Sb[a, s.col_idx[s.row_ptr[a]:s.row_ptr[a + 1]]] = 1.0
        Rb = np.zeros((sub.n, s.N))
        Rb[sub.label[sub.label >= 0], np.flatnonzero(sub.label >= 0)] = 1.0
        blk = np.kron((Rb @ Sb @ Rb.T) > 0, np.ones((3, 3), bool))
        assert np.array_equal(pattern_mask(sub), blk)


def test_two_level_column_sums_are_lumped_accumulation():
    """Every cell lies in exactly one row group of R_i, so 1^T R_i = 1^T and
    the scalar column sums of A_i are the lumped accumulations R_i acc."""
    s = gen.generate(6, 5, 4, seed=21)
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=3, sy=2, overlap=1, near=(2, 2, 2), far=(3, 3, 2))
    for i in range(P.nsub):
        sub = P.sub(i)
        cs = dense_local(sub).sum(axis=0).reshape(-1, 3)
        lumped = np.zeros((sub.n, 3))
        np.add.at(lumped, sub.label, s.acc)
        scale = np.abs(dense_local(sub)).sum(axis=0).reshape(-1, 3)
        assert np.all(np.abs(cs - lumped) <= 1e-12 * scale + 1e-14)


def test_two_level_unit_boxes_reproduce_the_exact_inverse():
    """With 1x1x1 boxes every outside cell is its own coarse variable, A_i is
    a permutation of A, and the exact-mode preconditioner is A^-1."""
    s = gen.generate(5, 4, 3, seed=17)
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=2, sy=2, overlap=1, near=(1, 1, 1),
                  far=(1, 1, 1), local=O.LOCAL_EXACT)
    r = np.random.default_rng(6).standard_normal(s.n)
    ref = np.linalg.solve(s.dense(), r)
    assert np.allclose(P.apply(r), ref, rtol=1e-8, atol=1e-9 * np.abs(ref).max())
    res = O.gmres(mat(s), P, s.b, rtol=1e-10)
    assert res.status == O.OK and res.iters == 1


@pytest.mark.parametrize("grid,sx,sy,delta,near,far", TL_CASES)
def test_appendix_b_lumped_residual_vanishes(grid, sx, sy, delta, near, far):
    """App. B, (B.4)-(B.6): after an exact solve of the lumped system the
    lumped residual R_i (r - A R_i^T A_i^-1 R_i r) is zero, so its total over
    all unknowns (the residual sum of Section 2) vanishes too."""
    s = gen.generate(*grid, seed=5)
    Ad = s.dense()
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=sx, sy=sy, overlap=delta, near=near, far=far,
                  local=O.LOCAL_EXACT)
    r = np.random.default_rng(7).standard_normal(s.n)
    for i in range(sx * sy):
        sub = P.sub(i)
        R = restriction(sub.label, sub.n)
        xh = P.sub_solve(i, R @ r)
        new_r = r - Ad @ (R.T @ xh)
        lumped = R @ new_r
        assert np.abs(lumped).max() <= 1e-9 * np.abs(r).max() * np.abs(Ad).max()
        assert abs(new_r.sum()) <= 1e-9 * np.abs(r).sum() * np.abs(Ad).max()


def test_two_level_exact_matches_brute_force_apply():
    """(4.2)-(4.5) with exact local solves: z takes each owned fine row of
    A_i^-1 R_i r; the coarse part is discarded."""
    grid, sx, sy, delta, near, far = (6, 5, 4), 3, 2, 1, (2, 2, 2), (3, 3, 2)
    s = gen.generate(*grid, seed=9)
    Ad = s.dense()
    own = owners(*grid, sx, sy)
    r = np.random.default_rng(8).standard_normal(s.n)
    z_ref = np.zeros(s.n)
    for i in range(sx * sy):
        lab, nf, nc = brute_labels(s, own, i, sx, sy, delta, near, far, True)
        R = restriction(lab, nf + nc)
        xh = np.linalg.solve(R @ Ad @ R.T, R @ r)
        for c in range(s.N):
            if own[c] == i:
                z_ref[3 * c:3 * c + 3] = xh[3 * lab[c]:3 * lab[c] + 3]
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, combine=O.RESTRICTED, sx=sx, sy=sy,
                  overlap=delta, near=near, far=far, local=O.LOCAL_EXACT)
    assert np.allclose(P.apply(r), z_ref, rtol=1e-8, atol=1e-9 * np.abs(z_ref).max())


def test_config1_two_level_sizes():
    """Config 1 (10x10x5, 4 subdomains along x, overlap 1, near 2^3, far
    5^3): x widths 3,3,2,2; extended fine rows 200/250/200/150."""
    s = gen.generate(10, 10, 5, seed=1)
    P = O.Precond(mat(s), kind=O.KIND_TWO_LEVEL, sx=4, sy=1, overlap=1, near=(2, 2, 2), far=(5, 5, 5))
    assert [P.sub(i).nfine for i in range(4)] == [200, 250, 200, 150]
    assert sum(P.sub(i).ncoarse for i in range(4)) == 115


# ---------------------------------------------------------------- GMRES
def test_gmres_unpreconditioned_finite_termination():
    """Without preconditioning and with restart >= n, GMRES reaches the
    exact solution in at most n steps."""
    s = gen.generate(2, 2, 2, seed=3)
    P = O.Precond(mat(s), kind=O.KIND_NONE)
    res = O.gmres(mat(s), P, s.b, restart=30, rtol=1e-10)
    assert res.status == O.OK and res.iters <= s.n and res.cycles == 1
    ref = np.linalg.solve(s.dense(), s.b)
    assert np.allclose(res.x, ref, rtol=1e-7, atol=1e-8 * np.abs(ref).max())


@pytest.mark.parametrize("kind", [O.KIND_NONE, O.KIND_CLASSICAL, O.KIND_TWO_LEVEL])
@pytest.mark.parametrize("k", [1, 2, 4, 6])
def test_gmres_minimal_residual_over_krylov_space(kind, k):
    """After k steps of right-preconditioned GMRES from x0,
    x_k = argmin ||b - A x|| over x0 + M K_k(A M, r0), M = B^-1; computed
    here by least squares over an explicit orthonormalised Krylov basis."""
    s = gen.generate(4, 3, 3, seed=19)
    Ad = s.dense()
    P = O.Precond(mat(s), kind=kind, combine=O.RESTRICTED, sx=2, sy=1, overlap=1,
                  near=(2, 2, 2), far=(2, 3, 3))
    M = precond_matrix(P, s.n)
    x0 = np.random.default_rng(9).standard_normal(s.n) * 0.1
    r0 = s.b - Ad @ x0
    K = np.empty((s.n, k))
    v = r0 / np.linalg.norm(r0)
    for j in range(k):
        K[:, j] = v
        v = Ad @ (M @ v)
        v /= np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(Ad @ M @ Q, r0, rcond=None)
    x_ref = x0 + M @ Q @ y
    res = O.gmres(mat(s), P, s.b, x0=x0, restart=30, fixed_iters=k)
    assert res.iters == k
    rn_ref = np.linalg.norm(s.b - Ad @ x_ref)
    rn = np.linalg.norm(s.b - Ad @ res.x)
    assert abs(rn - rn_ref) <= 1e-8 * np.linalg.norm(r0)
    assert abs(res.rel_res_true * np.linalg.norm(s.b) - rn) <= 1e-9 * np.linalg.norm(r0)
    assert np.allclose(res.x, x_ref, rtol=1e-6, atol=1e-7 * np.abs(x_ref).max())


def test_gmres_exact_preconditioner_one_step():
    s = gen.generate(4, 4, 3, seed=23)
    P = O.Precond(mat(s), kind=O.KIND_CLASSICAL, sx=1, sy=1, overlap=0, local=O.LOCAL_EXACT)
    res = O.gmres(mat(s), P, s.b, rtol=1e-10)
    assert res.status == O.OK and res.iters == 1
    ref = np.linalg.solve(s.dense(), s.b)
    assert np.allclose(res.x, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())


def test_gmres_restart_state_is_a_checkpoint():
    """Restarted GMRES carries only x between cycles: running 45 steps
    equals 30 steps then 15 more from the saved x, bitwise."""
    s = gen.generate(6, 5, 4, seed=29)
    A = mat(s)
    P = O.Precond(A, kind=O.KIND_CLASSICAL, combine=O.ADDITIVE, sx=3, sy=2, overlap=1)
    full = O.gmres(A, P, s.b, restart=30, fixed_iters=45)
    first = O.gmres(A, P, s.b, restart=30, fixed_iters=30)
    second = O.gmres(A, P, s.b, x0=first.x, restart=30, fixed_iters=15)
    assert full.iters == 45 and full.cycles == 2
    assert np.array_equal(full.x, second.x)


def test_gmres_converges_to_rtol_on_config1():
    s = gen.generate(10, 10, 5, seed=1)
    A = mat(s)
    Ad = s.dense()
    for kw in [dict(kind=O.KIND_CLASSICAL, combine=O.ADDITIVE),
               dict(kind=O.KIND_CLASSICAL, combine=O.RESTRICTED),
               dict(kind=O.KIND_TWO_LEVEL, combine=O.RESTRICTED)]:
        P = O.Precond(A, sx=4, sy=1, overlap=1, near=(2, 2, 2), far=(5, 5, 5), **kw)
        res = O.gmres(A, P, s.b, restart=30, rtol=1e-6)
        assert res.status == O.OK
        true = np.linalg.norm(s.b - Ad @ res.x) / np.linalg.norm(s.b)
        assert true <= 1e-6 and abs(true - res.rel_res_true) <= 1e-12


def test_gmres_iteration_limit_and_zero_rhs():
    s = gen.generate(5, 5, 5, seed=31)
    A = mat(s)
    P = O.Precond(A, kind=O.KIND_NONE)
    res = O.gmres(A, P, s.b, restart=10, rtol=1e-12, max_iters=7)
    assert res.status == O.NOT_CONVERGED and res.iters == 7
    assert np.all(np.isfinite(res.x)) and res.rel_res_true < 1.0
    z = O.gmres(A, P, np.zeros(s.n))
    assert z.status == O.OK and z.iters == 0 and not z.x.any()


# ---------------------------------------------------------------- error paths
def test_error_singular_pivot():
    s = gen.generate(4, 3, 3, seed=1)
    vals = s.vals.copy()
    d0 = np.flatnonzero(s.col_idx[s.row_ptr[0]:s.row_ptr[1]] == 0)[0]
    vals[s.row_ptr[0] + d0] = 0.0
    A = O.Matrix(s.nx, s.ny, s.nz, s.row_ptr, s.col_idx, vals)
    with pytest.raises(O.OracleError) as e:
        O.Precond(A, kind=O.KIND_CLASSICAL, sx=2, sy=1)
    assert e.value.status == O.SINGULAR
    assert "cell 0" in str(e.value)


def test_error_invalid_and_nonfinite():
    s = gen.generate(4, 3, 3, seed=1)
    A = mat(s)
    bad = s.col_idx.copy()
    bad[[1, 2]] = bad[[2, 1]]  # unsorted row 0
    with pytest.raises(O.OracleError) as e:
        O.Precond(O.Matrix(s.nx, s.ny, s.nz, s.row_ptr, bad, A.vals), kind=O.KIND_CLASSICAL)
    assert e.value.status == O.INVALID
    with pytest.raises(O.OracleError) as e:
        O.Precond(O.Matrix(s.nx, s.ny + 1, s.nz, s.row_ptr, s.col_idx, A.vals), kind=O.KIND_CLASSICAL)
    assert e.value.status == O.INVALID
    P = O.Precond(A, kind=O.KIND_CLASSICAL)
    b = s.b.copy()
    b[5] = np.nan
    with pytest.raises(O.OracleError) as e:
        O.gmres(A, P, b)
    assert e.value.status == O.NONFINITE
