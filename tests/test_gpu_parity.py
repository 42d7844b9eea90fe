"""GPU path (C-ABI library) against the CPU oracle, element by element.

Tolerances:
  * SpMV, assembled A_i: summation-order differences only, relative 1e-13
    (of the row scale).
  * ILU(0) factors and one preconditioner apply: rounding of the
    factorisation and triangular solves, relative 1e-10 of the vector's max.
  * GMRES at an equal iteration count: solution within relative 1e-8 (the
    parity bar of the solve), iteration counts to rtol 1e-6 within +-1.
"""
import json
import os
import sys

import numpy as np
import pytest

import gen
import oracle as O

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
sys.path.insert(0, GOLDEN)
import fingerprint as FP  # noqa: E402


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_7227_amd as lib
    lib.load()
    # the in-tree native library is the one loaded
    maps = open("/proc/self/maps").read()
    assert lib.LIB_PATH in maps
    return lib


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


CASES = [
    # name, grid, seed, opts
    ("c1_additive", (10, 10, 5), 1, dict(kind=1, combine=0, sx=4, sy=1, overlap=1)),
    ("c1_ras", (10, 10, 5), 1, dict(kind=1, combine=1, sx=4, sy=1, overlap=1)),
    ("c1_two_level", (10, 10, 5), 1, dict(kind=2, combine=1, sx=4, sy=1, overlap=1, near=(2, 2, 2), far=(5, 5, 5))),
    ("mid_two_level", (13, 11, 7), 5, dict(kind=2, combine=1, sx=3, sy=2, overlap=1, near=(2, 2, 2), far=(4, 4, 4))),
    ("mid_two_level_d2", (13, 11, 7), 5, dict(kind=2, combine=1, sx=4, sy=3, overlap=2, near=(2, 3, 2), far=(5, 4, 3))),
    ("mid_two_level_d0_unit_near", (13, 11, 7), 5, dict(kind=2, combine=1, sx=3, sy=3, overlap=0, near=(1, 1, 1), far=(3, 3, 3))),
    ("mid_two_level_additive", (13, 11, 7), 5, dict(kind=2, combine=0, sx=2, sy=2, overlap=1, near=(3, 2, 2), far=(6, 6, 7))),
    ("mid_classical_d2_additive", (13, 11, 7), 5, dict(kind=1, combine=0, sx=3, sy=3, overlap=2)),
    ("one_subdomain", (13, 11, 7), 5, dict(kind=1, combine=1, sx=1, sy=1, overlap=0)),
    ("tiles_two_level", (40, 36, 20), 9, dict(kind=2, combine=1, sx=5, sy=4, overlap=1, near=(4, 4, 4), far=(8, 8, 8))),
    ("tiles_classical", (40, 36, 20), 9, dict(kind=1, combine=1, sx=5, sy=4, overlap=1)),
]


def oracle_precond(s, o):
    return O.Precond(O.Matrix.from_system(s), kind=o["kind"], combine=o["combine"], sx=o["sx"], sy=o["sy"],
                     overlap=o["overlap"], near=o.get("near", (2, 2, 2)), far=o.get("far", (4, 4, 4)))


def gpu_precond(P, sysg, o, precision=0):
    return P.Precond(sysg, kind=o["kind"], combine=o["combine"], sx=o["sx"], sy=o["sy"], overlap=o["overlap"],
                     near=o.get("near", (2, 2, 2)), far=o.get("far", (4, 4, 4)), precision=precision)


# ---------------------------------------------------------------- SpMV
@pytest.mark.parametrize("grid", [(10, 10, 5), (13, 11, 7), (1, 1, 1), (7, 1, 3), (40, 36, 20)])
def test_spmv_matches_oracle(P, grid):
    import torch
    s = gen.generate(*grid, seed=3)
    x = np.random.default_rng(1).standard_normal(s.n)
    G = P.System.from_generated(s)
    y = to_np(G.spmv(torch.from_numpy(x).cuda()))
    ref = O.spmv(O.Matrix.from_system(s), x)
    scale = np.abs(s.vals).sum(axis=(1, 2)).max() * np.abs(x).max()
    assert np.abs(y - ref).max() <= 1e-13 * scale


def test_spmv_config2_full_size(P):
    """128x128x64 (1,048,576 cells) in the layout the benchmark times."""
    import torch
    s = gen.generate(128, 128, 64, seed=2)
    x = np.random.default_rng(2).standard_normal(s.n)
    G = P.System.from_generated(s)
    y = to_np(G.spmv(torch.from_numpy(x).cuda()))
    ref = O.spmv(O.Matrix.from_system(s), x)
    scale = np.abs(s.vals).sum(axis=(1, 2)).max() * np.abs(x).max()
    assert np.abs(y - ref).max() <= 1e-13 * scale


# ---------------------------------------------------------------- setup
@pytest.mark.parametrize("name,grid,seed,o", CASES[:9], ids=[c[0] for c in CASES[:9]])
def test_local_matrices_factors_labels_match_oracle(P, name, grid, seed, o):
    s = gen.generate(*grid, seed=seed)
    G = P.System.from_generated(s)
    B = gpu_precond(P, G, o)
    Bo = oracle_precond(s, o)
    st = B.stats()
    assert st["nsub"] == Bo.nsub
    assert st["ext_rows"] == sum(Bo.sub(i).n for i in range(Bo.nsub))
    for i in range(Bo.nsub):
        so, sg = Bo.sub(i), B.export_sub(i)
        assert sg.n == so.n
        assert np.array_equal(sg.rp, so.rp) and np.array_equal(sg.ci, so.ci)
        assert np.array_equal(sg.label, so.label)
        assert rel(sg.a, so.a) <= 1e-13
        assert rel(sg.f, so.f) <= 1e-10


# ---------------------------------------------------------------- apply
@pytest.mark.parametrize("name,grid,seed,o", CASES, ids=[c[0] for c in CASES])
def test_apply_matches_oracle(P, name, grid, seed, o):
    import torch
    s = gen.generate(*grid, seed=seed)
    r = np.random.default_rng(4).standard_normal(s.n)
    G = P.System.from_generated(s)
    z = to_np(gpu_precond(P, G, o).apply(torch.from_numpy(r).cuda()))
    zo = oracle_precond(s, o).apply(r)
    assert rel(z, zo) <= 1e-10


def test_apply_global_ilu_with_reloads(P):
    """One subdomain over 64x64x32 (global block ILU(0), 131,072 rows): the
    level fronts outgrow the on-chip vector pool, so values are reloaded
    from global memory by fill steps."""
    import torch
    s = gen.generate(64, 64, 32, seed=3)
    r = np.random.default_rng(5).standard_normal(s.n)
    G = P.System.from_generated(s)
    o = dict(kind=1, combine=1, sx=1, sy=1, overlap=0)
    B = gpu_precond(P, G, o)
    assert B.stats()["reloaded_rows"] > 0
    z = to_np(B.apply(torch.from_numpy(r).cuda()))
    zo = oracle_precond(s, o).apply(r)
    assert rel(z, zo) <= 1e-10
    # two subdomains with overlap 2, additive combine
    o2 = dict(kind=1, combine=0, sx=2, sy=1, overlap=2)
    z2 = to_np(gpu_precond(P, G, o2).apply(torch.from_numpy(r).cuda()))
    assert rel(z2, oracle_precond(s, o2).apply(r)) <= 1e-10


def test_split_rows_match_oracle(P):
    """Near boxes spanning a whole y-z face (1 x 16 x 64 cells): each near
    coarse row couples to 1,024 fine cells, more entries than one LDS record
    holds, so the sweeps compute it in pieces that carry the partial sum
    from step to step (and reload inputs without an on-chip slot).  Factors
    and one application against the oracle at 1e-10."""
    import torch
    s = gen.generate(24, 16, 64, seed=11)
    o = dict(kind=2, combine=1, sx=3, sy=1, overlap=1, near=(1, 16, 64), far=(8, 8, 8))
    G = P.System.from_generated(s)
    Bo = oracle_precond(s, o)
    r = np.random.default_rng(6).standard_normal(s.n)
    for prec in (0, 1):
        B = gpu_precond(P, G, o, precision=prec)
        st = B.stats()
        assert st["split_rows"] > 0 and st["reloaded_rows"] > 0
        if prec == 0:
            for i in range(Bo.nsub):
                so, sg = Bo.sub(i), B.export_sub(i)
                assert np.array_equal(sg.ci, so.ci) and np.array_equal(sg.label, so.label)
                assert rel(sg.a, so.a) <= 1e-13
                assert rel(sg.f, so.f) <= 1e-10
        z = to_np(B.apply(torch.from_numpy(r).cuda()))
        assert rel(z, Bo.apply(r)) <= (1e-10 if prec == 0 else 1e-4)


# ---------------------------------------------------------------- GMRES
SOLVE_CASES = [CASES[0], CASES[1], CASES[2], CASES[3], CASES[9], CASES[10]]


@pytest.mark.parametrize("name,grid,seed,o", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_gmres_matches_oracle(P, name, grid, seed, o):
    s = gen.generate(*grid, seed=seed)
    A = O.Matrix.from_system(s)
    Bo = oracle_precond(s, o)
    ref = O.gmres(A, Bo, s.b, restart=30, rtol=1e-6)
    assert ref.status == O.OK
    G = P.System.from_generated(s)
    B = gpu_precond(P, G, o)
    x, info = P.solve(G, B, s.b, restart=30, rtol=1e-6)
    assert info.status == P.OK
    assert abs(info.iters - ref.iters) <= 1
    assert info.rel_res_true <= 1e-6
    # equal iteration counts: solutions agree to 1e-8
    xf, inf2 = P.solve(G, B, s.b, restart=30, fixed_iters=ref.iters)
    assert inf2.iters == ref.iters
    xf = to_np(xf)
    assert np.linalg.norm(xf - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_gmres_restart_boundary_and_x0(P):
    """Fixed counts across a restart and from a non-zero x0."""
    s = gen.generate(13, 11, 7, seed=5)
    o = CASES[3][3]
    A = O.Matrix.from_system(s)
    x0 = np.random.default_rng(8).standard_normal(s.n)
    ref = O.gmres(A, oracle_precond(s, o), s.b, x0=x0, restart=10, fixed_iters=25)
    G = P.System.from_generated(s)
    x, info = P.solve(G, gpu_precond(P, G, o), s.b, x0=x0, restart=10, fixed_iters=25)
    assert info.iters == 25 and info.cycles == ref.cycles
    assert np.linalg.norm(to_np(x) - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_gmres_deterministic(P):
    s = gen.generate(40, 36, 20, seed=9)
    o = CASES[9][3]
    G = P.System.from_generated(s)
    B = gpu_precond(P, G, o)
    x1, i1 = P.solve(G, B, s.b)
    x2, i2 = P.solve(G, B, s.b)
    assert i1.iters == i2.iters
    assert np.array_equal(to_np(x1), to_np(x2))


def test_unpreconditioned_and_zero_rhs(P):
    s = gen.generate(2, 2, 2, seed=3)
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=P.KIND_NONE)
    x, info = P.solve(G, B, s.b, rtol=1e-10)
    ref = np.linalg.solve(s.dense(), s.b)
    assert info.status == P.OK and info.iters <= s.n
    assert np.allclose(to_np(x), ref, rtol=1e-7, atol=1e-8 * np.abs(ref).max())
    x, info = P.solve(G, B, np.zeros(s.n))
    assert info.status == P.OK and info.iters == 0 and not to_np(x).any()


def test_iteration_limit(P):
    s = gen.generate(10, 10, 5, seed=1)
    G = P.System.from_generated(s)
    B = gpu_precond(P, G, CASES[1][3])
    x, info = P.solve(G, B, s.b, rtol=1e-12, max_iters=7)
    assert info.status == P.NOT_CONVERGED and info.iters == 7
    assert np.all(np.isfinite(to_np(x)))


def test_fp32_preconditioner(P):
    """Single-precision factors in fine rows; the FP64 outer loop still
    reaches the true residual tolerance.  Error against the FP64 oracle is
    bounded by the conditioning, not pinned."""
    s = gen.generate(40, 36, 20, seed=9)
    o = CASES[9][3]
    ref = O.gmres(O.Matrix.from_system(s), oracle_precond(s, o), s.b, restart=30, rtol=1e-6)
    G = P.System.from_generated(s)
    x, info = P.solve(G, gpu_precond(P, G, o, precision=P.FP32), s.b, restart=30, rtol=1e-6)
    assert info.status == P.OK and info.rel_res_true <= 1e-6
    assert abs(info.iters - ref.iters) <= max(2, ref.iters // 10)
    err = np.linalg.norm(to_np(x) - ref.x) / np.linalg.norm(ref.x)
    assert err <= 1e-3


def test_update_values_and_refactor(P):
    import torch
    s = gen.generate(13, 11, 7, seed=5)
    s2 = gen.redraw_values(s, seed=6)
    o = CASES[3][3]
    G = P.System.from_generated(s)
    B = gpu_precond(P, G, o)
    G.update_values(torch.from_numpy(s2.vals.reshape(-1)).cuda())
    B.refactor()
    r = np.random.default_rng(5).standard_normal(s.n)
    z = to_np(B.apply(torch.from_numpy(r).cuda()))
    assert rel(z, oracle_precond(s2, o).apply(r)) <= 1e-10
    x, info = P.solve(G, B, s2.b)
    ref = O.gmres(O.Matrix.from_system(s2), oracle_precond(s2, o), s2.b)
    assert abs(info.iters - ref.iters) <= 1


# ---------------------------------------------------------------- error paths
def test_errors(P):
    import torch
    s = gen.generate(4, 3, 3, seed=1)
    vals = s.vals.copy()
    d0 = np.flatnonzero(s.col_idx[s.row_ptr[0]:s.row_ptr[1]] == 0)[0]
    vals[s.row_ptr[0] + d0] = 0.0
    G = P.System(s.nx, s.ny, s.nz, s.row_ptr, s.col_idx, vals)
    with pytest.raises(P.AsmError) as e:
        P.Precond(G, kind=P.KIND_CLASSICAL, sx=2, sy=1)
    assert e.value.status == P.ERR_SINGULAR_PIVOT and "cell 0" in str(e.value)
    bad = s.col_idx.copy()
    bad[[1, 2]] = bad[[2, 1]]
    with pytest.raises(P.AsmError) as e:
        P.System(s.nx, s.ny, s.nz, s.row_ptr, bad, s.vals)
    assert e.value.status == P.ERR_INVALID
    with pytest.raises(P.AsmError) as e:
        P.System(s.nx, s.ny + 1, s.nz, s.row_ptr, s.col_idx, s.vals)
    assert e.value.status == P.ERR_INVALID
    nanv = s.vals.copy()
    nanv[3, 1, 1] = np.inf
    with pytest.raises(P.AsmError) as e:
        P.System(s.nx, s.ny, s.nz, s.row_ptr, s.col_idx, nanv)
    assert e.value.status == P.ERR_NONFINITE
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=P.KIND_CLASSICAL, sx=2, sy=1)
    b = s.b.copy()
    b[5] = np.nan
    with pytest.raises(P.AsmError) as e:
        P.solve(G, B, torch.from_numpy(b).cuda())
    assert e.value.status == P.ERR_NONFINITE
    with pytest.raises(P.AsmError) as e:
        P.Precond(G, kind=P.KIND_CLASSICAL, sx=9, sy=1)
    assert e.value.status == P.ERR_INVALID


# ---------------------------------------------------------------- full size
def _golden():
    path = os.path.join(GOLDEN, "config2_oracle.json")
    if not os.path.exists(path):
        pytest.skip("oracle results for the 1M-cell system not generated")
    return json.load(open(path))


@pytest.mark.parametrize("variant", ["two_level_ras", "classical_ras", "classical_additive"])
def test_config2_solve_matches_oracle(P, variant):
    """128x128x64, 256 subdomains: iteration count within +-1 of the
    oracle's, true residual <= 1e-6, and at the oracle's iteration count the
    solution agrees to 1e-8 on the stored sample of unknowns."""
    gd = _golden()
    if variant not in gd:
        pytest.skip(f"{variant} not in golden file")
    g = gd[variant]
    s = gen.generate(*gd["grid"], seed=gd["seed"])
    G = P.System.from_generated(s)
    kind = P.KIND_TWO_LEVEL if variant.startswith("two") else P.KIND_CLASSICAL
    combine = P.ADDITIVE if variant.endswith("additive") else P.RESTRICTED
    B = P.Precond(G, kind=kind, combine=combine, sx=g["sx"], sy=g["sy"], overlap=g["overlap"],
                  near=tuple(g["near"]), far=tuple(g["far"]))
    x, info = P.solve(G, B, s.b, restart=30, rtol=1e-6, max_iters=3000)
    assert info.status == P.OK and info.rel_res_true <= 1e-6
    assert abs(info.iters - g["iters"]) <= 1
    xf, _ = P.solve(G, B, s.b, restart=30, fixed_iters=g["iters"])
    xh = to_np(xf)
    xs = xh[np.array(gd["sample"])]
    ref = np.array(g["x_sample"])
    assert np.linalg.norm(xs - ref) <= 1e-8 * np.linalg.norm(ref)
    # every subdomain: norms, component sums and projections of its owned cells
    if "x_fp" in g:
        worst, blk = FP.compare(FP.fingerprint(xh, gd["grid"], g["sx"], g["sy"]), g["x_fp"], 1e-8)
        assert worst <= 1.0, (variant, blk, worst)
    assert abs(np.linalg.norm(xh) - g["x_norm"]) <= 1e-8 * g["x_norm"]


def test_config3_fp32_factors_full_size_against_oracle(P):
    """128x128x64 two-level RAS with FP32 fine-row factors (Section 6's
    approximate local solves in single precision; Arnoldi, residual and
    coarse rows in FP64) against the FP64 oracle: status OK, true residual
    <= 1e-6, iteration count within max(2, 10%) of the FP64 oracle's, and at
    the oracle's iteration count the solution within a relative 1e-3 of the
    oracle's (on the sample, globally and per subdomain).  The measured
    error is printed: it is the figure this configuration reports."""
    gd = _golden()
    g = gd["two_level_ras"]
    s = gen.generate(*gd["grid"], seed=gd["seed"])
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, sx=g["sx"], sy=g["sy"], overlap=g["overlap"],
                  near=tuple(g["near"]), far=tuple(g["far"]), precision=P.FP32)
    x, info = P.solve(G, B, s.b, restart=30, rtol=1e-6, max_iters=3000)
    assert info.status == P.OK and info.rel_res_true <= 1e-6
    assert abs(info.iters - g["iters"]) <= max(2, int(0.1 * g["iters"]))
    xf, _ = P.solve(G, B, s.b, restart=30, fixed_iters=g["iters"])
    xh = to_np(xf)
    ref = np.array(g["x_sample"])
    err_sample = np.linalg.norm(xh[np.array(gd["sample"])] - ref) / np.linalg.norm(ref)
    assert err_sample <= 1e-3
    assert abs(np.linalg.norm(xh) - g["x_norm"]) <= 1e-3 * g["x_norm"]
    if "x_fp" in g:
        worst, blk = FP.compare(FP.fingerprint(xh, gd["grid"], g["sx"], g["sy"]), g["x_fp"], 1e-3)
        assert worst <= 1.0, (blk, worst)
    print(f"FP32 factors at 128x128x64: {info.iters} iterations (FP64 oracle {g['iters']}), "
          f"error vs the FP64 oracle at {g['iters']} iterations {err_sample:.3e} (sample)")


@pytest.mark.parametrize("variant", ["two_level_ras", "classical_ras", "classical_additive"])
def test_config2_apply_matches_oracle(P, variant):
    """One application z = B^-1 b at full size (128x128x64, 256 subdomains,
    the launch configuration of the benchmark): z on the stored sample of
    unknowns and the norm of the whole z agree with the oracle's to 1e-12
    (FP64 arithmetic, only the summation order differs)."""
    gd = _golden()
    if variant not in gd.get("apply", {}):
        pytest.skip(f"{variant} apply not in golden file")
    g = gd["apply"][variant]
    kinds = {"two_level_ras": (P.KIND_TWO_LEVEL, P.RESTRICTED), "classical_ras": (P.KIND_CLASSICAL, P.RESTRICTED),
             "classical_additive": (P.KIND_CLASSICAL, P.ADDITIVE)}
    kind, combine = kinds[variant]
    s = gen.generate(*gd["grid"], seed=gd["seed"])
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=kind, combine=combine, sx=16, sy=16, overlap=1, near=(4, 4, 4), far=(16, 16, 16))
    z = to_np(B.apply(s.b))
    ref = np.array(g["z_sample"])
    assert np.linalg.norm(z[np.array(gd["sample"])] - ref) <= 1e-12 * np.linalg.norm(ref)
    assert abs(np.linalg.norm(z) - g["z_norm"]) <= 1e-12 * g["z_norm"]
    # every subdomain: norms, component sums and projections of its owned cells
    if "z_fp" in g:
        worst, blk = FP.compare(FP.fingerprint(z, gd["grid"], 16, 16), g["z_fp"], 1e-12)
        assert worst <= 1.0, (variant, blk, worst)


# ---------------------------------------------------------------- batched solves
BATCH_CASES = [
    ((10, 10, 5), 1, dict(kind=2, combine=1, sx=4, sy=1, overlap=1, near=(2, 2, 2), far=(5, 5, 5)), 0),
    ((13, 11, 7), 5, dict(kind=1, combine=0, sx=3, sy=3, overlap=2), 0),
    ((16, 12, 8), 7, dict(kind=2, combine=1, sx=2, sy=2, overlap=1, near=(2, 2, 2), far=(4, 4, 4)), 1),
    ((9, 9, 6), 8, dict(kind=0, combine=1, sx=1, sy=1, overlap=0), 0),
    ((20, 18, 10), 9, dict(kind=1, combine=1, sx=3, sy=2, overlap=1), 0),
]


def _batch_setup(P):
    import torch
    systems, preconds, bs = [], [], []
    for grid, seed, o, prec in BATCH_CASES:
        s = gen.generate(*grid, seed=seed)
        G = P.System.from_generated(s)
        systems.append(G)
        preconds.append(gpu_precond(P, G, o, precision=prec))
        bs.append(torch.from_numpy(s.b).cuda())
    return systems, preconds, bs


@pytest.mark.parametrize("mode", ["rtol", "fixed", "limit"])
def test_solve_batch_equals_single_solves(P, mode):
    """Each system of a batch gets exactly the result of solving it alone
    (same kernels, same reduction order), whatever the others do."""
    systems, preconds, bs = _batch_setup(P)
    kw = dict(restart=30, rtol=1e-6, max_iters=2000)
    if mode == "fixed":
        kw.update(fixed_iters=37)
    if mode == "limit":
        kw.update(restart=8, max_iters=19)
    single = [P.solve(G, B, b, **kw) for G, B, b in zip(systems, preconds, bs)]
    xs, infos = P.solve_batch(systems, preconds, bs, **kw)
    for (x1, i1), x2, i2 in zip(single, xs, infos):
        assert (i1.status, i1.iters, i1.cycles) == (i2.status, i2.iters, i2.cycles)
        assert i1.rel_res_true == i2.rel_res_true
        assert np.array_equal(to_np(x1), to_np(x2))
    if mode == "rtol":  # the preconditioned ones converge (GMRES(30) alone may stagnate)
        assert all(i.status == P.OK for i, c in zip(infos, BATCH_CASES) if c[2]["kind"] != 0)
    if mode == "fixed":
        assert all(i.iters == 37 for i in infos)
    if mode == "limit":
        assert any(i.status == P.NOT_CONVERGED for i in infos)


def test_solve_batch_matches_oracle(P):
    """Every member of a batch against the FP64 CPU oracle: the rtol-stopped
    iteration count within +-1 (FP64 factors; max(2, 10%) with FP32
    factors) and, at the oracle's count (fixed_iters for the whole batch),
    the solution within a relative 1e-8 (FP64) or 1e-3 (FP32 factors)."""
    systems, preconds, bs = _batch_setup(P)
    xs, infos = P.solve_batch(systems, preconds, bs, restart=30, rtol=1e-6, max_iters=2000)
    for (grid, seed, o, prec), x, info in zip(BATCH_CASES, xs, infos):
        s = gen.generate(*grid, seed=seed)
        A = O.Matrix.from_system(s)
        Bo = oracle_precond(s, o)
        ref = O.gmres(A, Bo, s.b, restart=30, rtol=1e-6, max_iters=2000)
        assert info.status == ref.status, (grid, info, ref.status)
        bar = 1 if prec == 0 else max(2, int(0.1 * ref.iters))
        assert abs(info.iters - ref.iters) <= bar, (grid, info.iters, ref.iters)
    for fixed in (23, 61):
        xs, infos = P.solve_batch(systems, preconds, bs, restart=30, fixed_iters=fixed)
        for (grid, seed, o, prec), x, info in zip(BATCH_CASES, xs, infos):
            s = gen.generate(*grid, seed=seed)
            A = O.Matrix.from_system(s)
            ref = O.gmres(A, oracle_precond(s, o), s.b, restart=30, fixed_iters=fixed)
            assert info.iters == ref.iters == fixed
            err = np.linalg.norm(to_np(x) - ref.x) / np.linalg.norm(ref.x)
            assert err <= (1e-8 if prec == 0 else 1e-3), (grid, fixed, err)


# systems of the 256-system benchmark batch whose backward steps carry more
# than 128 rows with FP32 factors (a step's second input load per streaming
# wave): grid, seed, subdomains (sx, sy)
BIG_STEP_CASES = [((94, 26, 27), 1008, (8, 2)), ((81, 91, 14), 1023, (5, 5)), ((51, 83, 24), 1025, (4, 6)),
                  ((74, 94, 28), 1026, (6, 8)), ((88, 85, 32), 1040, (8, 7)), ((93, 59, 31), 1045, (8, 5))]


def test_big_steps_deterministic_in_batches(P):
    """Systems whose level steps hold more than 128 rows, two-level with FP32
    factors, solved in one batch twice and one at a time: every result is
    bit-identical (a step's inputs must all have landed before its rows are
    computed, whatever the load on the memory system)."""
    import torch
    systems, preconds, bs = [], [], []
    for grid, seed, (sx, sy) in BIG_STEP_CASES:
        s = gen.generate(*grid, seed=seed)
        G = P.System.from_generated(s)
        systems.append(G)
        preconds.append(P.Precond(G, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, sx=sx, sy=sy, overlap=1,
                                  near=(4, 4, 4), far=(16, 16, 16), precision=P.FP32))
        bs.append(torch.from_numpy(s.b).cuda())
    kw = dict(restart=30, fixed_iters=90)
    runs = [P.solve_batch(systems, preconds, bs, **kw) for _ in range(3)]
    single = [P.solve(G, B, b, **kw) for G, B, b in zip(systems, preconds, bs)]
    for k in range(len(systems)):
        ref = to_np(single[k][0])
        for xs, infos in runs:
            assert infos[k].iters == 90
            assert np.array_equal(to_np(xs[k]), ref), BIG_STEP_CASES[k]


@pytest.mark.parametrize("k", [0, 1])
def test_big_steps_apply_matches_oracle(P, k):
    """One application on a system whose backward steps hold more than 128
    rows (FP32 factors) against the FP64 oracle: FP64 factors within 1e-10,
    FP32 factors within the factors' rounding (1e-4)."""
    import torch
    grid, seed, (sx, sy) = BIG_STEP_CASES[k]
    s = gen.generate(*grid, seed=seed)
    o = dict(kind=2, combine=1, sx=sx, sy=sy, overlap=1, near=(4, 4, 4), far=(16, 16, 16))
    r = np.random.default_rng(11).standard_normal(s.n)
    zo = oracle_precond(s, o).apply(r)
    G = P.System.from_generated(s)
    for prec, bar in ((0, 1e-10), (1, 1e-4)):
        z = to_np(gpu_precond(P, G, o, precision=prec).apply(torch.from_numpy(r).cuda()))
        assert rel(z, zo) <= bar, (grid, prec, rel(z, zo))


def test_solve_batch_with_x0_and_errors(P):
    import torch
    systems, preconds, bs = _batch_setup(P)
    x0s = [torch.full_like(b, 0.25) for b in bs]
    single = [P.solve(G, B, b, x0=x0) for G, B, b, x0 in zip(systems, preconds, bs, x0s)]
    xs, infos = P.solve_batch(systems, preconds, bs, x0s)
    for (x1, i1), x2, i2 in zip(single, xs, infos):
        assert i1.iters == i2.iters and np.array_equal(to_np(x1), to_np(x2))
    with pytest.raises(P.AsmError):
        P.solve_batch([systems[0], systems[0]], [preconds[0], preconds[0]], [bs[0], bs[0]])
    with pytest.raises(P.AsmError):
        P.solve_batch([systems[0]], [preconds[1]], [bs[0]])
    bad = bs[1].clone()
    bad[5] = float("nan")
    with pytest.raises(P.AsmError):
        P.solve_batch(systems[:2], preconds[:2], [bs[0], bad])
