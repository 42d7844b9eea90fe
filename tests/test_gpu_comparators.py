"""The comparator preconditioners on the GPU against the CPU oracle.

Field variants of the two-level form (Section 5: near field only, far field
only, both) and the global coarse-grid corrections of Section 3 (eq. (3.5)
added to the Schwarz part, eq. (3.8) the two-stage form), with the
tolerances of the other parity tests: assembled A_i 1e-13, factors and one
application 1e-10 (relative to the largest entry), GMRES iteration counts
within 1 and solutions within 1e-8 at equal iteration counts.
"""
import numpy as np
import pytest

import gen
import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_7227_amd as lib
    lib.load()
    assert lib.LIB_PATH in open("/proc/self/maps").read()
    return lib


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def both(P, s, **o):
    G = P.System.from_generated(s)
    B = P.Precond(G, **{k: v for k, v in o.items() if k != "local"})
    ko = dict(o)
    if "cbox" in ko:
        ko["cbox"] = tuple(ko["cbox"])
    Bo = O.Precond(O.Matrix.from_system(s), **ko)
    return G, B, Bo


FIELD_CASES = [
    ("near_only", (13, 11, 7), 5, dict(kind=2, combine=1, sx=3, sy=2, overlap=1, near=(2, 2, 2), far=(4, 4, 4), field=1)),
    ("far_only", (13, 11, 7), 5, dict(kind=2, combine=1, sx=3, sy=2, overlap=1, near=(2, 2, 2), far=(4, 4, 4), field=2)),
    ("near_only_d0_x_split", (21, 21, 5), 3, dict(kind=2, combine=1, sx=6, sy=1, overlap=0, near=(3, 3, 3), far=(3, 3, 3), field=1)),
    ("far_only_d0_x_split", (21, 21, 5), 3, dict(kind=2, combine=1, sx=6, sy=1, overlap=0, near=(3, 3, 3), far=(3, 3, 3), field=2)),
    ("far_only_additive", (40, 36, 20), 9, dict(kind=2, combine=0, sx=5, sy=4, overlap=1, near=(4, 4, 4), far=(8, 8, 8), field=2)),
    ("near_only_tiles", (40, 36, 20), 9, dict(kind=2, combine=1, sx=5, sy=4, overlap=1, near=(4, 4, 4), far=(8, 8, 8), field=1)),
]


@pytest.mark.parametrize("name,grid,seed,o", FIELD_CASES, ids=[c[0] for c in FIELD_CASES])
def test_field_variants_match_oracle(P, name, grid, seed, o):
    import torch
    s = gen.generate(*grid, seed=seed)
    G, B, Bo = both(P, s, **o)
    for i in range(Bo.nsub):
        so, sg = Bo.sub(i), B.export_sub(i)
        assert sg.n == so.n
        assert np.array_equal(sg.rp, so.rp) and np.array_equal(sg.ci, so.ci)
        assert np.array_equal(sg.label, so.label)
        assert rel(sg.a, so.a) <= 1e-13
        assert rel(sg.f, so.f) <= 1e-10
    r = np.random.default_rng(4).standard_normal(s.n)
    assert rel(to_np(B.apply(torch.from_numpy(r).cuda())), Bo.apply(r)) <= 1e-10


COARSE_CASES = [
    ("add_classical", (13, 11, 7), 5, dict(kind=1, combine=1, sx=3, sy=2, overlap=1, coarse=1, cbox=(4, 4, 4))),
    ("two_stage_classical", (13, 11, 7), 5, dict(kind=1, combine=1, sx=3, sy=2, overlap=1, coarse=2, cbox=(4, 4, 4))),
    ("two_stage_two_level", (13, 11, 7), 5, dict(kind=2, combine=1, sx=3, sy=2, overlap=1, near=(2, 2, 2),
                                                    far=(4, 4, 4), coarse=2, cbox=(3, 5, 2))),
    ("add_classical_additive_d0", (21, 21, 5), 3, dict(kind=1, combine=0, sx=6, sy=1, overlap=0, coarse=1,
                                                         cbox=(2, 2, 2))),
    ("two_stage_d0_unit_z", (21, 21, 5), 3, dict(kind=1, combine=1, sx=6, sy=1, overlap=0, coarse=2, cbox=(3, 3, 1))),
    ("two_stage_tiles", (40, 36, 20), 9, dict(kind=1, combine=1, sx=5, sy=4, overlap=1, coarse=2, cbox=(8, 8, 10))),
]


@pytest.mark.parametrize("name,grid,seed,o", COARSE_CASES, ids=[c[0] for c in COARSE_CASES])
def test_coarse_correction_apply_matches_oracle(P, name, grid, seed, o):
    import torch
    s = gen.generate(*grid, seed=seed)
    G, B, Bo = both(P, s, **o)
    r = np.random.default_rng(5).standard_normal(s.n)
    assert rel(to_np(B.apply(torch.from_numpy(r).cuda())), Bo.apply(r)) <= 1e-10


@pytest.mark.parametrize("name,grid,seed,o", [COARSE_CASES[1], COARSE_CASES[3], FIELD_CASES[3]],
                         ids=["two_stage_classical", "add_classical_additive_d0", "far_only_d0_x_split"])
def test_comparator_gmres_matches_oracle(P, name, grid, seed, o):
    """Inside GMRES the basis vectors reach the preconditioner scaled (v_j =
    s_j U_j), which the two-stage form must apply before its residual."""
    s = gen.generate(*grid, seed=seed)
    G, B, Bo = both(P, s, **o)
    ref = O.gmres(O.Matrix.from_system(s), Bo, s.b, restart=30, rtol=1e-6)
    assert ref.status == O.OK
    x, info = P.solve(G, B, s.b, restart=30, rtol=1e-6)
    assert info.status == P.OK and abs(info.iters - ref.iters) <= 1
    xf, inf2 = P.solve(G, B, s.b, restart=30, fixed_iters=ref.iters)
    assert np.linalg.norm(to_np(xf) - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_two_stage_unit_boxes_converge_in_one_step(P):
    """1x1x1 coarse boxes: A_C = A and the two-stage preconditioner is A^-1."""
    s = gen.generate(6, 5, 4, seed=17)
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=1, combine=1, sx=2, sy=2, overlap=1, coarse=2, cbox=(1, 1, 1))
    x, info = P.solve(G, B, s.b, rtol=1e-10)
    assert info.status == P.OK and info.iters == 1


def test_coarse_refactor_clone_and_errors(P):
    import torch
    s1 = gen.generate(13, 11, 7, seed=5)
    s2 = gen.redraw_values(s1, seed=6)
    o = dict(kind=1, combine=1, sx=3, sy=2, overlap=1, coarse=2, cbox=(4, 4, 4))
    G1 = P.System.from_generated(s1)
    B1 = P.Precond(G1, **o)
    r = torch.from_numpy(np.random.default_rng(7).standard_normal(s1.n)).cuda()
    G2 = P.System.from_generated(s2)
    fresh = to_np(P.Precond(G2, **o).apply(r))
    assert np.array_equal(to_np(B1.clone(G2).apply(r)), fresh)
    G1.update_values(s2.vals)
    B1.refactor()
    assert np.array_equal(to_np(B1.apply(r)), fresh)
    with pytest.raises(P.AsmError):  # 3 x boxes above the dense limit
        P.Precond(P.System.from_generated(gen.generate(40, 40, 4, seed=1)), kind=1, sx=2, coarse=1,
                  cbox=(1, 1, 1))
    with pytest.raises(P.AsmError):
        P.Precond(G2, kind=0, coarse=1)
    with pytest.raises(P.AsmError):
        P.Precond(G2, kind=2, sx=2, field=5)
    with pytest.raises(P.AsmError):  # not in batched solves
        P.solve_batch([G2], [P.Precond(G2, **o)], [s2.b])


EXACT_CASES = [
    ("classical_ras", (13, 11, 7), 5, dict(kind=1, combine=1, sx=3, sy=2, overlap=1)),
    ("classical_additive_d2", (13, 11, 7), 5, dict(kind=1, combine=0, sx=3, sy=3, overlap=2)),
    ("two_level", (13, 11, 7), 5, dict(kind=2, combine=1, sx=3, sy=2, overlap=1, near=(2, 2, 2), far=(4, 4, 4))),
    ("far_only_d0_x_split", (21, 21, 5), 3, dict(kind=2, combine=1, sx=6, sy=1, overlap=0, near=(3, 3, 3),
                                                  far=(3, 3, 3), field=2)),
    ("near_only_d0_x_split", (21, 21, 5), 3, dict(kind=2, combine=1, sx=6, sy=1, overlap=0, near=(3, 3, 3),
                                                   far=(3, 3, 3), field=1)),
    ("two_stage_exact", (21, 21, 5), 3, dict(kind=1, combine=1, sx=6, sy=1, overlap=0, coarse=2, cbox=(3, 3, 5))),
]


@pytest.mark.parametrize("name,grid,seed,o", EXACT_CASES, ids=[c[0] for c in EXACT_CASES])
def test_exact_local_solves_match_oracle(P, name, grid, seed, o):
    """Exact local solves (Section 5): dense inverses of every A_i on the
    device against the oracle's dense LU; one application and GMRES."""
    import torch
    s = gen.generate(*grid, seed=seed)
    G = P.System.from_generated(s)
    B = P.Precond(G, local=P.LOCAL_EXACT, **o)
    Bo = O.Precond(O.Matrix.from_system(s), local=O.LOCAL_EXACT, **o)
    r = np.random.default_rng(6).standard_normal(s.n)
    assert rel(to_np(B.apply(torch.from_numpy(r).cuda())), Bo.apply(r)) <= 1e-9
    ref = O.gmres(O.Matrix.from_system(s), Bo, s.b, restart=30, rtol=1e-6)
    assert ref.status == O.OK
    x, info = P.solve(G, B, s.b, restart=30, rtol=1e-6)
    assert info.status == P.OK and abs(info.iters - ref.iters) <= 1
    xf, _ = P.solve(G, B, s.b, restart=30, fixed_iters=ref.iters)
    assert np.linalg.norm(to_np(xf) - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


def test_exact_unit_boxes_give_the_inverse(P):
    """Two-level with 1x1x1 boxes and exact local solves: every A_i is a
    permutation of A, so B^-1 = A^-1 and GMRES takes one step."""
    s = gen.generate(6, 5, 4, seed=17)
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=2, combine=1, sx=2, sy=2, overlap=1, near=(1, 1, 1), far=(1, 1, 1), local=P.LOCAL_EXACT)
    x, info = P.solve(G, B, s.b, rtol=1e-10)
    assert info.status == P.OK and info.iters == 1
    ref = np.linalg.solve(s.dense(), s.b)
    assert np.linalg.norm(to_np(x) - ref) <= 1e-9 * np.linalg.norm(ref)


def test_exact_refactor_clone_and_limits(P):
    import torch
    s1 = gen.generate(13, 11, 7, seed=5)
    s2 = gen.redraw_values(s1, seed=6)
    o = dict(kind=2, combine=1, sx=3, sy=2, overlap=1, near=(2, 2, 2), far=(4, 4, 4), local=P.LOCAL_EXACT)
    G1, G2 = P.System.from_generated(s1), P.System.from_generated(s2)
    B1 = P.Precond(G1, **o)
    r = torch.from_numpy(np.random.default_rng(7).standard_normal(s1.n)).cuda()
    fresh = to_np(P.Precond(G2, **o).apply(r))
    assert np.array_equal(to_np(B1.clone(G2).apply(r)), fresh)
    G1.update_values(s2.vals)
    B1.refactor()
    assert np.array_equal(to_np(B1.apply(r)), fresh)
    with pytest.raises(P.AsmError):  # one subdomain of 2,400 cells: 7,200 unknowns
        P.Precond(P.System.from_generated(gen.generate(20, 20, 6, seed=1)), kind=1, sx=1, sy=1, overlap=0,
                  local=P.LOCAL_EXACT)
    with pytest.raises(P.AsmError):
        P.solve_batch([G2], [P.Precond(G2, **o)], [s2.b])
