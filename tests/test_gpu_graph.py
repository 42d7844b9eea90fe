"""Restart cycles run as captured HIP graphs (asm_solve_graph) against the
CPU oracle and against the host-driven solve.

The graph-mode solve does the host loop's arithmetic with the Givens
rotations and the small triangular solve on the device, so it meets the
same parity bar as asm_solve: iteration counts to rtol 1e-6 within +-1 of
the oracle's, solutions within relative 1e-8 at equal iteration counts.
Against asm_solve itself, at equal iteration counts, the solutions differ
only by the rounding of the rotations (relative 1e-10).
"""
import numpy as np
import pytest

import gen
import oracle as O
from test_gpu_parity import CASES, gpu_precond, oracle_precond, to_np

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


GRAPH_CASES = [CASES[0], CASES[2], CASES[3], CASES[6], CASES[9], CASES[10]]


@pytest.mark.parametrize("name,grid,seed,o", GRAPH_CASES, ids=[c[0] for c in GRAPH_CASES])
def test_graph_solve_matches_oracle(P, name, grid, seed, o):
    s = gen.generate(*grid, seed=seed)
    ref = O.gmres(O.Matrix.from_system(s), oracle_precond(s, o), s.b, restart=30, rtol=1e-6)
    assert ref.status == O.OK
    G = P.System.from_generated(s)
    B = gpu_precond(P, G, o)
    x, info = P.solve(G, B, s.b, restart=30, rtol=1e-6, graph=True)
    assert info.status == P.OK and info.rel_res_true <= 1e-6
    assert abs(info.iters - ref.iters) <= 1
    xf, inf2 = P.solve(G, B, s.b, restart=30, fixed_iters=ref.iters, graph=True)
    assert inf2.iters == ref.iters and inf2.cycles == ref.cycles
    assert np.linalg.norm(to_np(xf) - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_solve_equals_host_loop(P, precision):
    """Same iteration counts, cycles and (up to the rotations' rounding) the
    same iterates as the host-driven solve; the host's residual estimate is
    reproduced too."""
    s = gen.generate(40, 36, 20, seed=9)
    G = P.System.from_generated(s)
    B = gpu_precond(P, G, CASES[9][3], precision=precision)
    xh, ih = P.solve(G, B, s.b, restart=30, rtol=1e-6)
    xg, ig = P.solve(G, B, s.b, restart=30, rtol=1e-6, graph=True)
    assert (ig.status, ig.iters, ig.cycles) == (ih.status, ih.iters, ih.cycles)
    assert abs(ig.rel_res_true - ih.rel_res_true) <= 1e-5 * ih.rel_res_true
    assert abs(ig.rel_res_est - ih.rel_res_est) <= 1e-6 * ih.rel_res_est
    assert np.linalg.norm(to_np(xg) - to_np(xh)) <= 1e-10 * np.linalg.norm(to_np(xh))
    xh, ih = P.solve(G, B, s.b, restart=12, fixed_iters=41)
    xg, ig = P.solve(G, B, s.b, restart=12, fixed_iters=41, graph=True)
    assert (ig.iters, ig.cycles) == (ih.iters, ih.cycles) == (41, 4)
    assert np.linalg.norm(to_np(xg) - to_np(xh)) <= 1e-10 * np.linalg.norm(to_np(xh))


def test_graph_reuse_new_values_and_restart(P):
    """A captured cycle is kept for later calls with the same vectors: new
    contents of b and x0 are picked up; another restart length captures
    again; an iteration limit cuts a cycle short."""
    import torch
    s = gen.generate(13, 11, 7, seed=5)
    o = CASES[3][3]
    A = O.Matrix.from_system(s)
    G = P.System.from_generated(s)
    B = gpu_precond(P, G, o)
    b = torch.from_numpy(s.b.copy()).cuda()
    x = torch.zeros_like(b)
    rng = np.random.default_rng(3)
    for trial in range(3):
        bn = s.b * (1.0 + trial) + rng.standard_normal(s.n) * 0.1 * np.abs(s.b).max()
        x0 = rng.standard_normal(s.n) if trial == 2 else np.zeros(s.n)
        b.copy_(torch.from_numpy(bn))
        x.copy_(torch.from_numpy(x0))
        restart = 30 if trial < 2 else 10
        _, info = P.solve(G, B, b, out=x, restart=restart, fixed_iters=23, graph=True)
        ref = O.gmres(A, oracle_precond(s, o), bn, x0=x0, restart=restart, fixed_iters=23)
        assert info.iters == 23 and info.cycles == ref.cycles
        assert np.linalg.norm(to_np(x) - ref.x) <= 1e-8 * np.linalg.norm(ref.x)
    x.zero_()
    _, info = P.solve(G, B, b, out=x, restart=8, rtol=1e-14, max_iters=19, graph=True)
    assert info.status == P.NOT_CONVERGED and info.iters == 19 and info.cycles == 3
    assert np.all(np.isfinite(to_np(x)))


def test_graph_unpreconditioned_and_zero_rhs(P):
    s = gen.generate(2, 2, 2, seed=3)
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=P.KIND_NONE)
    x, info = P.solve(G, B, s.b, rtol=1e-10, graph=True)
    ref = np.linalg.solve(s.dense(), s.b)
    assert info.status == P.OK and info.iters <= s.n
    assert np.allclose(to_np(x), ref, rtol=1e-7, atol=1e-8 * np.abs(ref).max())
    x, info = P.solve(G, B, np.zeros(s.n), graph=True)
    assert info.status == P.OK and info.iters == 0 and not to_np(x).any()


def test_graph_rejects_coarse_and_exact_modes(P):
    s = gen.generate(6, 5, 4, seed=2)
    G = P.System.from_generated(s)
    for kw in (dict(coarse=P.COARSE_TWO_STAGE, cbox=(2, 2, 2)), dict(local=P.LOCAL_EXACT)):
        B = P.Precond(G, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, sx=2, sy=1, overlap=1, **kw)
        with pytest.raises(P.AsmError):
            P.solve(G, B, s.b, graph=True)
