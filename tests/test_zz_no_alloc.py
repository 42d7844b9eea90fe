"""asm_solve_noalloc (the solve that allocates nothing) against asm_solve.

The no-allocation entry point runs the same GMRES with the same kernels on
work arrays carved from the library's fixed device array, so each call must
return what asm_solve returns for the same system: same status, iteration
and cycle counts, and the same solution (the parity bar for FP64 solves is a
relative 1e-8; the arithmetic is the same, so the results are expected bit
for bit).  Two calls in a row, the second with a smaller system, show that
what the first call left in the shared array does not leak into the second.
"""
import numpy as np
import pytest

import gen

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


CASES = [
    # larger first, then smaller: the second call reuses the array the first filled
    ((40, 36, 20), 9, dict(kind=2, combine=1, sx=5, sy=4, overlap=1, near=(4, 4, 4), far=(8, 8, 8))),
    ((13, 11, 7), 5, dict(kind=1, combine=0, sx=3, sy=3, overlap=2)),
    ((10, 10, 5), 1, dict(kind=2, combine=1, sx=4, sy=1, overlap=1, near=(2, 2, 2), far=(5, 5, 5))),
]


def _check_same(P, G, B, b, **kw):
    import torch
    x1, i1 = P.solve(G, B, b, **kw)
    out = torch.zeros_like(x1)
    x2, i2 = P.solve(G, B, b, out=out, noalloc=True, **kw)
    assert x2.data_ptr() == out.data_ptr()
    assert (i1.status, i1.iters, i1.cycles) == (i2.status, i2.iters, i2.cycles)
    a, c = to_np(x1), to_np(x2)
    assert np.linalg.norm(a - c) <= 1e-8 * np.linalg.norm(a)
    assert np.array_equal(a, c)
    assert i1.rel_res_true == i2.rel_res_true
    return i2


def test_noalloc_equals_solve_two_calls_smaller_second(P):
    import torch
    systems = []
    for grid, seed, o in CASES:
        s = gen.generate(*grid, seed=seed)
        G = P.System.from_generated(s)
        B = P.Precond(G, **o)
        systems.append((s, G, B))
    for s, G, B in systems:
        info = _check_same(P, G, B, torch.from_numpy(s.b).cuda(), restart=30, rtol=1e-6)
        assert info.status == P.OK and info.rel_res_true <= 1e-6
    # fixed iteration count, a non-zero x0, and a restart length of 12
    s, G, B = systems[1]
    b = torch.from_numpy(s.b).cuda()
    x0 = torch.full_like(b, 0.5)
    x1, i1 = P.solve(G, B, b, x0=x0, restart=12, fixed_iters=41)
    x2, i2 = P.solve(G, B, b, x0=x0, restart=12, fixed_iters=41, noalloc=True)
    assert i1.iters == i2.iters == 41 and np.array_equal(to_np(x1), to_np(x2))


def test_noalloc_limits_and_errors(P):
    import torch
    # too large for the fixed array: rejected, nothing written
    s = gen.generate(48, 48, 40, seed=3)  # 92,160 cells, 276,480 unknowns
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, sx=4, sy=4, overlap=1)
    b = torch.from_numpy(s.b).cuda()
    out = torch.full_like(b, 7.0)
    with pytest.raises(P.AsmError) as e:
        P.solve(G, B, b, out=out, noalloc=True)
    assert e.value.status == P.ERR_INVALID
    assert bool((out == 7.0).all())
    # a shorter restart needs less room: the same system fits at restart 10? (31 vs 11 basis columns)
    need = 8 * ((10 + 1) * 3 * s.N + 3 * 3 * s.N)
    if need + (1 << 20) < P.NOALLOC_SCRATCH_BYTES:
        _check_same(P, G, B, b, restart=10, rtol=1e-6, max_iters=400)
    # non-finite input and zero right-hand side, as asm_solve
    s2 = gen.generate(10, 10, 5, seed=1)
    G2 = P.System.from_generated(s2)
    B2 = P.Precond(G2, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, sx=4, sy=1, overlap=1)
    bad = torch.from_numpy(s2.b).cuda()
    bad[3] = float("nan")
    with pytest.raises(P.AsmError) as e:
        P.solve(G2, B2, bad, noalloc=True)
    assert e.value.status == P.ERR_NONFINITE
    z = torch.zeros(s2.n, dtype=torch.float64, device="cuda")
    x, info = P.solve(G2, B2, z, x0=torch.ones_like(z), noalloc=True)
    assert info.status == P.OK and bool((x == 0).all())
