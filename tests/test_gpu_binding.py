"""The Python binding checks every tensor it hands to the library by a bare
pointer (the C side cannot see an allocation's size): wrong length, dtype,
device or layout raises before any library call, so a caller's mistake never
becomes an out-of-bounds device access."""
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
    return lib


def test_vectors_are_checked(P):
    import torch
    s = gen.generate(6, 5, 4, seed=2)
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=P.KIND_CLASSICAL, combine=P.RESTRICTED, sx=2, sy=1, overlap=1)
    n = 3 * s.nx * s.ny * s.nz
    b = torch.from_numpy(s.b).cuda()
    with pytest.raises(ValueError, match="elements"):
        P.solve(G, B, b[:-3])
    with pytest.raises(ValueError, match="elements"):
        P.solve(G, B, b, x0=np.zeros(n + 3))
    with pytest.raises(TypeError, match="dtype"):
        P.solve(G, B, b, out=torch.zeros(n, dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError, match="contiguous"):
        P.solve(G, B, b, out=torch.zeros(2 * n, dtype=torch.float64, device="cuda")[::2])
    with pytest.raises(ValueError, match="GPU"):
        P.solve(G, B, b, out=torch.zeros(n, dtype=torch.float64))
    with pytest.raises(ValueError, match="elements"):
        B.apply(b, out=torch.zeros(n - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError, match="elements"):
        G.spmv(b[:n // 2])
    with pytest.raises(ValueError, match="elements"):
        G.update_values(s.vals.reshape(-1)[:-9])
    with pytest.raises(ValueError, match="elements"):
        P.System(s.nx, s.ny, s.nz, s.row_ptr, s.col_idx, s.vals.reshape(-1)[:-1])
    with pytest.raises(ValueError):
        P.solve_batch([G, G], [B], [b, b])
    # a correct call still works after the rejected ones
    x, info = P.solve(G, B, b, rtol=1e-8)
    assert info.status == P.OK


def test_server_request_tensors_are_checked(P):
    import torch
    s = gen.generate(6, 5, 4, seed=3)
    rp = torch.from_numpy(s.row_ptr).cuda()
    ci = torch.from_numpy(s.col_idx).cuda()
    v = torch.from_numpy(s.vals.reshape(-1).copy()).cuda()
    b = torch.from_numpy(s.b).cuda()
    srv = P.Server(max_active=2)
    popts = P.precond_opts(kind=P.KIND_CLASSICAL, sx=2, sy=1)
    grid = (s.nx, s.ny, s.nz)
    with pytest.raises(ValueError, match="elements"):
        srv.submit(1, grid, rp, ci, popts, [v], [b[:-1]], [torch.zeros_like(b)])
    with pytest.raises(TypeError, match="dtype"):
        srv.submit(1, grid, rp, ci, popts, [v.float()], [b], [torch.zeros_like(b)])
    assert srv.state()["queued"] == 0
    srv.close()


def test_solves_after_freed_systems_are_unchanged(P):
    """Each system's solver workspace holds pinned host memory through which
    the host reads the Hessenberg columns; the runtime hands freed pinned
    memory out again with the old contents still in it.  Systems created
    after others were freed must solve exactly as the first one did."""
    import gc
    import torch
    s = gen.generate(12, 10, 6, seed=4)
    o = dict(kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, sx=3, sy=2, overlap=1, near=(2, 2, 2), far=(4, 4, 4))
    b = torch.from_numpy(s.b).cuda()
    ref = None
    for rep in range(4):
        G = P.System.from_generated(s)
        B = P.Precond(G, **o)
        x, info = P.solve(G, B, b, restart=8, rtol=1e-8)
        got = (info.status, info.iters, info.cycles, x.cpu().numpy().copy())
        if ref is None:
            ref = got
        else:
            assert got[:3] == ref[:3]
            assert np.array_equal(got[3], ref[3])
        del G, B, x
        gc.collect()
