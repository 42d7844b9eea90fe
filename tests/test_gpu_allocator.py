"""Device-memory hooks (asm_set_allocator) routed through torch's caching
allocator: a handle's arrays come from torch and go back when it is closed,
and the results are those of hipMalloc'd handles, bit for bit."""
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


def _solve(P, s, b):
    G = P.System.from_generated(s)
    B = P.Precond(G, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, sx=3, sy=2, overlap=1, near=(2, 2, 2),
                  far=(4, 4, 4))
    x, info = P.solve(G, B, b, restart=20, fixed_iters=30)
    return G, B, x, info


def test_torch_allocator_hooks(P):
    import torch
    s = gen.generate(24, 20, 12, seed=21)
    b = torch.from_numpy(s.b).cuda()
    G0, B0, x0, _ = _solve(P, s, b)
    x0 = x0.cpu().numpy()
    B0.close()
    G0.close()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    P.use_torch_allocator(True)
    try:
        G, B, x, info = _solve(P, s, b)
        torch.cuda.synchronize()
        during = torch.cuda.memory_allocated()
        # the matrix values alone (9 doubles per stored block) live in torch's pool now
        assert during - before >= 72 * s.nnzb
        assert info.iters == 30
        assert np.array_equal(x.cpu().numpy(), x0)
        del x
        B.close()
        G.close()
        torch.cuda.synchronize()
        after = torch.cuda.memory_allocated()
        assert after <= before + 4096
        # handles created before the switch keep hipMalloc; a mixed pair works
        P.use_torch_allocator(False)
        G2 = P.System.from_generated(s)
        P.use_torch_allocator(True)
        B2 = P.Precond(G2, kind=P.KIND_TWO_LEVEL, combine=P.RESTRICTED, sx=3, sy=2, overlap=1, near=(2, 2, 2),
                       far=(4, 4, 4))
        x2, _ = P.solve(G2, B2, b, restart=20, fixed_iters=30)
        assert np.array_equal(x2.cpu().numpy(), x0)
        B2.close()
        G2.close()
    finally:
        P.use_torch_allocator(False)
