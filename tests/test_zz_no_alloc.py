"""assg_solve_noalloc (workspace in the library's static per-device scratch,
no allocation inside the call) against assg_solve through the C ABI: two
calls in a row, the second on a smaller system, each bit-identical to
assg_solve's result on the same handle and analysis (same kernels, same
partition); a system too large for the scratch and the options that would
allocate are refused."""
import numpy as np
import pytest

import oracle as O
import spd_problems as P
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = torch_cuda()
    import paper_1908_04081_amd as L
    L.lib()
    h = L.assg_create()
    yield torch, L, h
    L.assg_destroy(h)


def _both(torch, L, h, pr, **kw):
    Ad = L.csr_to_device(pr.A)
    L.assg_analyze(h, Ad)
    b = torch.from_numpy(pr.b).cuda()
    opts = L.assg_default_opts(**kw)
    x1 = torch.zeros_like(b)
    i1 = L.assg_solve(h, Ad, b, x1, opts)
    x2 = torch.zeros_like(b)
    i2 = L.assg_solve_noalloc(h, Ad, b, x2, opts)
    return x1.cpu().numpy(), i1, x2.cpu().numpy(), i2


def test_noalloc_matches_solve_twice_shrinking(env):
    torch, L, h = env
    for pr, kw in ((P.make_config("poisson3d_256", size=40), dict(s_max=10, tol=1e-10)),
                   (P.make_config("poisson2d_64", size=45), dict(s_max=7, tol=1e-10,
                                                                  basis="newton"))):
        x1, i1, x2, i2 = _both(torch, L, h, pr, **kw)
        assert i2["outcome"] == L.CONVERGED, i2
        assert np.array_equal(x1, x2), np.abs(x1 - x2).max()
        assert (i1["outer_iters"], i1["total_iters"]) == (i2["outer_iters"], i2["total_iters"])
        assert np.linalg.norm(pr.b - pr.A @ x2) / np.linalg.norm(pr.b) <= 1e-10
        xo, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, **kw)
        assert np.linalg.norm(x2 - xo) / np.linalg.norm(xo) <= 1e-8


def test_noalloc_limits(env):
    torch, L, h = env
    # 400,000 rows need more than the 64 MiB scratch at s_max = 10
    n = 400_000
    A = P.diagonal_matrix(np.linspace(1.0, 2.0, n))
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    assert L.assg_workspace_size(n, 10) > L.NOALLOC_SCRATCH_BYTES
    Ad = L.csr_to_device(A)
    L.assg_analyze(h, Ad)
    b = torch.ones(n, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(L.AssgError, match="scratch"):
        L.assg_solve_noalloc(h, Ad, b, x, L.assg_default_opts(s_max=10))
    # the same system fits at s_max = 4 (9 columns)
    assert L.assg_workspace_size(n, 4) <= L.NOALLOC_SCRATCH_BYTES
    info = L.assg_solve_noalloc(h, Ad, b, x, L.assg_default_opts(s_max=4, tol=1e-10))
    assert info["outcome"] == L.CONVERGED
    assert np.abs(x.cpu().numpy() * np.linspace(1.0, 2.0, n) - 1.0).max() <= 1e-9
    for bad in (dict(record_trace=1), dict(time_kernels=1)):
        with pytest.raises(L.AssgError, match="record_trace and time_kernels"):
            L.assg_solve_noalloc(h, Ad, b, x, L.assg_default_opts(s_max=4, **bad))
