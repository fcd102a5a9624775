"""The debug build (libassg_debug.so: the kernels check the partition and
index invariants they rely on and report a failed check as an error of the
call) runs every entry point on workloads that exercise the multi-block
reduction chunks, long rows, batches, forced schedules and the no-alloc
solve, in a process of its own: no check fails and the results still match
the oracle."""
import os
import subprocess
import sys

import pytest

from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import sys
sys.path.insert(0, ROOT)
sys.path.insert(0, ROOT + "/tests")
import numpy as np, torch
import paper_1908_04081_amd as L
import oracle as O, spd_problems as P
L.load(L.DEBUG_LIB_PATH)
from test_gpu_kernels import _poisson3d_with_long_row
h = L.assg_create()
# single solve with several row blocks per chunk, HSCG, forced schedule, no-alloc
pr = P.make_config("poisson3d_256", size=64)
A = L.csr_to_device(pr.A); L.assg_analyze(h, A)
b = torch.from_numpy(pr.b).cuda(); x = torch.zeros_like(b)
xo, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10)
info = L.assg_solve(h, A, b, x, L.assg_default_opts(s_max=10, tol=1e-10, record_trace=1))
assert info["outcome"] == L.CONVERGED, info
assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-8
x.zero_(); hi = L.assg_hscg_solve(h, A, b, x, 1e-10, 0)
assert hi["outcome"] == L.CONVERGED
x.zero_()
fi = L.assg_solve_forced_schedule(h, A, b, x, [r["sk"] for r in io["trace"]],
                                  L.assg_default_opts(s_max=10, tol=1e-10))
assert fi["outcome"] == L.CONVERGED
ps = P.make_config("poisson2d_64", size=60)
As = L.csr_to_device(ps.A); L.assg_analyze(h, As)
bs = torch.from_numpy(ps.b).cuda(); xs = torch.zeros_like(bs)
ni = L.assg_solve_noalloc(h, As, bs, xs, L.assg_default_opts(tol=1e-10))
assert ni["outcome"] == L.CONVERGED
# a row longer than a block inside a multi-block chunk: basis, Gram, product, gradient scatter
M = _poisson3d_with_long_row(side=64, extra=3000)
Ad = L.csr_to_device(M); L.assg_analyze(h, Ad)
n = M.shape[0]
rng = np.random.default_rng(5)
p, r = rng.standard_normal(n), rng.standard_normal(n)
prm = O.make_params("chebyshev", 10, 0.01, 1.99)
G = L.assg_basis_gram(h, Ad, torch.from_numpy(p).cuda(), torch.from_numpy(r).cuda(), 10, *prm)
assert np.all(np.isfinite(G))
y = torch.empty(n, dtype=torch.float64, device="cuda")
L.assg_spmv(h, Ad, torch.from_numpy(p).cuda(), y)
assert np.allclose(y.cpu().numpy(), M @ p, rtol=1e-12, atol=1e-12)
g = torch.empty(M.nnz, dtype=torch.float64, device="cuda")
L.assg_csr_outer_on_pattern(h, Ad, torch.from_numpy(p).cuda(), torch.from_numpy(r).cuda(), -1.0, g)
# a batch of uneven systems
probs = P.make_batch(count=12, lo=8, hi=200, seed=31)
Ab = [L.csr_to_device(q.A) for q in probs]
L.assg_batch_analyze(h, Ab)
bb = [torch.from_numpy(q.b).cuda() for q in probs]; xb = [torch.zeros_like(v) for v in bb]
infos = L.assg_batch_solve(h, Ab, bb, xb, L.assg_default_opts(s_max=10, tol=1e-10))
assert all(i["outcome"] == L.CONVERGED for i in infos)
L.assg_destroy(h)
print("DEBUG_BUILD_OK")
'''


def test_debug_build_runs_clean():
    torch_cuda()
    import paper_1908_04081_amd as L
    if not os.path.exists(L.DEBUG_LIB_PATH):
        pytest.skip("libassg_debug.so not built")
    code = "ROOT = %r\n" % ROOT + SCRIPT
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0 and "DEBUG_BUILD_OK" in r.stdout, (r.stdout[-2000:],
                                                                r.stderr[-4000:])
