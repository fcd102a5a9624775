"""The full-size workloads in the launch configuration the benchmark times
(sigma = 10, tol 1e-10, default options), and the 256^3 workload at the
largest sigma, 16.  The oracle cannot finish these
solves in test time, so it supplies the first two outer loops on the full
problem (the first with the monomial basis, the second with the first
Ritz-based parameters), compared record by record with the GPU trace; the
whole solve is checked by properties: outcome, true residual recomputed on
the host, and the reported residual."""
import numpy as np
import pytest

import oracle as O
import spd_problems as P
from gpu_util import torch_cuda

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


@pytest.fixture(scope="module")
def env():
    torch = torch_cuda()
    import paper_1908_04081_amd as L
    L.lib()
    h = L.assg_create()
    yield torch, L, h
    L.assg_destroy(h)


_CACHE = {}


def _problem(name):
    if name not in _CACHE:
        _CACHE.clear()
        _CACHE[name] = P.make_config(name)
    return _CACHE[name]


@pytest.mark.parametrize("name,basis,sigma", [("poisson3d_256", "chebyshev", 10),
                                              ("poisson3d_256", "newton", 10),
                                              ("poisson3d_256", "chebyshev", 16),
                                              ("diffusion27_160", "chebyshev", 10)])
def test_full_size_solve(env, name, basis, sigma):
    torch, L, h = env
    pr = _problem(name)
    print(f"[fullsize] {name} {basis} sigma={sigma}: n={pr.n} nnz={pr.A.nnz}", flush=True)
    A = L.csr_to_device(pr.A)
    L.assg_analyze(h, A)
    b = torch.from_numpy(pr.b).cuda()
    x = torch.zeros_like(b)
    info = L.assg_solve(h, A, b, x, L.assg_default_opts(s_max=sigma, tol=1e-10, basis=basis,
                                                        record_trace=1))
    tr = L.assg_get_trace(h)
    assert info["outcome"] == L.CONVERGED, info
    xg = x.cpu().numpy()
    rel = np.linalg.norm(pr.b - pr.A @ xg) / np.linalg.norm(pr.b)
    assert rel <= 1e-10, rel
    assert abs(info["relres_true"] - rel) <= 1e-3 * rel
    assert len(tr) == info["outer_iters"] and sum(t["sk"] for t in tr) == info["total_iters"]
    loops = 2 if sigma == 10 else 1   # the oracle's cost grows with sigma
    print(f"[fullsize] GPU: {info['outer_iters']} loops, relres {rel:.3e}; oracle loops "
          f"0-{loops - 1}", flush=True)
    _, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=sigma, tol=1e-10, basis=basis,
                                max_outer=loops)
    for k, ro in enumerate(io["trace"][:loops]):
        rg = tr[k]
        assert (rg["sbar"], rg["stilde"], rg["sk"]) == (ro["sbar"], ro["stilde"], ro["sk"]), (k, rg, ro)
        ko, kg = np.array(ro["kappa"]), np.array(rg["kappa"])
        fin = np.isfinite(ko) & (ko < 1e6)
        tol_k = 1e-10 + 16 * U * ko[fin] ** 2
        assert np.all(np.abs(kg[fin] - ko[fin]) <= tol_k * ko[fin]), (k, kg, ko)
        for key in ("relres_updated", "phi", "psi", "c"):
            assert abs(rg[key] - ro[key]) <= 1e-9 * abs(ro[key]), (k, key, rg[key], ro[key])
        if np.isfinite(ro["lmax"]):
            assert abs(rg["lmax"] - ro["lmax"]) <= 1e-9 * abs(ro["lmax"])
            assert abs(rg["lmin"] - ro["lmin"]) <= 1e-9 * abs(ro["lmin"])
