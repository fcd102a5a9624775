"""The differentiable solve (forward solve, adjoint solve, gradient scatter
on A's pattern) through the C ABI, against the dense reference gradient and
central finite differences."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import spd_problems as P
from gpu_util import torch_cuda
from test_gradient_reference import reference_gradient

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = torch_cuda()
    import paper_1908_04081_amd as L
    L.lib()
    return torch, L


def _rows(A):
    return np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))


def _ragged(n=3001, seed=7):
    rng = np.random.default_rng(seed)
    i = np.concatenate([rng.integers(0, n, 6 * n), np.full(5000, 17)])
    j = np.concatenate([rng.integers(0, n, 6 * n), rng.integers(0, n, 5000)])
    M = sp.coo_matrix((rng.uniform(-1, 1, i.size), (i, j)), shape=(n, n)).tocsr()
    M = (M + M.T + sp.eye(n) * 10).tocsr()
    M.sort_indices()
    M.indices = M.indices.astype(np.int32)
    M.indptr = M.indptr.astype(np.int32)
    return M


@pytest.mark.parametrize("name", ["poisson2d_37", "ragged_long_row", "varcoef7_9"])
def test_outer_on_pattern_is_exact(env, name):
    """alpha u_i v_j on every stored entry, bit for bit (one rounding of
    (alpha u_i) v_j), including a row longer than one block's capacity."""
    torch, L = env
    A = {"poisson2d_37": lambda: P.poisson2d(37), "ragged_long_row": _ragged,
         "varcoef7_9": lambda: P.varcoef7(9, 1.0, 105)}[name]()
    n = A.shape[0]
    assert np.diff(A.indptr).max() > 2048 or name != "ragged_long_row"
    rng = np.random.default_rng(5)
    u, v = rng.standard_normal(n), rng.standard_normal(n)
    h = L.assg_create()
    Ad = L.csr_to_device(A)
    L.assg_analyze(h, Ad)
    out = torch.full((A.nnz,), np.nan, dtype=torch.float64, device="cuda")
    L.assg_csr_outer_on_pattern(h, Ad, torch.from_numpy(u).cuda(), torch.from_numpy(v).cuda(),
                                -0.75, out)
    ref = (-0.75 * u[_rows(A)]) * v[A.indices]
    assert np.array_equal(out.cpu().numpy(), ref)
    L.assg_destroy(h)


def _kappa(A):
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(A, k=1, sigma=0, which="LM", return_eigenvectors=False)[0]
    return lmax / lmin


def test_gradient_matches_dense_reference(env):
    """varcoef7 16^3 (lognormal sigma=1): autograd gradients in b and in A's
    values against dense solves.  Both solves stop at relative residual
    1e-12, so x and lambda carry relative errors up to kappa(A) * 1e-12; the
    bound below allows 4 kappa(A) * 1e-12."""
    torch, L = env
    from paper_1908_04081_amd.autograd import solve
    A = P.varcoef7(16, 1.0, 105)
    n = A.shape[0]
    b = P.rhs_normal(n, 1105)
    t = P.rhs_normal(n, 2105)
    x_ref, gb_ref, gval_ref = reference_gradient(A, b, t)
    pat = L.csr_to_device(A)
    val = pat.val.clone().requires_grad_(True)
    bt = torch.from_numpy(b).cuda().requires_grad_(True)
    x = solve(pat, val, bt, tol=1e-12, s_max=10, basis="chebyshev")
    loss = ((x - torch.from_numpy(t).cuda()) ** 2).sum()
    loss.backward()
    bound = 4 * _kappa(A) * 1e-12
    ex = np.linalg.norm(x.detach().cpu().numpy() - x_ref) / np.linalg.norm(x_ref)
    eb = np.linalg.norm(bt.grad.cpu().numpy() - gb_ref) / np.linalg.norm(gb_ref)
    ev = np.linalg.norm(val.grad.cpu().numpy() - gval_ref) / np.linalg.norm(gval_ref)
    assert ex <= bound and eb <= bound and ev <= 2 * bound, (ex, eb, ev, bound)


def test_gradient_central_differences_full_size(env):
    """The differentiable workload itself: varcoef7 128^3 (N = 2.1M),
    L = ||x - t||^2, t ~ N(0, 1), solves at 1e-12.  Central differences along
    16 random directions (8 symmetric directions in A's values, 8 in b),
    step 1e-5 of the norms.  The difference quotient carries the truncation
    error O(h^2) and the solve error of the two losses divided by h; 1e-4
    relative covers both here.  The adjoint right-hand side 2 (x - t) is not
    solvable to 1e-12 in FP64 by CG on this matrix: the forward solve must
    converge, and the adjoint must reach 1e-12 or at least the relative
    residual that plain HSCG on the GPU attains on the same right-hand side
    (when it stops above 1e-12 the solver reports STAGNATED, warns, and
    returns its iterate)."""
    torch, L = env
    from paper_1908_04081_amd.autograd import solve
    pr = P.make_config("varcoef7_128")
    A, b = pr.A, pr.b
    n = A.shape[0]
    t = torch.from_numpy(P.rhs_normal(n, 2105)).cuda()
    pat = L.csr_to_device(A)
    h = L.assg_create()
    L.assg_analyze(h, pat)
    opts = dict(tol=1e-12, s_max=10, basis="chebyshev")
    val0 = pat.val.clone()
    b0 = torch.from_numpy(b).cuda()

    def loss(val, bv):
        x = solve(pat, val, bv, handle=h, **opts)
        return ((x - t) ** 2).sum()

    import warnings

    from paper_1908_04081_amd.autograd import SolveStagnated, last_info
    val = val0.clone().requires_grad_(True)
    bt = b0.clone().requires_grad_(True)
    with warnings.catch_warnings(record=True) as caught:
        warnings.simplefilter("always")
        x = solve(pat, val, bt, handle=h, **opts)
        ((x - t) ** 2).sum().backward()
    fi, ai = last_info["forward"], last_info["adjoint"]
    assert fi["outcome"] == L.CONVERGED and fi["relres_true"] <= 1e-12, fi
    g = (2.0 * (x.detach() - t)).contiguous()
    lam = torch.zeros_like(g)
    hi = L.assg_hscg_solve(h, pat, g, lam, 1e-12, 0)
    print(f"adjoint: {ai['outcome_name']} {ai['relres_true']:.3e}; HSCG on the same "
          f"right-hand side: {hi['outcome_name']} {hi['relres_true']:.3e}", flush=True)
    assert ai["relres_true"] <= max(1e-12, hi["relres_true"]), (ai, hi)
    stagnated = [w for w in caught if issubclass(w.category, SolveStagnated)]
    assert bool(stagnated) == (ai["outcome"] == L.STAGNATED)
    gval, gb = val.grad.cpu().numpy(), bt.grad.cpu().numpy()
    worst = 0.0
    with torch.no_grad():
        for k in range(8):
            d = P.symmetric_direction(A, 300 + k)
            hv = 1e-5 * np.linalg.norm(A.data) / np.linalg.norm(d)
            dt = torch.from_numpy(hv * d).cuda()
            fd = (loss(val0 + dt, b0).item() - loss(val0 - dt, b0).item()) / (2 * hv)
            an = float(gval @ d)
            worst = max(worst, abs(fd - an) / abs(an))
            db = P.rhs_normal(n, 400 + k)
            hb = 1e-5 * np.linalg.norm(b) / np.linalg.norm(db)
            dbt = torch.from_numpy(hb * db).cuda()
            fd = (loss(val0, b0 + dbt).item() - loss(val0, b0 - dbt).item()) / (2 * hb)
            an = float(gb @ db)
            worst = max(worst, abs(fd - an) / abs(an))
            print(f"direction {k}: worst relative difference so far {worst:.2e}", flush=True)
    assert worst <= 1e-4, worst
    L.assg_destroy(h)
