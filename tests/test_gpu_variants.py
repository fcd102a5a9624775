"""The comparison methods of Section 5 on the GPU (the same kernels, the
controller switching its s-selection, c and break rules) against the
oracle's variants."""
import numpy as np
import pytest

import oracle as O
import spd_problems as P
from gpu_util import check_outer_parity, torch_cuda

pytestmark = pytest.mark.gpu

OUTCOME = {O.Outcome.CONVERGED: 0, O.Outcome.STAGNATED: 1, O.Outcome.DIVERGED: 2,
           O.Outcome.BREAKDOWN: 3, O.Outcome.MAX_ITER: 4}


@pytest.fixture(scope="module")
def env():
    torch = torch_cuda()
    import paper_1908_04081_amd as L
    L.lib()
    h = L.assg_create()
    yield torch, L, h
    L.assg_destroy(h)


def _problem(name):
    if name == "poisson2d_45":
        return P.make_config("poisson2d_64", size=45)
    if name == "poisson2d_64":
        return P.make_config("poisson2d_64")
    return P.make_config("varcoef7_128", size=10)


def _gpu(torch, L, h, pr, **opts):
    Ad = L.csr_to_device(pr.A)
    L.assg_analyze(h, Ad)
    b = torch.from_numpy(pr.b).cuda()
    x = torch.zeros_like(b)
    info = L.assg_solve(h, Ad, b, x, L.assg_default_opts(**opts))
    return x.cpu().numpy(), info


@pytest.mark.parametrize("name", ["poisson2d_45", "varcoef7_10"])
@pytest.mark.parametrize("variant", ["improved_c_ratio", "improved_c_one", "old", "fixed"])
@pytest.mark.parametrize("sigma", [5, 10])
def test_variant_matches_oracle(env, name, variant, sigma):
    torch, L, h = env
    pr = _problem(name)
    kw = dict(s_max=sigma, tol=1e-10, basis="chebyshev", variant=variant, max_outer=3000)
    xo, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, **kw)
    xg, ig = _gpu(torch, L, h, pr, s_init=sigma, growth=sigma, record_trace=1, **kw)
    assert ig["outcome"] == OUTCOME[io["outcome"]], (ig["outcome_name"], io["outcome"])
    if io["outcome"] != O.Outcome.CONVERGED:
        return
    rel = np.linalg.norm(pr.b - pr.A @ xg) / np.linalg.norm(pr.b)
    assert rel <= 1e-10
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 1e-8
    check_outer_parity(torch, L, h, pr, ig, xo, io, dict(s_init=sigma, growth=sigma, **kw),
                       tg=L.assg_get_trace(h), case=f"variant {name} {variant} sigma={sigma}")


def test_fixed_sstep_breaks_down_at_s15(env):
    """sigma = 15 on the 64 x 64 Poisson workload: the monomial basis of
    fixed s-step CG is numerically singular, and both sides break down.  The
    Gram matrix's condition number is far beyond 1/eps, so the loop in which
    a quadratic form first comes out non-positive is set by rounding (the
    order of the Gram sums); only the outcome, and that it comes long before
    a converging run would finish (HSCG needs about 18 loops' worth of
    iterations), are compared."""
    torch, L, h = env
    pr = _problem("poisson2d_64")
    kw = dict(s_max=15, tol=1e-10, variant="fixed", max_outer=3000)
    _, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, **kw)
    _, ig = _gpu(torch, L, h, pr, s_init=15, growth=15, **kw)
    assert io["outcome"] == O.Outcome.BREAKDOWN and io["outer"] < 6
    assert ig["outcome"] == L.BREAKDOWN and ig["outer_iters"] < 6, ig


def test_old_adaptive_at_s15_follows_oracle_until_singular(env):
    """Algorithm 2 (monomial basis, c = 1) at sigma = 15 on the 64 x 64
    Poisson workload.  With c = 1 the bound of (3.2), eps*/(eps rho), grows as
    the residual falls, so the method selects monomial bases whose Gram
    matrix has kappa(G) = kappa(Y)^2 >= 1/eps: from that loop on the computed
    G no longer carries Y's conditioning (its small eigenvalues are
    rounding), and s~, the break and the iterates are set by the order of the
    Gram sums.  Compared: (i) the oracle's run reaches that regime before it
    converges (the defect of the old method that Section 5 shows);
    (ii) s-bar, s~ and s_k of every loop before the first such loop are the
    same on both sides (loop 0, where p = r makes every basis exactly
    singular, included); (iii) afterwards only validity: a GPU run that
    reports convergence meets the tolerance on the host; (iv) Algorithm 5 on
    the same workload stays within 5% of HSCG's iterations."""
    torch, L, h = env
    pr = _problem("poisson2d_64")
    xh, ih = O.hscg(pr.A, pr.b, pr.x0, tol=1e-10)
    kw = dict(s_max=15, tol=1e-10, variant="old", max_outer=3000)
    _, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, **kw)
    xg, ig = _gpu(torch, L, h, pr, s_init=15, growth=15, record_trace=1, **kw)
    tg = L.assg_get_trace(h)
    to = io["trace"]
    u = 2.0 ** -53
    # loops whose selected basis is numerically singular (loop 0 aside: there
    # p = r, every Y_{0,l} is exactly singular and s~ = 1 on any machine)
    sing = [k for k, rec in enumerate(to)
            if k > 0 and rec["kappa"][rec["stilde"] - 1] ** 2 >= 1.0 / u]
    assert sing and sing[0] < len(to) - 1, "the oracle never reached kappa(G) >= 1/eps"
    k_sing = sing[0]
    assert len(tg) > k_sing
    for k in range(k_sing):
        assert (tg[k]["sbar"], tg[k]["stilde"], tg[k]["sk"]) == \
            (to[k]["sbar"], to[k]["stilde"], to[k]["sk"]), (k, tg[k], to[k]["stilde"])
    if ig["outcome"] == L.CONVERGED:
        assert np.linalg.norm(pr.b - pr.A @ xg) / np.linalg.norm(pr.b) <= 1e-10
    _, ii = _gpu(torch, L, h, pr, s_max=15, s_init=15, growth=15, tol=1e-10)
    assert ii["outcome"] == L.CONVERGED and ii["total_iters"] <= 1.05 * ih["iters"]


def test_bad_variant_options_are_rejected(env):
    torch, L, h = env
    pr = _problem("poisson2d_45")
    with pytest.raises(L.AssgError):
        _gpu(torch, L, h, pr, variant=7)
    with pytest.raises(L.AssgError):
        _gpu(torch, L, h, pr, variant="old", c_const=0.0)
