"""Batched solves (many systems per launch, captured outer loops) through the
C ABI: every system against the oracle on small batches, and the batched
workload itself (64 systems, sides 32..512) by properties checked on the
host."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import spd_problems as P
from gpu_util import check_outer_parity, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = torch_cuda()
    import paper_1908_04081_amd as L
    L.lib()
    h = L.assg_create()
    yield torch, L, h
    L.assg_destroy(h)


def _mixed_batch():
    """Uneven sizes and kinds: shifted 2D Poisson, scaled 3D Poisson, a
    27-point lognormal diffusion and a variable-coefficient 7-point operator."""
    out = P.make_batch(count=4, lo=12, hi=40, seed=7)
    for pr in (P.make_config("poisson3d_256", size=9), P.make_config("diffusion27_160", size=7),
               P.make_config("varcoef7_128", size=8)):
        out.append(pr)
    return out


def _run(torch, L, h, probs, **opts):
    As = [L.csr_to_device(pr.A) for pr in probs]
    L.assg_batch_analyze(h, As)
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    xs = [torch.from_numpy(pr.x0.copy()).cuda() for pr in probs]
    infos = L.assg_batch_solve(h, As, bs, xs, L.assg_default_opts(**opts))
    return [x.cpu().numpy() for x in xs], infos


@pytest.mark.parametrize("basis", ["chebyshev", "newton"])
@pytest.mark.parametrize("sigma", [5, 10])
def test_batch_matches_oracle_per_system(env, basis, sigma):
    torch, L, h = env
    probs = _mixed_batch()
    tol = 1e-10
    xs, infos = _run(torch, L, h, probs, s_max=sigma, s_init=sigma, growth=sigma, tol=tol,
                     basis=basis)
    for pr, xg, ig in zip(probs, xs, infos):
        xo, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=sigma, tol=tol, basis=basis)
        assert io["outcome"] == O.Outcome.CONVERGED
        assert ig["outcome"] == L.CONVERGED, (pr.name, ig)
        rel = np.linalg.norm(pr.b - pr.A @ xg) / np.linalg.norm(pr.b)
        assert rel <= tol, (pr.name, rel)
        assert abs(ig["relres_true"] - rel) <= 1e-3 * rel
        err = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
        assert err <= 1e-8, (pr.name, err)
        check_outer_parity(torch, L, h, pr, ig, xo, io,
                           dict(s_max=sigma, s_init=sigma, growth=sigma, tol=tol, basis=basis),
                           case=f"batch {pr.name} {basis} sigma={sigma}")


def test_batch_zero_rhs_and_breakdown_are_per_system(env):
    """A zero right-hand side gives x = 0 at once and a non-SPD system breaks
    down, while the other systems of the batch still converge."""
    torch, L, h = env
    probs = P.make_batch(count=3, lo=16, hi=24, seed=9)
    z = probs[1]
    probs[1] = P.Problem(name="zero_rhs", A=z.A, b=np.zeros(z.n), x0=np.ones(z.n))
    n = 30
    M = sp.diags([np.r_[np.ones(n - 1), -1.0]], [0], format="csr")   # indefinite
    M.sort_indices()
    M = sp.csr_matrix((M.data, M.indices.astype(np.int32), M.indptr.astype(np.int32)), shape=M.shape)
    probs.append(P.Problem(name="indefinite", A=M, b=np.ones(n), x0=np.zeros(n)))
    xs, infos = _run(torch, L, h, probs, s_max=10, tol=1e-10)
    assert infos[1]["outcome"] == L.CONVERGED and infos[1]["outer_iters"] == 0
    assert np.all(xs[1] == 0.0) and infos[1]["relres_true"] == 0.0
    assert infos[3]["outcome"] in (L.BREAKDOWN, L.DIVERGED, L.STAGNATED, L.MAX_ITER)
    for i in (0, 2):
        pr = probs[i]
        assert infos[i]["outcome"] == L.CONVERGED
        assert np.linalg.norm(pr.b - pr.A @ xs[i]) / np.linalg.norm(pr.b) <= 1e-10


def test_batch_repeat_is_deterministic(env):
    """Two solves after one analysis are bitwise identical.  (A new analysis
    may pick another row-block shape by timing, and with it another grouping
    of the Gram partial sums, so only the same analysis fixes the rounding.)"""
    torch, L, h = env
    probs = _mixed_batch()
    As = [L.csr_to_device(pr.A) for pr in probs]
    L.assg_batch_analyze(h, As)
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    runs = []
    for _ in range(2):
        xs = [torch.from_numpy(pr.x0.copy()).cuda() for pr in probs]
        infos = L.assg_batch_solve(h, As, bs, xs, L.assg_default_opts(s_max=10, tol=1e-10))
        runs.append(([x.cpu().numpy() for x in xs], infos))
    (x1, i1), (x2, i2) = runs
    for a, b_, p, q in zip(x1, x2, i1, i2):
        assert np.array_equal(a, b_)
        assert p["outer_iters"] == q["outer_iters"]


def test_batched_workload_full_size(env):
    """64 shifted 2D Poisson systems, sides 32..512 (6.2M rows in all), random
    normal right-hand sides, tol 1e-10: every system converges with true
    relative residual <= 1e-10 recomputed on the host; the ten smallest
    against the oracle; the tuner reports every size class present with a
    pick among its candidates (timed, or from the process cache)."""
    torch, L, h = env
    probs = P.make_batch()
    xs, infos = _run(torch, L, h, probs, s_max=10, tol=1e-10)
    tune = L.assg_batch_tuning(h)
    classes = [0 if pr.n < 4096 else 1 if pr.n < 65536 else 2 if pr.n < 1048576 else 3
               for pr in probs]
    for cl, t in enumerate(tune):
        assert t["systems"] == classes.count(cl)
        if t["systems"]:
            assert (t["rows"], t["nnz_cap"]) in L.TUNE_SHAPES
            us = list(t["candidates_us"].values())
            assert all(v == 0 for v in us) if t["cached"] else all(v > 0 for v in us)
    for pr, xg, ig in zip(probs, xs, infos):
        assert ig["outcome"] == L.CONVERGED, (pr.name, ig)
        rel = np.linalg.norm(pr.b - pr.A @ xg) / np.linalg.norm(pr.b)
        assert rel <= 1e-10, (pr.name, rel)
    order = np.argsort([pr.n for pr in probs])[:10]
    for i in order:
        pr = probs[i]
        xo, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10, basis="chebyshev")
        assert np.linalg.norm(xs[i] - xo) / np.linalg.norm(xo) <= 1e-8
        check_outer_parity(torch, L, h, pr, infos[i], xo, io,
                           dict(s_max=10, tol=1e-10, basis="chebyshev"),
                           case=f"batched workload {pr.name}")


def test_batch_at_maximum_size(env):
    """ASSG_MAX_BATCH = 2048 small systems (2D Poisson, sides 2..6, shifted)
    in one batch: every system converges with true relative residual <= tol
    recomputed on the host, every 64th against the oracle; one system more
    is refused."""
    torch, L, h = env
    probs = P.make_batch(count=2048, lo=2, hi=6, seed=11)
    As = [L.csr_to_device(pr.A) for pr in probs]
    L.assg_batch_analyze(h, As)
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    xs = [torch.from_numpy(pr.x0.copy()).cuda() for pr in probs]
    infos = L.assg_batch_solve(h, As, bs, xs, L.assg_default_opts(tol=1e-10))
    for pr, x, ig in zip(probs, xs, infos):
        assert ig["outcome"] == L.CONVERGED, (pr.name, ig)
        xg = x.cpu().numpy()
        assert np.linalg.norm(pr.b - pr.A @ xg) / np.linalg.norm(pr.b) <= 1e-10
    for i in range(0, 2048, 64):
        pr = probs[i]
        xo, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10)
        assert abs(infos[i]["outer_iters"] - io["outer"]) <= 1, (i, infos[i], io["outer"])
        xg = xs[i].cpu().numpy()
        assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 1e-8
    with pytest.raises(L.AssgError, match="nsys"):
        L.assg_batch_analyze(h, As + As[:1])


def test_tuner_cache_reuses_choices(env):
    """A second analysis of a batch with the same size classes and nonzeros
    per row takes every class's shape from the process cache (no timing),
    and the same shapes; the solve is unchanged."""
    torch, L, h = env
    probs = P.make_batch(count=6, lo=40, hi=300, seed=21)
    As = [L.csr_to_device(pr.A) for pr in probs]
    L.assg_batch_analyze(h, As)
    first = L.assg_batch_tuning(h)
    L.assg_batch_analyze(h, As)
    second = L.assg_batch_tuning(h)
    for a, b in zip(first, second):
        assert a["systems"] == b["systems"]
        if a["systems"]:
            assert b["cached"] and (a["rows"], a["nnz_cap"]) == (b["rows"], b["nnz_cap"])
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    xs = [torch.zeros_like(b) for b in bs]
    infos = L.assg_batch_solve(h, As, bs, xs, L.assg_default_opts(s_max=10, tol=1e-10))
    for pr, x, ig in zip(probs, xs, infos):
        assert ig["outcome"] == L.CONVERGED
        xg = x.cpu().numpy()
        assert np.linalg.norm(pr.b - pr.A @ xg) / np.linalg.norm(pr.b) <= 1e-10
