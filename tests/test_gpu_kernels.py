"""GPU parity of single steps of the hot path, through the C ABI, against the
CPU oracle on the same seeded inputs (sizes spanning several tiles with a
ragged tail)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import spd_problems as P
from gpu_util import (block_state_from_oracle, interleave_perm, to_interleaved_matrix,
                      to_interleaved_vec, torch_cuda)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = torch_cuda()
    import paper_1908_04081_amd as L
    L.lib()
    h = L.assg_create()
    yield torch, L, h
    L.assg_destroy(h)


def _ragged_spd(n=3001, seed=7):
    """SPD with ragged row lengths: a random sparse pattern, one long row and
    one dense-ish column, made diagonally dominant."""
    rng = np.random.default_rng(seed)
    nnz_off = 6 * n
    i = rng.integers(0, n, nnz_off)
    j = rng.integers(0, n, nnz_off)
    i = np.concatenate([i, np.full(400, 17), rng.integers(0, n, 300)])
    j = np.concatenate([j, rng.integers(0, n, 400), np.full(300, 5)])
    v = rng.uniform(-1, 1, i.size)
    M = sp.coo_matrix((v, (i, j)), shape=(n, n)).tocsr()
    M = M + M.T
    d = np.asarray(abs(M).sum(axis=1)).ravel() + 0.5
    M = (M + sp.diags(d)).tocsr()
    M.sort_indices()
    M.indices = M.indices.astype(np.int32)
    M.indptr = M.indptr.astype(np.int32)
    return P.diag_scale(M)


def _arrow_spd(n=6000):
    """Arrow matrix: row/column 0 dense (a row longer than a workgroup's
    nonzero block), unit-diagonal-dominant otherwise."""
    rows = np.concatenate([np.zeros(n - 1, dtype=np.int64), np.arange(1, n), np.arange(n)])
    cols = np.concatenate([np.arange(1, n), np.zeros(n - 1, dtype=np.int64), np.arange(n)])
    vals = np.concatenate([np.full(n - 1, -0.5 / n), np.full(n - 1, -0.5 / n),
                           np.linspace(1.0, 2.0, n)])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    M.sort_indices()
    M.indices = M.indices.astype(np.int32)
    M.indptr = M.indptr.astype(np.int32)
    return M


PROBLEMS = {
    "arrow_6000": lambda: _arrow_spd(6000),
    "poisson2d_64": lambda: P.poisson2d(64),
    "poisson2d_37": lambda: P.poisson2d(37),
    "poisson3d_21": lambda: P.poisson3d(21),
    "diffusion27_13": lambda: P.diffusion27(13, 2.0, 103),
    "varcoef7_11": lambda: P.varcoef7(11, 1.0, 105),
    "ragged_3001": lambda: _ragged_spd(3001),
    "one_row": lambda: sp.csr_matrix(np.array([[2.0]])),
}


def _dev(torch, L, h, A):
    Ad = L.csr_to_device(A)
    L.assg_analyze(h, Ad)
    return Ad


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_spmv_matches_scipy(env, name):
    torch, L, h = env
    A = PROBLEMS[name]()
    Ad = _dev(torch, L, h, A)
    x = np.random.default_rng(1).standard_normal(A.shape[0])
    y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    L.assg_spmv(h, Ad, torch.from_numpy(x).cuda(), y)
    ref = A @ x
    scale = abs(A) @ np.abs(x)
    err = np.abs(y.cpu().numpy() - ref)
    assert np.all(err <= 1e-14 * scale + 1e-300), float((err / (scale + 1e-300)).max())


@pytest.mark.parametrize("name", sorted(PROBLEMS))
def test_spmv_bitwise_in_row_order(env, name):
    """Rows of at most 2048 nonzeros are summed product by product in column
    order, which is scipy's sequential CSR product: bit-identical results."""
    torch, L, h = env
    A = PROBLEMS[name]()
    Ad = _dev(torch, L, h, A)
    x = np.random.default_rng(2).standard_normal(A.shape[0])
    y = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
    L.assg_spmv(h, Ad, torch.from_numpy(x).cuda(), y)
    short = np.diff(A.indptr) <= 2048
    assert np.array_equal(y.cpu().numpy()[short], (A @ x)[short])


@pytest.mark.parametrize("name", ["poisson2d_37", "poisson3d_21", "diffusion27_13", "ragged_3001",
                                  "arrow_6000"])
@pytest.mark.parametrize("basis", ["monomial", "newton", "chebyshev"])
@pytest.mark.parametrize("s", [1, 3, 10, 16])
def test_basis_and_gram_match_oracle(env, name, basis, s):
    """(2.2)-(2.3) basis columns and G = Y^T Y against the oracle (same
    parameters), plus the change-of-basis identity (2.4) on the GPU basis."""
    torch, L, h = env
    A = PROBLEMS[name]()
    n = A.shape[0]
    Ad = _dev(torch, L, h, A)
    rng = np.random.default_rng(s + 17)
    p, r = rng.standard_normal(n), rng.standard_normal(n)
    prm = O.make_params(basis, s, 0.05, 1.9)
    Yg = torch.empty((2 * s + 1, n), dtype=torch.float64, device="cuda")
    Gg = L.assg_basis_gram(h, Ad, torch.from_numpy(p).cuda(), torch.from_numpy(r).cuda(), s,
                           *prm, Y_out=Yg)
    Yg = Yg.cpu().numpy().T                                   # n x (2s+1), interleaved
    Yo = O.sstep_basis(A, p, r, s, prm)[:, interleave_perm(s)]
    cn = np.linalg.norm(Yo, axis=0)
    colerr = np.linalg.norm(Yg - Yo, axis=0) / cn
    assert colerr.max() <= 1e-12, colerr
    Go = Yo.T @ Yo
    scale = np.sqrt(np.outer(np.diag(Go), np.diag(Go)))
    assert np.abs(Gg - Go).max() / 1.0 <= (1e-12 * scale).max()
    assert np.all(np.abs(Gg - Go) <= 1e-12 * scale)
    assert np.array_equal(Gg, Gg.T)
    # (2.4) on the GPU basis: A Y_ = Y B (interleaved: zero columns 2s-1 and 2s)
    B = O.change_of_basis(s, prm)
    pi = interleave_perm(s)
    Bi = B[np.ix_(pi, pi)]
    Yu = Yg.copy(); Yu[:, 2 * s] = 0.0; Yu[:, 2 * s - 1] = 0.0
    res = np.linalg.norm(A @ Yu - Yg @ Bi) / np.linalg.norm(Yg)
    assert res <= 1e-14


@pytest.mark.parametrize("basis", ["chebyshev", "newton"])
def test_controller_replays_oracle_loops(env, basis):
    """The device controller, fed the oracle's G and carried state at every
    outer loop, reproduces s~, s_k, alpha/beta, the recovery coordinates, the
    Ritz estimates, psi, c and the next basis parameters."""
    torch, L, h = env
    pr = P.make_config("poisson2d_64")
    _, info = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10, basis=basis,
                                  record_gram=True)
    nb = float(np.linalg.norm(pr.b))
    tr = info["trace"]
    for k, rec in enumerate(tr):
        sbar = rec["sbar"]
        G = to_interleaved_matrix(rec["G"], sbar)
        S = block_state_from_oracle(L, rec["state_in"])
        res = L.assg_block_controller(h, G, sbar, nb, 1e-10, basis, 10, S)
        assert res.stilde == rec["stilde"], (k, res.stilde, rec["stilde"])
        assert res.sk == rec["sk"], (k, res.sk, rec["sk"])
        assert bool(res.candidate) == bool(rec["candidate"])
        kap_o = np.array(rec["kappa"])
        kap_g = np.array(res.kappa[:sbar])
        # kappa(Y) = sqrt(kappa(G)); any backward-stable eigensolver gets
        # lambda_min(G) to about u*||G||, i.e. kappa(Y) to about u*kappa(G)
        fin = np.isfinite(kap_o) & (kap_o < 1e6)
        tol = 1e-12 + 16 * 2.0 ** -53 * kap_o[fin] ** 2
        assert np.all(np.abs(kap_g[fin] - kap_o[fin]) <= tol * kap_o[fin]), (k, kap_g, kap_o)
        np.testing.assert_allclose(res.alpha[:res.sk], rec["alphas"], rtol=1e-12)
        np.testing.assert_allclose(res.beta[:res.sk], rec["betas"], rtol=1e-10)
        st = res.stilde
        for name, key in (("coef_x", "xc"), ("coef_r", "rc"), ("coef_p", "pc")):
            got = np.array(getattr(res, name)[:2 * st + 1])
            ref = to_interleaved_vec(rec[key], st)
            assert np.abs(got - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max()), (k, name)
        if k + 1 < len(tr):
            nxt = tr[k + 1]["state_in"]
            np.testing.assert_allclose(S.psi, nxt["psi"], rtol=1e-10)
            np.testing.assert_allclose(S.c, nxt["c"], rtol=1e-10)
            if np.isfinite(nxt["lmax"]):
                np.testing.assert_allclose([S.lmin, S.lmax], [nxt["lmin"], nxt["lmax"]],
                                           rtol=1e-11)
                th = nxt["params"][0]
                np.testing.assert_allclose(np.array(S.theta[:th.size]), th, rtol=1e-11)


@pytest.mark.parametrize("name", ["poisson3d_21", "ragged_3001"])
@pytest.mark.parametrize("s", list(range(1, 17)))
def test_basis_and_gram_every_s(env, name, s):
    """Every s = 1..16 has its own instance of the fused last sweep (2s+1
    columns on the matrix cores in 1, 2 or 3 groups of 16): basis columns
    and G against the oracle for each, Chebyshev parameters."""
    torch, L, h = env
    A = PROBLEMS[name]()
    n = A.shape[0]
    Ad = _dev(torch, L, h, A)
    rng = np.random.default_rng(100 + s)
    p, r = rng.standard_normal(n), rng.standard_normal(n)
    prm = O.make_params("chebyshev", s, 0.05, 1.9)
    Yg = torch.empty((2 * s + 1, n), dtype=torch.float64, device="cuda")
    Gg = L.assg_basis_gram(h, Ad, torch.from_numpy(p).cuda(), torch.from_numpy(r).cuda(), s,
                           *prm, Y_out=Yg)
    Yo = O.sstep_basis(A, p, r, s, prm)[:, interleave_perm(s)]
    colerr = np.linalg.norm(Yg.cpu().numpy().T - Yo, axis=0) / np.linalg.norm(Yo, axis=0)
    assert colerr.max() <= 1e-12, colerr
    Go = Yo.T @ Yo
    scale = np.sqrt(np.outer(np.diag(Go), np.diag(Go)))
    assert np.all(np.abs(Gg - Go) <= 1e-12 * scale)
    assert np.array_equal(Gg, Gg.T)
