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


def _geom_problem(n=100, cond=1e4, seed=1):
    """Diagonal SPD matrix with a geometric spectrum in [2/cond, 2]: CG's
    residual norm oscillates there, and the break (4.7) fires in many loops."""
    vals = np.geomspace(1.0 / cond, 1.0, n) * 2.0
    A = P.diagonal_matrix(vals)
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    b = np.random.default_rng(seed).standard_normal(n)
    return P.Problem(name="geom_100", A=A, b=b, x0=np.zeros(n))


@pytest.mark.parametrize("name,basis,sigma", [("poisson2d_64", "chebyshev", 10),
                                              ("poisson2d_64", "newton", 10),
                                              ("geom_100", "chebyshev", 10),
                                              ("geom_100", "newton", 15)])
def test_controller_replays_oracle_loops(env, name, basis, sigma):
    """The device controller, fed the oracle's G and carried state at every
    outer loop, reproduces s~, s_k (the break (4.7) and the stopping
    candidate), alpha/beta, the recovery coordinates, the Ritz estimates,
    psi, c and the next basis parameters.  On the geometric spectrum the
    break ends at least five loops."""
    torch, L, h = env
    pr = P.make_config("poisson2d_64") if name == "poisson2d_64" else _geom_problem()
    _, info = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=sigma, tol=1e-10, basis=basis,
                                  record_gram=True)
    nb = float(np.linalg.norm(pr.b))
    tr = info["trace"]
    breaks = sum(1 for rec in tr if rec["broke"])
    if name == "geom_100":
        assert breaks >= 5, breaks
    ties = compared_breaks = 0
    for k, rec in enumerate(tr):
        sbar = rec["sbar"]
        G = to_interleaved_matrix(rec["G"], sbar)
        S = block_state_from_oracle(L, rec["state_in"])
        res = L.assg_block_controller(h, G, sbar, nb, 1e-10, basis, sigma, S)
        if res.stilde != rec["stilde"]:
            # only where the deciding leading block of G is numerically
            # singular (smallest eigenvalue within rounding of 0, where the
            # sign, and so kappa = inf or not, is the eigensolver's): both
            # choices are correct and the rest of the loop differs
            l = min(res.stilde, rec["stilde"]) + 1
            ev = np.linalg.eigvalsh(rec["G"][np.ix_(O.sub_indices(sbar, l), O.sub_indices(sbar, l))])
            assert ev[0] <= 64 * 2.0 ** -53 * (2 * l + 1) * ev[-1], (k, res.stilde, rec["stilde"], ev[0], ev[-1])
            ties += 1
            continue
        assert res.stilde == rec["stilde"], (k, res.stilde, rec["stilde"])
        assert res.sk == rec["sk"], (k, res.sk, rec["sk"], rec["broke"])
        compared_breaks += bool(rec["broke"])
        assert bool(res.candidate) == bool(rec["candidate"])
        kap_o = np.array(rec["kappa"])
        kap_g = np.array(res.kappa[:sbar])
        # kappa(Y) = sqrt(kappa(G)); any backward-stable eigensolver gets
        # lambda_min(G) to about u*||G||, i.e. kappa(Y) to about u*kappa(G)
        fin = np.isfinite(kap_o) & (kap_o < 1e6)
        tol = 1e-12 + 16 * 2.0 ** -53 * kap_o[fin] ** 2
        assert np.all(np.abs(kap_g[fin] - kap_o[fin]) <= tol * kap_o[fin]), (k, kap_g, kap_o)
        # alpha, beta, the coordinates and what follows from them (psi, the
        # Ritz estimates, c, the next parameters) come from quadratic forms in
        # G over the selected basis: two summation orders differ by about
        # u * kappa(G_s~) = u * kappa(Y_{k,s~})^2 relative
        st = res.stilde
        rt = 16 * 2.0 ** -53 * rec["kappa"][st - 1] ** 2 if st > 1 else 0.0
        np.testing.assert_allclose(res.alpha[:res.sk], rec["alphas"], rtol=1e-12 + rt)
        np.testing.assert_allclose(res.beta[:res.sk], rec["betas"], rtol=1e-10 + rt)
        for field, key in (("coef_x", "xc"), ("coef_r", "rc"), ("coef_p", "pc")):
            got = np.array(getattr(res, field)[:2 * st + 1])
            ref = to_interleaved_vec(rec[key], st)
            assert np.abs(got - ref).max() <= (1e-10 + rt) * max(1.0, np.abs(ref).max()), \
                (k, field)
        if k + 1 < len(tr):
            nxt = tr[k + 1]["state_in"]
            np.testing.assert_allclose(S.psi, nxt["psi"], rtol=1e-10 + rt)
            np.testing.assert_allclose(S.c, nxt["c"], rtol=1e-10 + rt)
            if np.isfinite(nxt["lmax"]):
                np.testing.assert_allclose([S.lmin, S.lmax], [nxt["lmin"], nxt["lmax"]],
                                           rtol=1e-11 + rt)
                th = nxt["params"][0]
                np.testing.assert_allclose(np.array(S.theta[:th.size]), th, rtol=1e-11 + rt)
    assert ties <= len(tr) // 2, ties
    if name == "geom_100":
        assert compared_breaks >= 3, (breaks, compared_breaks, ties)


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


def _poisson3d_with_long_row(side=96, extra=3000, seed=5):
    """3-D 7-point Poisson on a 96^3 grid (884,736 rows: about 3,460 row
    blocks of at most 256 rows, so each of the fused last sweep's reduction
    chunks walks several blocks) with one row in the middle holding 3,000
    more off-diagonal entries (a row longer than a block's 2,048 nonzeros,
    so a block of its own inside a multi-block chunk), symmetric and
    diagonally dominant."""
    A = P.poisson3d(side).tocoo()
    n = A.shape[0]
    rng = np.random.default_rng(seed)
    i0 = n // 2 + 77
    cols = np.unique(rng.integers(0, n, extra))
    cols = cols[np.abs(cols - i0) > side * side]
    w = np.full(cols.size, -1e-4)
    rows = np.concatenate([A.row, np.full(cols.size, i0), cols, [i0], cols])
    cc = np.concatenate([A.col, cols, np.full(cols.size, i0), [i0], cols])
    vv = np.concatenate([A.data, w, w, [1e-4 * cols.size], np.full(cols.size, 1e-4)])
    M = sp.csr_matrix((vv, (rows, cc)), shape=(n, n))
    M.sum_duplicates()
    M.sort_indices()
    M.indices = M.indices.astype(np.int32)
    M.indptr = M.indptr.astype(np.int32)
    assert np.diff(M.indptr)[i0] > 2048
    return M


@pytest.mark.parametrize("s", [3, 10])
def test_basis_and_gram_many_blocks_per_chunk(env, s):
    """The fused last sweep with several row blocks per reduction chunk (the
    prefetch of the next block's nonzeros and bounds, the LDS tile reused
    across blocks, the chunk's Gram accumulated over its blocks) and a long
    row inside such a chunk: every basis column and every entry of G against
    the oracle, element-wise, as for the small matrices."""
    torch, L, h = env
    A = _poisson3d_with_long_row()
    n = A.shape[0]
    Ad = _dev(torch, L, h, A)
    rng = np.random.default_rng(300 + s)
    p, r = rng.standard_normal(n), rng.standard_normal(n)
    prm = O.make_params("chebyshev", s, 0.01, 1.99)
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
