"""The diagonal storage of stencil matrices (assg_set_format): which storage
the analysis picks, and that the kernels reading it give the CSR kernels'
results (bit for bit where both storages cut the rows into the same blocks)
and the oracle's, with values refreshed on every call."""
import numpy as np
import pytest
import scipy.sparse as sp

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
    L.assg_set_format(h, "auto")
    L.assg_destroy(h)


def _analyze(L, h, Ad, fmt):
    L.assg_set_format(h, fmt)
    try:
        L.assg_analyze(h, Ad)
    finally:
        L.assg_set_format(h, "auto")
    return L.assg_get_format(h)


def _random_spd(n, seed):
    """Random sparse SPD matrix whose entries lie on far more than 32
    diagonals."""
    rng = np.random.default_rng(seed)
    R = sp.random(n, n, density=8.0 / n, random_state=rng, format="csr")
    A = (R + R.T + sp.diags(np.full(n, 20.0))).tocsr()
    A.sort_indices()
    return A


def test_format_choice(env):
    torch, L, h = env
    assert L.lib().assg_set_format(h.ptr, 7) == L.ERR_INVALID_ARG
    pr = P.make_config("poisson3d_256", size=20)
    Ad = L.csr_to_device(pr.A)
    assert _analyze(L, h, Ad, "auto") == "dia"
    assert _analyze(L, h, Ad, "csr") == "csr"
    assert _analyze(L, h, Ad, "dia") == "dia"
    R = _random_spd(3000, 7)
    Rd = L.csr_to_device(R)
    assert _analyze(L, h, Rd, "auto") == "csr"
    with pytest.raises(L.AssgError, match="unsupported"):
        _analyze(L, h, Rd, "dia")
    with pytest.raises(L.AssgError):            # a failed analysis leaves none behind
        L.assg_get_format(h)
    # a tridiagonal matrix with one far pair of entries in a row the
    # analysis does not sample: the probe finds it, AUTO falls back to CSR
    n = 5000
    T = sp.diags([np.full(n - 1, -1.0), np.full(n, 4.0), np.full(n - 1, -1.0)], [-1, 0, 1],
                 format="lil")
    T[1234, 4321] = T[4321, 1234] = -0.5
    T = T.tocsr()
    T.sort_indices()
    Td = L.csr_to_device(T)
    assert _analyze(L, h, Td, "auto") == "csr"
    with pytest.raises(L.AssgError):
        _analyze(L, h, Td, "dia")
    # the diagonals of a 27-point stencil are 27 of 32 allowed; on a 12^3
    # grid the boundary rows leave 19% of their positions empty, more than
    # AUTO accepts, on 30^3 7%
    D = P.make_config("diffusion27_160", size=12)
    assert _analyze(L, h, L.csr_to_device(D.A), "auto") == "csr"
    assert _analyze(L, h, L.csr_to_device(D.A), "dia") == "dia"
    D = P.make_config("diffusion27_160", size=30)
    assert _analyze(L, h, L.csr_to_device(D.A), "auto") == "dia"


def _basis_gram(torch, L, h, Ad, n, s, fmt, seed=3):
    rng = np.random.default_rng(seed)
    p = torch.from_numpy(rng.standard_normal(n)).cuda()
    r = torch.from_numpy(rng.standard_normal(n)).cuda()
    _analyze(L, h, Ad, fmt)
    Y = torch.empty((2 * s + 1, n), dtype=torch.float64, device="cuda")
    G = L.assg_basis_gram(h, Ad, p, r, s, *O.make_params("chebyshev", s, 0.05, 1.95), Y_out=Y)
    return G, Y.cpu().numpy()


@pytest.mark.parametrize("name,size,same_blocks", [("poisson3d_256", 40, True),
                                                   ("poisson2d_64", 50, True),
                                                   ("diffusion27_160", 18, False)])
@pytest.mark.parametrize("s", [3, 10, 16])
def test_basis_and_gram_equal_csr(env, name, size, same_blocks, s):
    """Every basis row is bit-identical; the Gram matrix too when the two
    storages cut the rows alike (at most 8 entries per row), else to the
    rounding of a regrouped sum; and it matches Y^T Y of the oracle's basis."""
    torch, L, h = env
    pr = P.make_config(name, size=size)
    Ad = L.csr_to_device(pr.A)
    Gc, Yc = _basis_gram(torch, L, h, Ad, pr.n, s, "csr")
    Gd, Yd = _basis_gram(torch, L, h, Ad, pr.n, s, "dia")
    assert np.array_equal(Yc, Yd)
    if same_blocks:
        assert np.array_equal(Gc, Gd)
    sc = np.sqrt(np.outer(np.diag(Gc), np.diag(Gc)))
    assert np.max(np.abs(Gd - Gc) / sc) <= 1e-14
    Gr = Yd @ Yd.T
    assert np.max(np.abs(Gd - Gr) / sc) <= 1e-12


def _banded_spd(n, offsets, seed):
    """Symmetric matrix with full diagonals at the given positive offsets
    (and their mirrors), random off-diagonal values and a dominant diagonal:
    SPD."""
    rng = np.random.default_rng(seed)
    A = sp.diags([np.full(n, 2.0 * len(offsets) + 1.0)], [0], format="lil").tocsr()
    for o in offsets:
        v = rng.uniform(-1.0, 1.0, n - o)
        A = A + sp.diags([v, v], [o, -o], shape=(n, n), format="csr")
    A = A.tocsr()
    A.sort_indices()
    return A


@pytest.mark.parametrize("s", [4, 10])
def test_irregular_diagonals_bit_identical_to_csr(env, s):
    """Offsets with runs of consecutive diagonals of several lengths (whose
    source entries the sweeps pass between lanes), runs that cross the groups
    of eight diagonals the kernels load at a time, isolated diagonals, and a
    ragged row count: every basis row equals the CSR kernels' bit for bit,
    and the Gram matrix matches Y^T Y."""
    torch, L, h = env
    n = 3001
    A = _banded_spd(n, [1, 6, 7, 50, 297, 298, 299, 300], seed=11)
    offs = np.unique(np.concatenate([A.indices[A.indptr[i]:A.indptr[i + 1]] - i
                                     for i in (0, 1500, n - 1)]))
    assert len(offs) == 17
    Ad = L.csr_to_device(A)
    assert _analyze(L, h, Ad, "auto") == "dia"
    Gc, Yc = _basis_gram(torch, L, h, Ad, n, s, "csr", seed=5)
    Gd, Yd = _basis_gram(torch, L, h, Ad, n, s, "dia", seed=5)
    assert np.array_equal(Yc, Yd)
    sc = np.sqrt(np.outer(np.diag(Gc), np.diag(Gc)))
    assert np.max(np.abs(Gd - Gc) / sc) <= 1e-14
    assert np.max(np.abs(Gd - Yd @ Yd.T) / sc) <= 1e-12


def _solve(torch, L, h, pr, fmt, **opts):
    Ad = L.csr_to_device(pr.A)
    assert _analyze(L, h, Ad, fmt) == fmt
    b = torch.from_numpy(pr.b).cuda()
    x = torch.zeros_like(b)
    info = L.assg_solve(h, Ad, b, x, L.assg_default_opts(**opts))
    xh = torch.zeros_like(b)
    ih = L.assg_hscg_solve(h, Ad, b, xh, opts["tol"], 0)
    return x.cpu().numpy(), info, xh.cpu().numpy(), ih


@pytest.mark.parametrize("basis", ["chebyshev", "newton"])
@pytest.mark.parametrize("name,size", [("poisson3d_256", 24), ("poisson2d_64", None)])
def test_solves_bit_identical_to_csr(env, basis, name, size):
    """7- and 5-point stencils: both storages give 256-row blocks, so
    Algorithm 5 and HSCG take the same roundings in the same order."""
    torch, L, h = env
    pr = P.make_config(name, size=size)
    opts = dict(s_max=10, tol=1e-10, basis=basis)
    xc, ic, hc, ihc = _solve(torch, L, h, pr, "csr", **opts)
    xd, id_, hd, ihd = _solve(torch, L, h, pr, "dia", **opts)
    assert ic["outcome"] == id_["outcome"] == L.CONVERGED
    for k in ("outer_iters", "total_iters", "relres_true", "relres_updated", "lambda_min_est",
              "lambda_max_est", "c_last"):
        assert ic[k] == id_[k], k
    assert np.array_equal(xc, xd)
    assert ihc["total_iters"] == ihd["total_iters"] and ihc["relres_true"] == ihd["relres_true"]
    assert np.array_equal(hc, hd)


@pytest.mark.parametrize("basis", ["chebyshev", "newton"])
def test_27_point_solves_match_oracle_in_both_storages(env, basis):
    """27-point diffusion: the storages group the Gram sums differently, so
    each is held to the oracle (same iteration counts, solution to 1e-8)."""
    torch, L, h = env
    pr = P.make_config("diffusion27_160", size=14)
    xo, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10, basis=basis)
    _, ih = O.hscg(pr.A, pr.b, pr.x0, tol=1e-10)
    for fmt in ("csr", "dia"):
        x, info, xh, ihg = _solve(torch, L, h, pr, fmt, s_max=10, tol=1e-10, basis=basis)
        assert info["outcome"] == L.CONVERGED, (fmt, info)
        assert abs(info["outer_iters"] - io["outer"]) <= 1, fmt
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-8, fmt
        assert np.linalg.norm(pr.b - pr.A @ x) / np.linalg.norm(pr.b) <= 1e-10
        assert abs(ihg["total_iters"] - ih["iters"]) <= 1, fmt
        assert np.linalg.norm(pr.b - pr.A @ xh) / np.linalg.norm(pr.b) <= 1e-10


def test_values_refreshed_every_solve(env):
    """The diagonal storage is refilled from the CSR values at each call:
    values changed on the device after the analysis are the ones solved
    with, for Algorithm 5, HSCG and assg_basis_gram."""
    torch, L, h = env
    pr = P.make_config("poisson3d_256", size=20)
    n = pr.n
    Ad = L.csr_to_device(pr.A)
    b = torch.from_numpy(pr.b).cuda()
    rng = np.random.default_rng(11)
    p = torch.from_numpy(rng.standard_normal(n)).cuda()
    r = torch.from_numpy(rng.standard_normal(n)).cuda()
    prm = O.make_params("chebyshev", 6, 0.05, 1.95)
    val0 = Ad.val.clone()
    out = {}
    for fmt in ("dia", "csr"):
        assert _analyze(L, h, Ad, fmt) == fmt
        x0 = torch.zeros_like(b)
        L.assg_solve(h, Ad, b, x0, L.assg_default_opts(tol=1e-10))
        Ad.val.mul_(3.0)
        Ad.val[0] += 0.25          # row 0's first entry is its diagonal: A stays SPD
        x1 = torch.zeros_like(b)
        i1 = L.assg_solve(h, Ad, b, x1, L.assg_default_opts(tol=1e-10))
        xh = torch.zeros_like(b)
        L.assg_hscg_solve(h, Ad, b, xh, 1e-10, 0)
        G = L.assg_basis_gram(h, Ad, p, r, 6, *prm)
        Ad.val.copy_(val0)
        out[fmt] = (x0, x1, i1["outer_iters"], xh, G)
    assert not torch.equal(out["dia"][0], out["dia"][1])
    assert torch.equal(out["dia"][1], out["csr"][1]) and out["dia"][2] == out["csr"][2]
    assert torch.equal(out["dia"][3], out["csr"][3])
    assert np.array_equal(out["dia"][4], out["csr"][4])
    A3 = pr.A.copy()
    A3.data = A3.data * 3.0
    A3.data[0] += 0.25
    x1 = out["dia"][1].cpu().numpy()
    assert np.linalg.norm(pr.b - A3 @ x1) / np.linalg.norm(pr.b) <= 1e-10


def test_noalloc_and_forced_schedule_read_the_diagonal_storage(env):
    """The other solve entry points refresh and read it too."""
    torch, L, h = env
    pr = P.make_config("poisson2d_64", size=40)
    Ad = L.csr_to_device(pr.A)
    b = torch.from_numpy(pr.b).cuda()
    res = {}
    val0 = Ad.val.clone()
    for fmt in ("csr", "dia"):
        assert _analyze(L, h, Ad, fmt) == fmt
        Ad.val.mul_(2.0)
        x = torch.zeros_like(b)
        i = L.assg_solve_noalloc(h, Ad, b, x, L.assg_default_opts(tol=1e-10))
        xf = torch.zeros_like(b)
        jf = L.assg_solve_forced_schedule(h, Ad, b, xf, [3, 5, 7],
                                          L.assg_default_opts(tol=1e-10))
        Ad.val.copy_(val0)
        res[fmt] = (x.cpu().numpy(), i["outer_iters"], xf.cpu().numpy(), jf["outer_iters"])
    assert np.array_equal(res["csr"][0], res["dia"][0]) and res["csr"][1] == res["dia"][1]
    assert np.array_equal(res["csr"][2], res["dia"][2]) and res["csr"][3] == res["dia"][3]


def _batch(torch, L, h, probs, fmt, opts, scale=None):
    As = [L.csr_to_device(pr.A) for pr in probs]
    L.assg_set_format(h, fmt)
    try:
        L.assg_batch_analyze(h, As)
    finally:
        L.assg_set_format(h, "auto")
    got = L.assg_batch_format(h)
    if scale is not None:                       # values changed after the analysis
        i, f = scale
        As[i].val.mul_(f)
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    xs = [torch.zeros_like(b) for b in bs]
    infos = L.assg_batch_solve(h, As, bs, xs, L.assg_default_opts(**opts))
    return got, [x.cpu().numpy() for x in xs], infos


@pytest.mark.parametrize("basis", ["chebyshev", "newton"])
def test_batch_in_both_storages(env, basis):
    """A batch of 2-D Poisson systems of uneven sides takes the diagonal
    storage (each system with its own diagonals); both storages converge
    every system to the tolerance with the same outer-loop counts (+-1), and
    the solutions agree with the oracle's."""
    torch, L, h = env
    probs = P.make_batch(count=8, lo=16, hi=120, seed=41)
    opts = dict(s_max=10, tol=1e-10, basis=basis)
    fc, xc, ic = _batch(torch, L, h, probs, "csr", opts)
    fd, xd, id_ = _batch(torch, L, h, probs, "auto", opts)
    assert fc == "csr" and fd == "dia"
    for pr, a, b, i, j in zip(probs, xc, xd, ic, id_):
        assert i["outcome"] == j["outcome"] == L.CONVERGED
        assert abs(i["outer_iters"] - j["outer_iters"]) <= 1
        for x in (a, b):
            assert np.linalg.norm(pr.b - pr.A @ x) / np.linalg.norm(pr.b) <= 1e-10
        xo, io = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10, basis=basis)
        assert abs(j["outer_iters"] - io["outer"]) <= 1
        assert np.linalg.norm(b - xo) / np.linalg.norm(xo) <= 1e-8


def test_batch_storage_choice_and_refresh(env):
    """One system off 32 diagonals keeps the whole batch in CSR (AUTO) or
    fails the forced analysis; values changed after the analysis are the
    ones solved with."""
    torch, L, h = env
    probs = P.make_batch(count=4, lo=20, hi=60, seed=43)
    R = _random_spd(900, 9)
    rhs = P.rhs_normal(900, 5)
    mixed = list(probs) + [P.Problem(name="random", A=R, b=rhs, x0=np.zeros(900))]
    got, xs, infos = _batch(torch, L, h, mixed, "auto", dict(tol=1e-10))
    assert got == "csr" and all(i["outcome"] == L.CONVERGED for i in infos)
    with pytest.raises(L.AssgError, match="unsupported"):
        _batch(torch, L, h, mixed, "dia", dict(tol=1e-10))
    with pytest.raises(L.AssgError):
        L.assg_batch_format(h)
    opts = dict(s_max=10, tol=1e-10)
    fd, xd, id_ = _batch(torch, L, h, probs, "dia", opts, scale=(2, 4.0))
    fc, xc, ic = _batch(torch, L, h, probs, "csr", opts, scale=(2, 4.0))
    assert fd == "dia" and fc == "csr"
    A2 = probs[2].A * 4.0
    for k, (pr, a, b) in enumerate(zip(probs, xc, xd)):
        M = A2 if k == 2 else pr.A
        for x in (a, b):
            assert np.linalg.norm(pr.b - M @ x) / np.linalg.norm(pr.b) <= 1e-10
