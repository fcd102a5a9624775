"""Argument checks of the C ABI on the GPU: malformed CSR patterns are
rejected by the analyses before any kernel reads through them, a failed
analysis leaves nothing to solve with, and a solve must use the analyzed
pattern.  No kernel in these tests runs on invalid data: the only device
work on a rejected pattern is the in-bounds scan of its column indices."""
import numpy as np
import pytest

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


def _valid(L):
    pr = P.make_config("poisson2d_64", size=21)
    return pr, L.csr_to_device(pr.A)


def _with(L, A, row_ptr=None, col_idx=None):
    return L.DeviceCSR(A.row_ptr if row_ptr is None else row_ptr,
                       A.col_idx if col_idx is None else col_idx, A.val, A.n, A.nnz)


def _solve(torch, L, h, pr, A):
    b = torch.from_numpy(pr.b).cuda()
    x = torch.zeros_like(b)
    return L.assg_solve(h, A, b, x, L.assg_default_opts(tol=1e-10))


@pytest.mark.parametrize("where", ["first", "middle", "last"])
@pytest.mark.parametrize("value", ["minus_one", "n", "int_max"])
def test_column_out_of_range_rejected(env, where, value):
    torch, L, h = env
    pr, A = _valid(L)
    ci = A.col_idx.clone()
    pos = {"first": 0, "middle": A.nnz // 2, "last": A.nnz - 1}[where]
    ci[pos] = {"minus_one": -1, "n": A.n, "int_max": 2**31 - 1}[value]
    with pytest.raises(L.AssgError, match="column index"):
        L.assg_analyze(h, _with(L, A, col_idx=ci))


def test_failed_analysis_leaves_nothing_to_solve(env):
    """After a valid analysis, a rejected re-analysis (same row_ptr, bad
    columns) must not leave the earlier analysis in force."""
    torch, L, h = env
    pr, A = _valid(L)
    L.assg_analyze(h, A)
    assert _solve(torch, L, h, pr, A)["outcome"] == L.CONVERGED
    ci = A.col_idx.clone()
    ci[7] = A.n + 5
    bad = _with(L, A, col_idx=ci)
    with pytest.raises(L.AssgError):
        L.assg_analyze(h, bad)
    with pytest.raises(L.AssgError, match="not analyzed"):
        _solve(torch, L, h, pr, bad)
    with pytest.raises(L.AssgError, match="not analyzed"):
        _solve(torch, L, h, pr, A)
    L.assg_analyze(h, A)
    assert _solve(torch, L, h, pr, A)["outcome"] == L.CONVERGED


def test_solve_needs_the_analyzed_column_array(env):
    torch, L, h = env
    pr, A = _valid(L)
    L.assg_analyze(h, A)
    other = _with(L, A, col_idx=A.col_idx.clone())   # same contents, another array
    with pytest.raises(L.AssgError, match="not analyzed"):
        _solve(torch, L, h, pr, other)


def test_row_pointer_checks(env):
    torch, L, h = env
    pr, A = _valid(L)
    rp = A.row_ptr.clone()
    rp[-1] = A.nnz - 1                                   # row_ptr[n] != nnz
    with pytest.raises(L.AssgError, match="row_ptr"):
        L.assg_analyze(h, _with(L, A, row_ptr=rp))
    rp = A.row_ptr.clone()
    rp[3], rp[4] = rp[4].item(), rp[3].item()            # decreasing
    with pytest.raises(L.AssgError, match="nondecreasing"):
        L.assg_analyze(h, _with(L, A, row_ptr=rp))
    rp = A.row_ptr.clone()
    rp[0] = 1
    with pytest.raises(L.AssgError, match="row_ptr"):
        L.assg_analyze(h, _with(L, A, row_ptr=rp))


def test_batch_rejects_bad_system_and_keeps_no_batch(env):
    torch, L, h = env
    probs = P.make_batch(count=3, lo=12, hi=20, seed=3)
    As = [L.csr_to_device(pr.A) for pr in probs]
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    xs = [torch.zeros_like(b) for b in bs]
    L.assg_batch_analyze(h, As)
    infos = L.assg_batch_solve(h, As, bs, xs, L.assg_default_opts(tol=1e-10))
    assert all(i["outcome"] == L.CONVERGED for i in infos)
    ci = As[1].col_idx.clone()
    ci[-1] = As[1].n                                      # in range of the batch, not of system 1
    bad = list(As)
    bad[1] = _with(L, As[1], col_idx=ci)
    with pytest.raises(L.AssgError, match="column index"):
        L.assg_batch_analyze(h, bad)
    with pytest.raises(L.AssgError):
        L.assg_batch_solve(h, As, bs, xs, L.assg_default_opts(tol=1e-10))


def test_batch_solve_arguments_must_match(env):
    torch, L, h = env
    probs = P.make_batch(count=2, lo=12, hi=20, seed=4)
    As = [L.csr_to_device(pr.A) for pr in probs]
    bs = [torch.from_numpy(pr.b).cuda() for pr in probs]
    xs = [torch.zeros_like(b) for b in bs]
    L.assg_batch_analyze(h, As)
    with pytest.raises(L.AssgError, match="do not match"):
        L.assg_batch_solve(h, As[:1], bs[:1], xs[:1], L.assg_default_opts())
    moved = [As[0], _with(L, As[1], row_ptr=As[1].row_ptr.clone())]
    with pytest.raises(L.AssgError):
        L.assg_batch_solve(h, moved, bs, xs, L.assg_default_opts())
    infos = L.assg_batch_solve(h, As, bs, xs, L.assg_default_opts(tol=1e-10))
    assert all(i["outcome"] == L.CONVERGED for i in infos)
    for pr, x in zip(probs, xs):
        xr = x.cpu().numpy()
        assert np.linalg.norm(pr.b - pr.A @ xr) / np.linalg.norm(pr.b) <= 1e-10


def test_binding_checks_dtype_and_length(env):
    """The binding refuses tensors whose type or length differs from what
    the C ABI assumes, before the library is called."""
    torch, L, h = env
    pr, A = _valid(L)
    L.assg_analyze(h, A)
    b = torch.from_numpy(pr.b).cuda()
    x = torch.zeros_like(b)
    opts = L.assg_default_opts(tol=1e-10)
    with pytest.raises(TypeError):
        L.assg_solve(h, A, b.float(), x, opts)
    with pytest.raises(ValueError):
        L.assg_solve(h, A, b, x[:-1].contiguous(), opts)
    with pytest.raises(ValueError):
        L.assg_solve(h, A, b, x[::2], opts)
    with pytest.raises(TypeError):
        L.assg_solve(h, _with(L, A, col_idx=A.col_idx.long()), b, x, opts)
    with pytest.raises(ValueError):
        L.assg_spmv(h, A, b, torch.empty(A.n + 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        L.assg_csr_outer_on_pattern(h, A, b, b, 1.0,
                                    torch.empty(A.nnz - 1, dtype=torch.float64, device="cuda"))
    assert L.assg_solve(h, A, b, x, opts)["outcome"] == L.CONVERGED


def test_overlapping_vectors_refused(env):
    """b and x (and the SpMV's x and y) must not share memory: the library
    reads one while it writes the other."""
    torch, L, h = env
    pr, A = _valid(L)
    L.assg_analyze(h, A)
    buf = torch.zeros(2 * A.n, dtype=torch.float64, device="cuda")
    b = buf[:A.n]
    with pytest.raises(L.AssgError, match="overlap"):
        L.assg_solve(h, A, b, b, L.assg_default_opts(tol=1e-10))
    with pytest.raises(L.AssgError, match="overlap"):
        L.assg_hscg_solve(h, A, b, buf[1:A.n + 1], 1e-10, 0)
    with pytest.raises(L.AssgError, match="overlap"):
        L.assg_spmv(h, A, b, b)
    y = buf[A.n:]
    L.assg_spmv(h, A, b, y)                                # adjacent, not overlapping
