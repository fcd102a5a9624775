"""Input generators: structure, symmetry, SPD and closed-form spectra."""
import numpy as np
import pytest

import spd_problems as P


def test_poisson2d_structure_and_spectrum():
    n = 9
    A = P.poisson2d(n)
    assert A.shape == (n * n, n * n)
    assert A.nnz == 5 * n * n - 4 * n
    assert abs(A - A.T).max() == 0.0
    assert np.all(A.diagonal() == 1.0)                 # 4/4 after scaling
    ev = np.linalg.eigvalsh(A.toarray())
    np.testing.assert_allclose(ev, P.poisson2d_eigs(n), rtol=0, atol=1e-13)


def test_poisson3d_structure_and_spectrum():
    n = 6
    A = P.poisson3d(n)
    assert A.nnz == 7 * n ** 3 - 6 * n ** 2
    assert abs(A - A.T).max() == 0.0
    ev = np.linalg.eigvalsh(A.toarray())
    np.testing.assert_allclose(ev, P.poisson3d_eigs(n), rtol=0, atol=1e-13)
    # sorted, int32 CSR
    assert A.indptr.dtype == np.int32 and A.indices.dtype == np.int32
    for i in range(A.shape[0]):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)


@pytest.mark.parametrize("n", [3, 5, 7])
def test_diffusion27_spd_unit_diagonal(n):
    A = P.diffusion27(n, 2.0, 7)
    assert A.nnz == (3 * n - 2) ** 3
    assert abs(A - A.T).max() == 0.0
    np.testing.assert_allclose(A.diagonal(), 1.0, rtol=0, atol=1e-15)
    assert np.linalg.eigvalsh(A.toarray()).min() > 0.0
    # with unit weights the operator is the classic 27-point stencil 26/-1
    B = P.diffusion27(n, 0.0, 7, scaled=False).toarray()
    inner = (n // 2) * (n * n + n + 1)
    assert B[inner, inner] == 26.0
    row = B[inner][B[inner] != 0.0]
    assert row.size == 27 and np.sort(row)[:26].tolist() == [-1.0] * 26


def test_varcoef7_spd():
    A = P.varcoef7(5, 1.0, 5)
    assert A.nnz == 7 * 125 - 6 * 25
    assert abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A.toarray()).min() > 0.0


def test_diag_scale_is_two_sided_row_max():
    rng = np.random.default_rng(0)
    M = rng.standard_normal((7, 7))
    M = M @ M.T + 7 * np.eye(7)
    import scipy.sparse as sp
    S = P.diag_scale(sp.csr_matrix(M)).toarray()
    d = np.abs(M).max(axis=1)
    np.testing.assert_allclose(S, M / np.sqrt(np.outer(d, d)), rtol=1e-15)


def test_rhs_seeded():
    A = P.poisson2d(8)
    b1, x1 = P.rhs_from_solution(A, 101)
    b2, x2 = P.rhs_from_solution(A, 101)
    assert np.array_equal(b1, b2) and np.all(np.abs(x1) <= 1)
    np.testing.assert_allclose(b1, A @ x1)


def test_batch_specs():
    sides, shifts = P.batch_poisson2d_specs()
    assert sides.size == 64 and sides.min() >= 32 and sides.max() <= 512
    lmax = 8 - 8 * np.sin(np.pi / (2 * (sides + 1))) ** 2
    assert np.all(shifts >= 0) and np.all(shifts <= 0.1 * lmax)
