"""The reference gradient of x = A^{-1} b used by the GPU autograd tests,
pinned on the CPU: for L(x) = ||x - t||^2, dL/db = lambda and
dL/dA_ij = -lambda_i x_j with A lambda = dL/dx, checked against central
finite differences of dense solves (symmetric directions in A's stored
values, random directions in b)."""
import numpy as np
import scipy.sparse as sp

import spd_problems as P


def reference_gradient(A, b, t):
    Ad = A.toarray()
    x = np.linalg.solve(Ad, b)
    lam = np.linalg.solve(Ad, 2.0 * (x - t))
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    return x, lam, -lam[rows] * x[A.indices]


def _loss(A, val, b, t):
    M = sp.csr_matrix((val, A.indices, A.indptr), shape=A.shape).toarray()
    x = np.linalg.solve(M, b)
    return float(np.sum((x - t) ** 2))


def test_reference_gradient_matches_central_differences():
    A = P.varcoef7(5, 1.0, 105)
    n = A.shape[0]
    b = P.rhs_normal(n, 3)
    t = P.rhs_normal(n, 4)
    _, gb, gval = reference_gradient(A, b, t)
    for seed in range(6):
        d = P.symmetric_direction(A, 100 + seed)
        h = 1e-6 * np.linalg.norm(A.data) / np.linalg.norm(d)
        fd = (_loss(A, A.data + h * d, b, t) - _loss(A, A.data - h * d, b, t)) / (2 * h)
        assert abs(fd - gval @ d) <= 1e-6 * abs(gval @ d), (seed, fd, gval @ d)
        db = P.rhs_normal(n, 200 + seed)
        hb = 1e-6 * np.linalg.norm(b) / np.linalg.norm(db)
        fdb = (_loss(A, A.data, b + hb * db, t) - _loss(A, A.data, b - hb * db, t)) / (2 * hb)
        assert abs(fdb - gb @ db) <= 1e-6 * abs(gb @ db), (seed, fdb, gb @ db)


def test_symmetric_direction_is_symmetric():
    A = P.varcoef7(4, 1.0, 105)
    d = P.symmetric_direction(A, 1)
    D = sp.csr_matrix((d, A.indices, A.indptr), shape=A.shape)
    assert abs(D - D.T).max() == 0.0
