"""Seeded synthetic SPD test problems (inputs only).

The paper's experiments run on small SuiteSparse matrices that are not
available here; these generators build stand-ins with the same conventions
(Section 5, experimental setup): FP64, x0 = 0, and two-sided diagonal scaling
D^{-1/2} A D^{-1/2} with D the largest absolute entry of each row.

This module holds none of the solver's arithmetic.  It only builds CSR
matrices (int32 row pointers and column indices, sorted columns, both
triangles stored), right-hand sides and starting vectors, each from a
numpy ``Generator(PCG64(seed))``.  Both the CPU oracle and the GPU library
consume its output; neither is imported here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

__all__ = [
    "Problem", "poisson2d", "poisson3d", "diffusion27", "varcoef7",
    "diag_scale", "rhs_from_solution", "rhs_normal", "diagonal_matrix",
    "poisson2d_eigs", "poisson3d_eigs", "make_config", "CONFIGS",
    "batch_poisson2d_specs",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _stencil_csr(shape, offsets, values):
    """CSR of a stencil operator on a structured grid with Dirichlet boundary.

    ``shape`` is (nz, ny, nx) (use 1 for absent dimensions); ``offsets`` is a
    list of (dz, dy, dx); ``values[k]`` is either a scalar or an array of
    length N giving entry (i, i + offset_k) for row i.  Offsets must be sorted
    so that the linear column offsets dz*ny*nx + dy*nx + dx ascend; rows then
    come out with sorted columns.  Entries whose neighbour falls outside the
    grid are dropped.
    """
    nz, ny, nx = shape
    n = nz * ny * nx
    iz, iy, ix = np.meshgrid(np.arange(nz, dtype=np.int64),
                             np.arange(ny, dtype=np.int64),
                             np.arange(nx, dtype=np.int64), indexing="ij")
    iz = iz.ravel(); iy = iy.ravel(); ix = ix.ravel()
    lin = [dz * ny * nx + dy * nx + dx for (dz, dy, dx) in offsets]
    assert all(lin[k] < lin[k + 1] for k in range(len(lin) - 1)), "offsets must ascend"
    k = len(offsets)
    valid = np.empty((n, k), dtype=bool)
    cols = np.empty((n, k), dtype=np.int32)
    vals = np.empty((n, k), dtype=np.float64)
    base = np.arange(n, dtype=np.int64)
    for j, (dz, dy, dx) in enumerate(offsets):
        ok = ((iz + dz >= 0) & (iz + dz < nz) & (iy + dy >= 0) & (iy + dy < ny)
              & (ix + dx >= 0) & (ix + dx < nx))
        valid[:, j] = ok
        c = base + lin[j]
        c[~ok] = 0
        cols[:, j] = c.astype(np.int32)
        vals[:, j] = values[j]
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31, "nnz must fit int32"
    col_idx = cols[valid]
    val = vals[valid]
    del valid, cols, vals
    return sp.csr_matrix((val, col_idx, row_ptr.astype(np.int32)), shape=(n, n))


def poisson2d(n: int, scaled: bool = True) -> sp.csr_matrix:
    """5-point Dirichlet Laplacian on an n x n grid (stencil 4, -1 x 4).

    With ``scaled`` the two-sided diagonal scaling of the experiments is
    applied, which for this matrix is A/4.
    """
    offs = [(0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0)]
    vals = [-1.0, -1.0, 4.0, -1.0, -1.0]
    A = _stencil_csr((1, n, n), offs, vals)
    return diag_scale(A) if scaled else A


def poisson3d(n: int, scaled: bool = True) -> sp.csr_matrix:
    """7-point Dirichlet Laplacian on an n^3 grid (stencil 6, -1 x 6)."""
    offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    vals = [-1.0, -1.0, -1.0, 6.0, -1.0, -1.0, -1.0]
    A = _stencil_csr((n, n, n), offs, vals)
    return diag_scale(A) if scaled else A


def poisson2d_eigs(n: int, scaled: bool = True) -> np.ndarray:
    """Closed-form spectrum of ``poisson2d(n)`` (sorted ascending)."""
    j = np.arange(1, n + 1)
    s = 4.0 * np.sin(j * np.pi / (2 * (n + 1))) ** 2
    lam = (s[:, None] + s[None, :]).ravel()
    if scaled:
        lam = lam / 4.0
    return np.sort(lam)


def poisson3d_eigs(n: int, scaled: bool = True) -> np.ndarray:
    j = np.arange(1, n + 1)
    s = 4.0 * np.sin(j * np.pi / (2 * (n + 1))) ** 2
    lam = (s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel()
    if scaled:
        lam = lam / 6.0
    return np.sort(lam)


def _face_weight_operator(n: int, offsets_pos, sigma: float, seed: int) -> sp.csr_matrix:
    """Graph-Laplacian-like SPD operator with lognormal edge weights.

    Every undirected neighbour pair (i, j) gets one weight exp(sigma * Z),
    Z ~ N(0, 1); entry a_ij = a_ji = -w_ij.  Every node also gets an
    independent weight for each neighbour direction that leaves the domain
    (Dirichlet boundary).  The diagonal is the sum of all of a node's weights,
    so the matrix is symmetric, weakly diagonally dominant, strictly so on the
    boundary, and irreducible: SPD.  With all weights 1 it is the constant
    coefficient stencil.
    """
    rng = _rng(seed)
    nz = ny = nx = n
    N = n ** 3
    iz, iy, ix = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    iz = iz.ravel(); iy = iy.ravel(); ix = ix.ravel()

    def inside(dz, dy, dx):
        return ((iz + dz >= 0) & (iz + dz < nz) & (iy + dy >= 0) & (iy + dy < ny)
                & (ix + dx >= 0) & (ix + dx < nx))

    lin = lambda o: o[0] * ny * nx + o[1] * nx + o[2]
    diag = np.zeros(N)
    wpos = {}
    for o in offsets_pos:                      # one weight per undirected edge
        w = np.exp(sigma * rng.standard_normal(N))
        ok = inside(*o)
        w[~ok] = 0.0
        wpos[o] = w
    for o in offsets_pos:                      # boundary weights, both directions
        for sgn in (1, -1):
            oo = tuple(sgn * t for t in o)
            wb = np.exp(sigma * rng.standard_normal(N))
            wb[inside(*oo)] = 0.0
            diag += wb
    offsets = []
    values = []
    for o in offsets_pos:
        neg = tuple(-t for t in o)
        # entry (i, i - o) couples i with the node whose positive edge o lands on i
        wneg = np.zeros(N)
        ok = inside(*neg)
        src = np.nonzero(ok)[0]
        wneg[src] = wpos[o][src + lin(neg)]
        offsets.append(neg); values.append(-wneg)
        offsets.append(o); values.append(-wpos[o])
        diag += wpos[o] + wneg
    offsets.append((0, 0, 0)); values.append(diag)
    order = np.argsort([lin(o) for o in offsets], kind="stable")
    offsets = [offsets[k] for k in order]
    values = [values[k] for k in order]
    return _stencil_csr((n, n, n), offsets, values)


def diffusion27(n: int, sigma: float = 2.0, seed: int = 103, scaled: bool = True) -> sp.csr_matrix:
    """27-point variable-coefficient diffusion on an n^3 grid (26-neighbour
    graph, lognormal face weights), Jacobi-scaled to unit diagonal."""
    pos = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
           if (dz, dy, dx) > (0, 0, 0)]
    A = _face_weight_operator(n, pos, sigma, seed)
    return diag_scale(A) if scaled else A


def varcoef7(n: int, sigma: float = 1.0, seed: int = 105, scaled: bool = False) -> sp.csr_matrix:
    """7-point variable-coefficient Laplacian (lognormal face weights)."""
    pos = [(0, 0, 1), (0, 1, 0), (1, 0, 0)]
    A = _face_weight_operator(n, pos, sigma, seed)
    return diag_scale(A) if scaled else A


def diag_scale(A: sp.csr_matrix) -> sp.csr_matrix:
    """Two-sided scaling D^{-1/2} A D^{-1/2}, D = largest |a_ij| of each row
    (Section 5 setup)."""
    A = A.tocsr()
    counts = np.diff(A.indptr)
    if np.any(counts == 0):
        raise ValueError("a row without entries cannot be scaled (matrix not SPD)")
    rows = np.repeat(np.arange(A.shape[0], dtype=np.int64), counts)
    d = np.maximum.reduceat(np.abs(A.data), A.indptr[:-1].astype(np.int64))
    s = 1.0 / np.sqrt(d)
    data = A.data * (s[rows] * s[A.indices])      # s_i*s_j == s_j*s_i keeps symmetry exact
    return sp.csr_matrix((data, A.indices.astype(np.int32), A.indptr.astype(np.int32)), shape=A.shape)


def diagonal_matrix(eigs) -> sp.csr_matrix:
    """Diagonal SPD matrix with the given eigenvalues (spectrum known exactly)."""
    e = np.asarray(eigs, dtype=np.float64)
    n = e.size
    return sp.csr_matrix((e, np.arange(n, dtype=np.int32), np.arange(n + 1, dtype=np.int32)),
                         shape=(n, n))


def rhs_from_solution(A: sp.csr_matrix, seed: int):
    """x* ~ U(-1, 1) from ``seed``; returns (b = A x*, x*)."""
    xs = _rng(seed).uniform(-1.0, 1.0, A.shape[0])
    return A @ xs, xs


def rhs_normal(n: int, seed: int) -> np.ndarray:
    return _rng(seed).standard_normal(n)


def batch_poisson2d_specs(count: int = 64, lo: int = 32, hi: int = 512, seed: int = 104):
    """Side lengths n_i ~ U{lo..hi} and shifts c_i ~ U(0, 0.1) * lambda_max(A_i)
    for a batch of unscaled 2D Poisson systems A_i + c_i I."""
    rng = _rng(seed)
    sides = rng.integers(lo, hi + 1, size=count)
    fr = rng.uniform(0.0, 0.1, size=count)
    lmax = 8.0 - 8.0 * np.sin(np.pi / (2 * (sides + 1))) ** 2
    return sides, fr * lmax


@dataclass
class Problem:
    """One linear system A x = b with its generating recipe."""
    name: str
    A: sp.csr_matrix
    b: np.ndarray
    x0: np.ndarray
    xstar: np.ndarray | None = None
    opts: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]


CONFIGS = {
    "poisson2d_64": "2D 5-point Poisson 64x64 (N=4,096), scaled, b=A x*, x* ~ U(-1,1) seed 101",
    "poisson3d_256": "3D 7-point Poisson 256^3 (N=16,777,216), scaled, b=A x*, x* ~ U(-1,1) seed 102",
    "diffusion27_160": "3D 27-point lognormal(sigma=2) diffusion 160^3 (N=4,096,000), Jacobi-scaled, b ~ N(0,1) seed 1103",
}


def make_config(name: str, size: int | None = None) -> Problem:
    """Build one of the named workloads.  ``size`` overrides the grid side
    (same recipe at a smaller size, used by tests)."""
    if name == "poisson2d_64":
        n = size or 64
        A = poisson2d(n)
        b, xs = rhs_from_solution(A, 101)
    elif name == "poisson3d_256":
        n = size or 256
        A = poisson3d(n)
        b, xs = rhs_from_solution(A, 102)
    elif name == "diffusion27_160":
        n = size or 160
        A = diffusion27(n, 2.0, 103)
        b, xs = rhs_normal(A.shape[0], 1103), None
    elif name == "varcoef7_128":
        n = size or 128
        A = varcoef7(n, 1.0, 105)
        b, xs = rhs_normal(A.shape[0], 1105), None
    else:
        raise KeyError(name)
    return Problem(name=name, A=A, b=b, x0=np.zeros(A.shape[0]), xstar=xs)


def transpose_index(A: sp.csr_matrix) -> np.ndarray:
    """For a CSR matrix with a symmetric pattern: t[k] = position of the
    entry (j, i) for the stored entry k = (i, j)."""
    A = A.tocsr()
    P = sp.csr_matrix((np.arange(A.nnz, dtype=np.float64), A.indices, A.indptr), shape=A.shape)
    T = P.T.tocsr()
    T.sort_indices()
    if not (np.array_equal(T.indptr, A.indptr) and np.array_equal(T.indices, A.indices)):
        raise ValueError("pattern is not symmetric")
    return T.data.astype(np.int64)


def symmetric_direction(A: sp.csr_matrix, seed: int) -> np.ndarray:
    """A random direction in the stored values of A that keeps A symmetric:
    d_k = z_k + z_t(k), z ~ N(0, 1)."""
    z = _rng(seed).standard_normal(A.nnz)
    return z + z[transpose_index(A)]


def make_batch(count: int = 64, lo: int = 32, hi: int = 512, seed: int = 104) -> list:
    """The batched workload: ``count`` unscaled 2D 5-point Poisson systems
    A_i + c_i I with sides n_i ~ U{lo..hi}, shifts c_i ~ U(0, 0.1) lambda_max(A_i)
    and right-hand sides b_i ~ N(0, 1) (seed + 1000 + i), x0 = 0."""
    sides, shifts = batch_poisson2d_specs(count, lo, hi, seed)
    out = []
    for i, (m, c) in enumerate(zip(sides, shifts)):
        A = (poisson2d(int(m), scaled=False) + c * sp.identity(int(m) * int(m), format="csr")).tocsr()
        A.sort_indices()
        A = sp.csr_matrix((A.data, A.indices.astype(np.int32), A.indptr.astype(np.int32)),
                          shape=A.shape)
        b = rhs_normal(A.shape[0], seed + 1000 + i)
        out.append(Problem(name=f"batch{i}_poisson2d_{int(m)}", A=A, b=b, x0=np.zeros(A.shape[0])))
    return out
