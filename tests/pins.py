"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each ``pin_*`` function raises AssertionError when the oracle disagrees with
an independent fact: a closed form, a textbook/library routine, an explicit
brute-force construction, or an exact-arithmetic equivalence.  They are run
as tests (test_oracle_pins.py) and, with mistakes planted in the oracle, by
test_oracle_mutations.py to show that each plausible mistake is caught.
"""
import math

import numpy as np
import scipy.linalg as sla
from numpy.polynomial import chebyshev as npcheb

import oracle as O
import spd_problems as P


def _small_spd(n=40, seed=3, cond=50.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n) / cond * 1.9
    M = (Q * ev) @ Q.T
    M = 0.5 * (M + M.T)
    import scipy.sparse as sp
    return sp.csr_matrix(M), ev


# --------------------------------------------------------------------- HSCG
def pin_hscg_dense_cholesky():
    """HSCG solution agrees with a dense Cholesky solve within kappa * tol."""
    A, ev = _small_spd(60, 1, 200.0)
    b = np.random.default_rng(2).standard_normal(60)
    x, info = O.hscg(A, b, tol=1e-12)
    assert info["outcome"] == O.Outcome.CONVERGED
    xc = sla.cho_solve(sla.cho_factor(A.toarray()), b)
    kappa = ev.max() / ev.min()
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) <= kappa * 1e-12
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) <= 1e-12


def pin_hscg_finite_termination():
    """CG on a matrix with 6 distinct eigenvalues terminates in 6 steps."""
    vals = np.repeat([0.1, 0.3, 0.7, 1.1, 1.5, 1.9], 10)
    A = P.diagonal_matrix(vals)
    b = np.random.default_rng(4).standard_normal(vals.size)
    x, info = O.hscg(A, b, tol=1e-13)
    assert info["outcome"] == O.Outcome.CONVERGED and info["iters"] == 6
    np.testing.assert_allclose(x, b / vals, rtol=1e-11)


def pin_psi_identity():
    """(4.5): psi_i from the recurrence equals ||r_i||^2 / ||p_i||^2."""
    A, _ = _small_spd(50, 5, 100.0)
    b = np.random.default_rng(6).standard_normal(50)
    _, info = O.hscg(A, b, tol=1e-10, record=True)
    psi = 1.0
    for i, beta in enumerate(info["betas"][:25]):
        psi = O.psi_update(psi, beta)
        direct = info["rnorms"][i + 1] ** 2 / info["pnorms"][i + 1] ** 2
        assert abs(psi - direct) <= 1e-12 * direct


# --------------------------------------------------------------- Lanczos T
def pin_lanczos_T_equals_VtAV():
    """(1.1): T_i from alpha, beta equals V^T A V with V the normalized
    residuals with alternating signs."""
    A, _ = _small_spd(60, 7, 30.0)
    b = np.random.default_rng(8).standard_normal(60)
    _, info = O.hscg(A, b, tol=1e-14, record=True, record_vectors=True)
    i = 12
    V = np.stack([(-1) ** j * info["rvecs"][j] / np.linalg.norm(info["rvecs"][j])
                  for j in range(i)], axis=1)
    T = O.lanczos_tridiagonal(info["alphas"], info["betas"], i)
    np.testing.assert_allclose(T, V.T @ (A @ V), rtol=0, atol=1e-12)


def pin_lanczos_cholesky():
    """(4.1): T_i = L_i L_i^T with the bidiagonal factor built from zeta, eta."""
    A, _ = _small_spd(40, 9, 80.0)
    b = np.random.default_rng(10).standard_normal(40)
    _, info = O.hscg(A, b, tol=1e-12, record=True)
    i = 15
    U = O.lanczos_cholesky_factor(info["alphas"], info["betas"], i)
    T = O.lanczos_tridiagonal(info["alphas"], info["betas"], i)
    np.testing.assert_allclose(U.T @ U, T, rtol=1e-13, atol=1e-14)


def _cg_coeffs(vals, seed=11, iters=None):
    A = P.diagonal_matrix(vals)
    b = np.random.default_rng(seed).standard_normal(len(vals))
    _, info = O.hscg(A, b, tol=1e-15, record=True, max_iters=iters)
    return info["alphas"], info["betas"]


def _explicit_rayleigh_ritz(M_of, nsteps):
    """Brute force: keep the explicit unit vector y and solve each bordered
    2x2 Rayleigh-Ritz problem on span{[y;0], e_new} with a dense eigensolver."""
    y = np.array([1.0])
    out = []
    for k in range(1, nsteps + 1):
        M = M_of(k + 1)
        yy = np.append(y, 0.0)
        e = np.zeros(k + 1); e[k] = 1.0
        H = np.array([[yy @ M @ yy, yy @ M @ e], [e @ M @ yy, e @ M @ e]])
        w, V = np.linalg.eigh(H)
        v = V[:, -1]
        y = v[0] * yy + v[1] * e
        out.append(w[-1])
    return out


def pin_alg3_is_rayleigh_ritz():
    """Algorithm 3 reproduces explicit 2x2 Rayleigh-Ritz steps on T."""
    al, be = _cg_coeffs(np.linspace(0.02, 1.95, 30))
    n = 20
    T = O.lanczos_tridiagonal(al, be, n + 1)
    ref = _explicit_rayleigh_ritz(lambda k: T[:k, :k], n)
    est = O.MaxRitzEstimate(1.0 / math.sqrt(al[0]))
    for l in range(n):
        got = est.step(math.sqrt(be[l] / al[l]), 1.0 / math.sqrt(al[l + 1]))
        assert abs(got - ref[l]) <= 1e-12 * ref[l], (l, got, ref[l])


def pin_alg4_is_rayleigh_ritz():
    """Algorithm 4 reproduces explicit 2x2 Rayleigh-Ritz steps on
    L^{-1} L^{-T} (whose largest eigenvalue is ||L^{-1}||^2)."""
    al, be = _cg_coeffs(np.linspace(0.02, 1.95, 30))
    n = 20
    U = O.lanczos_cholesky_factor(al, be, n + 1)       # L^T
    Linv = np.linalg.inv(U.T)

    def M_of(k):
        W = np.linalg.inv(U[:k, :k].T)
        return W @ W.T
    ref = _explicit_rayleigh_ritz(M_of, n)
    est = O.MinRitzEstimate(1.0 / math.sqrt(al[0]))
    for l in range(n):
        got = est.step(math.sqrt(be[l] / al[l]), 1.0 / math.sqrt(al[l + 1]))
        assert abs(1.0 / got - ref[l]) <= 1e-11 * ref[l], (l, 1.0 / got, ref[l])


def pin_ritz_exact_at_two():
    """After one step the 2x2 problem is the whole of T_2: the estimates are
    the exact extremal eigenvalues of T_2 (closed form of a 2x2)."""
    al, be = _cg_coeffs(np.linspace(0.1, 1.9, 12))
    T2 = O.lanczos_tridiagonal(al, be, 2)
    tr, det = T2[0, 0] + T2[1, 1], T2[0, 0] * T2[1, 1] - T2[0, 1] ** 2
    disc = math.sqrt(tr * tr / 4 - det)
    lo, hi = tr / 2 - disc, tr / 2 + disc
    mx = O.MaxRitzEstimate(1 / math.sqrt(al[0]))
    mn = O.MinRitzEstimate(1 / math.sqrt(al[0]))
    eta, zeta = math.sqrt(be[0] / al[0]), 1 / math.sqrt(al[1])
    assert abs(mx.step(eta, zeta) - hi) <= 1e-14 * hi
    assert abs(mn.step(eta, zeta) - lo) <= 1e-13 * lo


def pin_ritz_inside_spectrum():
    """On a diagonal matrix with known eigenvalues:
    lmin(A) <= lmin(T_i) <= lmin~ <= lmax~ <= lmax(T_i) <= lmax(A), with
    lmax~ nondecreasing and lmin~ nonincreasing."""
    vals = np.linspace(0.01, 2.0, 40)
    al, be = _cg_coeffs(vals, 12)
    mx = O.MaxRitzEstimate(1 / math.sqrt(al[0]))
    mn = O.MinRitzEstimate(1 / math.sqrt(al[0]))
    prev_hi, prev_lo = -np.inf, np.inf
    for l in range(len(al) - 1):
        hi = mx.step(math.sqrt(be[l] / al[l]), 1 / math.sqrt(al[l + 1]))
        lo = mn.step(math.sqrt(be[l] / al[l]), 1 / math.sqrt(al[l + 1]))
        ev = np.linalg.eigvalsh(O.lanczos_tridiagonal(al, be, l + 2))
        tol = 1e-12
        assert vals.min() * (1 - tol) <= ev[0] * (1 + tol)
        assert ev[0] <= lo * (1 + tol) and lo <= hi * (1 + tol)
        assert hi <= ev[-1] * (1 + tol) and ev[-1] <= vals.max() * (1 + tol)
        assert hi >= prev_hi * (1 - tol) and lo <= prev_lo * (1 + tol)
        prev_hi, prev_lo = hi, lo


# ------------------------------------------------------------------ basis
def pin_leja_points():
    """(2.7) on [-1,1]: t0=1, t1=-1, t2=0, t3=-1/sqrt(3) (tie broken to the
    smaller), and every t_l maximizes prod |t - t_m| over a fine grid."""
    t = O.leja_reference_points(14)
    np.testing.assert_allclose(t[:4], [1.0, -1.0, 0.0, -1 / math.sqrt(3)], rtol=0, atol=1e-14)
    grid = np.linspace(-1, 1, 400001)
    for l in range(2, 14):
        prod = lambda z: np.prod(np.abs(z[..., None] - t[:l]), axis=-1)
        assert prod(np.array(t[l])) >= prod(grid).max() * (1 - 1e-9)
    assert len(set(np.round(t, 12))) == 14


def pin_basis_closed_forms():
    """On a diagonal A the basis columns equal the polynomials evaluated at
    the eigenvalues: z^l (monomial), prod_{m<l}(z - theta_m) (Newton),
    T_l(2(z - c)/Delta) (Chebyshev, numpy's chebval)."""
    z = np.linspace(0.05, 1.95, 50)
    A = P.diagonal_matrix(z)
    v = np.random.default_rng(13).standard_normal(50)
    s = 10
    cols = O.polynomial_columns(A, v, s, *O.params_monomial(s))
    for l in range(s + 1):
        np.testing.assert_allclose(cols[:, l], z ** l * v, rtol=1e-13, atol=1e-15)
    lo, hi = 0.08, 1.9
    th, ga, mu = O.params_newton(lo, hi, s)
    cols = O.polynomial_columns(A, v, s, th, ga, mu)
    for l in range(s + 1):
        ref = np.prod(z[:, None] - th[None, :l], axis=1) * v
        np.testing.assert_allclose(cols[:, l], ref, rtol=1e-12, atol=1e-14)
    assert th[0] == hi and th[1] == lo
    th, ga, mu = O.params_chebyshev(lo, hi, s)
    cols = O.polynomial_columns(A, v, s, th, ga, mu)
    tt = 2 * (z - 0.5 * (lo + hi)) / (hi - lo)
    for l in range(s + 1):
        ref = npcheb.chebval(tt, np.eye(s + 1)[l]) * v
        np.testing.assert_allclose(cols[:, l], ref, rtol=1e-11, atol=1e-11)


def pin_change_of_basis():
    """(2.4): A Y_ = Y B for every basis type, where Y_ zeroes the last P and
    the last R column; also for a restriction to s~ < sbar levels."""
    A = P.poisson2d(12)
    rng = np.random.default_rng(14)
    p, r = rng.standard_normal(144), rng.standard_normal(144)
    for kind in ("monomial", "newton", "chebyshev"):
        s = 7
        prm = O.make_params(kind, s, 0.01, 1.99)
        Y = O.sstep_basis(A, p, r, s, prm)
        B = O.change_of_basis(s, prm)
        Yu = Y.copy(); Yu[:, s] = 0.0; Yu[:, 2 * s] = 0.0
        res = np.linalg.norm(A @ Yu - Y @ B) / (np.linalg.norm(Y) + 1e-300)
        assert res <= 1e-14, (kind, res)
        for st in (1, 3, 6):
            idx = O.sub_indices(s, st)
            Ys = Y[:, idx]
            Bs = O.change_of_basis(st, prm)
            Ysu = Ys.copy(); Ysu[:, st] = 0.0; Ysu[:, 2 * st] = 0.0
            assert np.linalg.norm(A @ Ysu - Ys @ Bs) <= 1e-14 * np.linalg.norm(Ys)


def pin_sub_indices_are_smaller_basis():
    """(2.2): Y_{k,l} built directly with l levels equals the columns
    sub_indices(sbar, l) of Y_{k,sbar}."""
    A = P.poisson2d(8)
    rng = np.random.default_rng(15)
    p, r = rng.standard_normal(64), rng.standard_normal(64)
    prm = O.make_params("chebyshev", 9, 0.02, 1.98)
    Y = O.sstep_basis(A, p, r, 9, prm)
    for l in range(1, 10):
        np.testing.assert_array_equal(O.sstep_basis(A, p, r, l, prm), Y[:, O.sub_indices(9, l)])


# ---------------------------------------------------------------- s-step CG
def pin_sstep_sigma1_equals_hscg():
    """With sigma = 1 every outer loop is one CG step in coordinates: the
    same iterates as HSCG (exact-arithmetic equivalence, Section 2)."""
    A = P.poisson2d(16)
    b, _ = P.rhs_from_solution(A, 16)
    xh, ih = O.hscg(A, b, tol=1e-10, record=True)
    xs, isg = O.adaptive_sstep_cg(A, b, s_max=1, tol=1e-10)
    assert isg["outcome"] == O.Outcome.CONVERGED
    assert isg["iters"] == ih["iters"] and isg["outer"] == ih["iters"]
    np.testing.assert_allclose(isg["alphas"], ih["alphas"], rtol=1e-10)
    np.testing.assert_allclose(isg["betas"], ih["betas"], rtol=1e-9)
    assert np.linalg.norm(xs - xh) <= 1e-11 * np.linalg.norm(xh)


def pin_sstep_monomial_matches_hscg_coefficients():
    """s-step CG with a small monomial basis reproduces the HSCG alpha/beta
    sequence on a well-conditioned problem (Section 2 equivalence)."""
    vals = np.linspace(0.5, 1.5, 200)
    A = P.diagonal_matrix(vals)
    b = np.random.default_rng(17).standard_normal(200)
    _, ih = O.hscg(A, b, tol=1e-10, record=True)
    _, isg = O.adaptive_sstep_cg(A, b, s_max=3, tol=1e-10, basis="monomial")
    n = min(len(ih["alphas"]), len(isg["alphas"]))
    np.testing.assert_allclose(isg["alphas"][:n], ih["alphas"][:n], rtol=1e-9)
    np.testing.assert_allclose(isg["betas"][:n - 1], ih["betas"][:n - 1], rtol=1e-8)


def pin_sstep_solves():
    """Algorithm 5 reaches the requested true relative residual and agrees
    with a dense Cholesky solve within kappa * tol."""
    A = P.poisson2d(20)
    rng = np.random.default_rng(18)
    b = rng.standard_normal(400)
    ev = P.poisson2d_eigs(20)
    xc = sla.cho_solve(sla.cho_factor(A.toarray()), b)
    for basis in ("chebyshev", "newton"):
        x, info = O.adaptive_sstep_cg(A, b, s_max=10, tol=1e-10, basis=basis)
        assert info["outcome"] == O.Outcome.CONVERGED
        assert info["relres_true"] <= 1e-10
        assert np.linalg.norm(x - xc) / np.linalg.norm(xc) <= ev[-1] / ev[0] * 1e-10
        # the adaptive c lies in [1, kappa(A)] (Section 4, xi bounds)
        cs = [t["c"] for t in info["trace"][2:]]
        assert min(cs) >= 1.0 and max(cs) <= ev[-1] / ev[0]


def pin_adaptive_c_at_least_one():
    """xi >= 1 by its definition (Section 4), so the adaptive c of Algorithm 5
    never drops below 1.  On a spectrum in [0.5, 0.6] the estimate
    lambda_max (psi / lambda_min)^(1/2) is about 0.8 in every loop, so this
    holds only through the max{1, .} of Algorithm 5."""
    A = P.diagonal_matrix(np.linspace(0.5, 0.6, 200))
    b = np.random.default_rng(21).standard_normal(200)
    for basis in ("chebyshev", "newton"):
        _, info = O.adaptive_sstep_cg(A, b, s_max=10, tol=1e-12, basis=basis)
        assert info["outcome"] == O.Outcome.CONVERGED
        cs = [t["c"] for t in info["trace"][1:]]
        assert len(cs) >= 2 and min(cs) >= 1.0, cs


ALL_PINS = [v for k, v in dict(globals()).items() if k.startswith("pin_")]
