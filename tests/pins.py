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



# ------------------------------------------------- adaptive control (a4, a5)
# These pins hold the wiring of Algorithm 5 (which quantities feed (3.2),
# (4.5)-(4.7) and the basis update) to facts computed independently of the
# oracle's code: condition numbers from an SVD of the recorded basis, the
# Ritz estimates from explicit 2x2 Rayleigh-Ritz problems on T of (1.1),
# psi and the residual norms from the recovered vectors, the basis from the
# Chebyshev closed form on a diagonal matrix.

U = 2.0 ** -53


def _geom_problem(n=100, cond=1e4, seed=1):
    """Diagonal SPD matrix with a geometric spectrum in [2/cond, 2]: CG's
    residual norm oscillates, so the break (4.7) fires in several loops."""
    vals = np.geomspace(1.0 / cond, 1.0, n) * 2.0
    A = P.diagonal_matrix(vals)
    b = np.random.default_rng(seed).standard_normal(n)
    return A, b, vals


def _recorded_run(A, b, **kw):
    x, info = O.adaptive_sstep_cg(A, b, record_gram=True, record_basis=True, **kw)
    assert info["outcome"] == O.Outcome.CONVERGED, info["outcome"]
    return x, info


def _svd_cond(Y):
    sv = np.linalg.svd(Y, compute_uv=False)
    return sv[0] / sv[-1] if sv[-1] > 0 else math.inf


def pin_kappa_is_basis_condition_number():
    """Section 3: kappa(Y_{k,l}) is estimated as the square root of the
    condition number of the matching principal submatrix of G.  Every
    recorded kappa of a run whose basis is well enough conditioned for the
    estimate to be accurate (kappa(Y) < 1e5) equals the 2-norm condition
    number of the recorded basis columns, from an SVD."""
    A, b, _ = _geom_problem()
    _, info = _recorded_run(A, b, s_max=10, tol=1e-10, basis="chebyshev")
    checked = 0
    for rec in info["trace"][2:]:
        Y, sbar = rec["Y"], rec["sbar"]
        for l in range(1, sbar + 1):
            ref = _svd_cond(Y[:, O.sub_indices(sbar, l)])
            if ref < 1e5:
                got = rec["kappa"][l - 1]
                assert abs(got - ref) <= 1e-6 * ref, (rec["k"], l, got, ref)
                checked += 1
    assert checked > 100, checked


def pin_relative_residual_scale_invariance():
    """eps* is a relative tolerance (Section 3), and (3.2) and (4.7) compare
    against relative residual norms: scaling b by 2^20 or 2^-20 (exact in
    binary floating point) scales every vector of the run and leaves every
    decision, hence s~, s_k and the outer-loop count, unchanged."""
    cases = [(_geom_problem()[:2], dict(s_max=10, basis="chebyshev")),
             ((P.poisson2d(20), np.random.default_rng(31).standard_normal(400)),
              dict(s_max=10, basis="newton"))]
    for (A, b), kw in cases:
        ref = None
        for scale in (1.0, 2.0 ** 20, 2.0 ** -20):
            _, info = O.adaptive_sstep_cg(A, b * scale, tol=1e-10, **kw)
            sched = [(t["sbar"], t["stilde"], t["sk"]) for t in info["trace"]]
            if ref is None:
                ref = (info["outer"], sched)
                assert any(st < kw["s_max"] for _, st, _ in sched[2:])   # thr matters
            else:
                assert (info["outer"], sched) == ref, scale


def _rayleigh_ritz_extremes(alphas, betas, nsteps):
    """Brute force for Algorithms 3 and 4: explicit unit vectors and dense
    2x2 eigenproblems on T of (1.1) (largest) and on L^{-1} L^{-T} of (4.1)
    (whose largest eigenvalue is 1 / lambda_min(T)), bordered one row at a
    time."""
    T = O.lanczos_tridiagonal(alphas, betas, nsteps + 1)
    Lt = O.lanczos_cholesky_factor(alphas, betas, nsteps + 1)
    hi = _explicit_rayleigh_ritz(lambda k: T[:k, :k], nsteps)

    def inv_gram(k):
        W = np.linalg.inv(Lt[:k, :k].T)
        return W @ W.T
    lo = _explicit_rayleigh_ritz(inv_gram, nsteps)
    return np.array(hi), 1.0 / np.array(lo)


def pin_ritz_estimates_follow_the_run():
    """Algorithm 5 updates the estimates after global iteration i = m + j
    whenever i >= 1, from T_{i+1} built with the run's own alpha_0..alpha_i
    and beta_0..beta_{i-1}: the recorded lambda~max / lambda~min after each
    inner step equal explicit Rayleigh-Ritz values on that T."""
    A, b, _ = _geom_problem()
    _, info = _recorded_run(A, b, s_max=10, tol=1e-10, basis="chebyshev")
    steps = [st for rec in info["trace"] for st in rec["steps"]]
    nchk = 60
    hi, lo = _rayleigh_ritz_extremes(info["alphas"], info["betas"], nchk)
    assert math.isnan(steps[0]["lmax"]) and math.isnan(steps[0]["lmin"])
    for i in range(1, nchk + 1):
        assert abs(steps[i]["lmax"] - hi[i - 1]) <= 1e-10 * hi[i - 1], (i, steps[i]["lmax"], hi[i - 1])
        assert abs(steps[i]["lmin"] - lo[i - 1]) <= 1e-8 * lo[i - 1], (i, steps[i]["lmin"], lo[i - 1])


def pin_adaptive_c_follows_the_run():
    """(4.5)/(4.6) in the run: after every inner step the recorded psi equals
    ||r||^2 / ||p||^2 of the vectors Y r', Y p' of that step, and c equals
    max{1, lambda~max (psi / lambda~min)^(1/2)} with those estimates (the
    estimates themselves are pinned above); on this spectrum c is far above
    1, so both the estimates' roles and the max are exercised.  The identity
    behind (4.5) needs r_{i+1} orthogonal to p_i, which rounding erodes as
    the solve goes on (at kappa(A) = 1e4 the drift is ~1e-7 over the first
    150 iterations checked here and ~1e-6 by iteration 270), hence the 1e-5
    tolerance."""
    A, b, _ = _geom_problem()
    _, info = _recorded_run(A, b, s_max=10, tol=1e-10, basis="chebyshev")
    checked = 0
    for rec in info["trace"][1:]:
        Ys = rec["Y"][:, O.sub_indices(rec["sbar"], rec["stilde"])]
        if _svd_cond(Ys) > 1e5 or rec["m"] >= 150:
            continue
        for st in rec["steps"]:
            r, pv = Ys @ st["rc"], Ys @ st["pc"]
            psi = float(r @ r) / float(pv @ pv)
            assert abs(st["psi"] - psi) <= 1e-5 * psi, (rec["k"], st["psi"], psi)
            xi = st["lmax"] * math.sqrt(psi / st["lmin"])
            assert xi > 2.0
            assert abs(st["c"] - max(1.0, xi)) <= 1e-5 * xi, (rec["k"], st["c"], xi)
            checked += 1
    assert checked > 40, checked


def pin_basis_follows_ritz_estimates():
    """Algorithm 5 regenerates the basis parameters from the latest estimates
    after every loop once m > 1: on a diagonal A the P columns of loop k are
    T_l(2 (z - theta)/Delta) p with theta, Delta from the estimates at the
    end of loop k-1 (numpy's chebval); on the 2-D Poisson matrix the
    resulting basis is far better conditioned than the monomial basis built
    from the same p and r."""
    A, b, z = _geom_problem()
    _, info = _recorded_run(A, b, s_max=10, tol=1e-10, basis="chebyshev")
    tr = info["trace"]
    checked = 0
    for k in range(1, len(tr)):
        if tr[k]["m"] <= 1:
            continue
        lo, hi = tr[k - 1]["lmin"], tr[k - 1]["lmax"]
        Y, sbar = tr[k]["Y"], tr[k]["sbar"]
        p = Y[:, 0]
        t = 2.0 * (z - 0.5 * (lo + hi)) / (hi - lo)
        for l in range(sbar + 1):
            ref = npcheb.chebval(t, np.eye(sbar + 1)[l]) * p
            assert np.linalg.norm(Y[:, l] - ref) <= 1e-9 * np.linalg.norm(ref), (k, l)
        checked += 1
    assert checked > 50
    A = P.poisson2d(20)
    b = np.random.default_rng(31).standard_normal(400)
    _, info = _recorded_run(A, b, s_max=10, tol=1e-10, basis="chebyshev")
    # before m reaches sbar, [P, R] spans K_{m+sbar+1}(A, r_0) with 2 sbar + 1
    # columns and is singular for any polynomials
    late = [rec for rec in info["trace"] if rec["sbar"] == 10 and rec["m"] >= 10]
    assert len(late) >= 5
    for rec in late:
        Y = rec["Y"]
        mono = O.sstep_basis(A, Y[:, 0], Y[:, 11], 10, O.params_monomial(10))
        assert _svd_cond(Y) < 1e-3 * _svd_cond(mono), (rec["k"], _svd_cond(Y), _svd_cond(mono))


def pin_break_rule_4_7():
    """(4.7) as Algorithm 5 writes it: after inner step j < s~-1 the loop
    ends exactly when kappa(Y_{k,j+2}) >= eps* / (c_{m+j+1} eps phi), phi the
    largest relative residual norm of the loop so far.  Every decision of a
    run on a spectrum where this fires in several loops is recomputed with
    kappa from an SVD of the recorded basis and phi from the norms of the
    recovered residual vectors (decisions within 1e-4 of the threshold are
    skipped: there the two computations may legitimately differ)."""
    A, b, _ = _geom_problem()
    for kw in (dict(s_max=10, basis="chebyshev"), dict(s_max=15, basis="newton")):
        _, info = _recorded_run(A, b, tol=1e-10, **kw)
        nb = float(np.linalg.norm(b))
        verified_breaks = 0
        for rec in info["trace"]:
            st, sbar = rec["stilde"], rec["sbar"]
            Ys = rec["Y"][:, O.sub_indices(sbar, st)]
            phi = np.linalg.norm(rec["Y"][:, sbar + 1]) / nb
            for j, step in enumerate(rec["steps"]):
                phi = max(phi, np.linalg.norm(Ys @ step["rc"]) / nb)
                if j >= st - 1 or step["rho"] <= 1e-10:
                    continue
                gamma = _svd_cond(rec["Y"][:, O.sub_indices(sbar, j + 2)])
                thr = 1e-10 / (step["c"] * U * phi)
                if abs(gamma / thr - 1.0) < 1e-4 + 16 * U * gamma * gamma:
                    continue
                broke_here = rec["broke"] and j == rec["sk"] - 1
                assert (gamma >= thr) == broke_here, (rec["k"], j, gamma, thr, rec["sk"])
                verified_breaks += broke_here
        assert verified_breaks >= 5, verified_breaks


def pin_stilde_is_first_failure():
    """(3.2): s~ is the largest l whose basis passes; kappa(Y_{k,l}) is
    nondecreasing in l in exact arithmetic (interlacing), so on monotone
    values this is the paper's literal maximum, at least 1.  On values whose
    order rounding has broken (a numerically singular G reporting kappa = inf
    before a finite value), no basis past the first failure is taken, so
    every sub-basis the inner loop uses passes (3.2).  Runs obey the same:
    every kappa(Y_{k,l}), l <= s~, passes whenever s~ > 1."""
    rng = np.random.default_rng(41)
    for _ in range(200):
        kap = np.sort(10.0 ** rng.uniform(0, 8, rng.integers(1, 17)))
        thr = 10.0 ** rng.uniform(0, 8)
        passing = [l for l in range(1, kap.size + 1) if kap[l - 1] <= thr]
        assert O.select_stilde(list(kap), thr) == (max(passing) if passing else 1)
    assert O.select_stilde([2.0, 5.0, math.inf, 3.0, 4.0], 10.0) == 2
    assert O.select_stilde([2.0, 50.0, 3.0], 10.0) == 1
    assert O.select_stilde([math.inf, 1.0], 10.0) == 1
    A, b, _ = _geom_problem()
    _, info = O.adaptive_sstep_cg(A, b, s_max=15, tol=1e-10, basis="newton")
    for rec in info["trace"]:
        if rec["stilde"] > 1:
            assert all(kp <= rec["thr"] for kp in rec["kappa"][:rec["stilde"]]), rec["k"]


ALL_PINS = [v for k, v in dict(globals()).items() if k.startswith("pin_")]
