"""s-step bases (oracle; test infrastructure only).

* Basis parameters: monomial (Section 2, after (2.5)), Newton with Leja
  ordered shifts (2.7), Chebyshev (2.8).
* ``polynomial_columns``: rho_0(A)v, ..., rho_L(A)v by the three-term
  recurrence (2.3).
* ``sstep_basis``: Y_{k,s} = [P_{k,s}, R_{k,s}] of (2.2), paper column order.
* ``change_of_basis``: the block matrix of (2.5) with A Y_ = Y B (2.4).
* ``sub_indices``: the columns of Y_{k,l} inside Y_{k,sbar}.
"""
from __future__ import annotations

import numpy as np


# --------------------------------------------------------------------------
# Newton shifts: Leja ordering on the real interval (2.7)
# --------------------------------------------------------------------------
def _log_prod_dist(t: float, pts) -> float:
    return float(np.sum(np.log(np.abs(t - np.asarray(pts)))))


def leja_reference_points(count: int) -> np.ndarray:
    """Leja points of [-1, 1] in the order of (2.7): t_0 = 1 (lambda_max),
    t_1 = -1 (lambda_min), t_l = argmax over [-1, 1] of prod_m |t - t_m|.

    Reading: the ordering is affine invariant, so the points are computed
    once on [-1, 1] and mapped to [lambda_min, lambda_max].  The maximum is
    found among the critical points of the product polynomial (roots of its
    derivative, polished by Newton's method on the logarithmic derivative,
    which is monotone between consecutive points).  When several candidates
    attain the maximum to a relative 1e-9 (symmetric ties such as
    t_3 = -1/sqrt(3) versus +1/sqrt(3)), the smallest t is taken.
    """
    pts = [1.0, -1.0][:count]
    while len(pts) < count:
        coeffs = np.poly(np.asarray(pts))          # monic prod (t - t_m)
        crit = np.roots(np.polyder(coeffs))
        cand = []
        srt = np.sort(np.asarray(pts))
        for z in crit:
            if abs(z.imag) > 1e-8:
                continue
            t = float(z.real)
            # Newton polish on f(t) = sum 1/(t - t_m) inside the gap holding t
            k = np.searchsorted(srt, t)
            if k == 0 or k == srt.size:
                continue
            lo, hi = srt[k - 1], srt[k]
            for _ in range(60):
                f = float(np.sum(1.0 / (t - srt)))
                fp = -float(np.sum(1.0 / (t - srt) ** 2))
                tn = t - f / fp
                if not (lo < tn < hi):
                    tn = 0.5 * (t + (lo if f < 0 else hi))
                if tn == t:
                    break
                t = tn
            cand.append(t)
        vals = np.array([_log_prod_dist(t, pts) for t in cand])
        best = vals.max()
        # log-domain tie window equivalent to a relative 1e-9 on the product
        ties = [t for t, v in zip(cand, vals) if v >= best - 1e-9]
        pts.append(min(ties))
    return np.asarray(pts)


# --------------------------------------------------------------------------
# Basis parameters: arrays theta (s), gamma (s), mu (max(s-1, 0))
# --------------------------------------------------------------------------
def params_monomial(s: int):
    """theta = 0, gamma = 1, mu = 0: the monomial basis of (2.3) (Section 2),
    used before the first Ritz estimates and by the comparison methods."""
    return np.zeros(s), np.ones(s), np.zeros(max(s - 1, 0))


def params_newton(lmin: float, lmax: float, s: int):
    """Newton basis (2.7): mu = 0, gamma = 1, theta_0 = lambda_max,
    theta_1 = lambda_min, theta_l (l >= 2) the Leja points of
    [lambda_min, lambda_max], computed as (lmin+lmax)/2 + ((lmax-lmin)/2) t_l."""
    t = leja_reference_points(max(s, 2))
    c = 0.5 * (lmin + lmax)
    h = 0.5 * (lmax - lmin)
    theta = np.empty(s)
    for l in range(s):
        theta[l] = lmax if l == 0 else (lmin if l == 1 else c + h * t[l])
    return theta, np.ones(s), np.zeros(max(s - 1, 0))


def params_chebyshev(lmin: float, lmax: float, s: int):
    """Chebyshev basis on [lambda_min, lambda_max].

    Reading of (2.8): theta_l = (lmin+lmax)/2 as printed, but gamma_0 =
    Delta/2 and gamma_l = mu_l = Delta/4 (Delta = lmax - lmin), so that
    rho_l(z) = T_l(2 (z - theta)/Delta) exactly.  With the printed
    gamma_0 = Delta, gamma_l = Delta/2 the recurrence yields
    c^l T_l(t/(2c)) with c^2 = 2 mu / Delta; the printed mu = 2 Delta gives
    c = 2, a Chebyshev polynomial of an interval four times too wide (a worse
    conditioned basis than the monomial one in practice), contradicting the
    paper's results; only mu = Delta/8 would match the interval.
    """
    c = 0.5 * (lmin + lmax)
    d = lmax - lmin
    theta = np.full(s, c)
    gamma = np.full(s, 0.25 * d)
    if s > 0:
        gamma[0] = 0.5 * d
    mu = np.full(max(s - 1, 0), 0.25 * d)
    return theta, gamma, mu


def make_params(kind: str, s: int, lmin=None, lmax=None):
    """(theta, gamma, mu) of the recurrence (2.3) for the monomial basis, the
    Newton basis (2.7) or the Chebyshev basis (2.8) on [lmin, lmax]."""
    if kind == "monomial":
        return params_monomial(s)
    if kind == "newton":
        return params_newton(lmin, lmax, s)
    if kind == "chebyshev":
        return params_chebyshev(lmin, lmax, s)
    raise ValueError(kind)


# --------------------------------------------------------------------------
# Basis vectors and change of basis
# --------------------------------------------------------------------------
def polynomial_columns(A, v, nlev: int, theta, gamma, mu) -> np.ndarray:
    """Columns rho_0(A) v .. rho_nlev(A) v of the recurrence (2.3):
    rho_0 = 1, rho_1 = (z - theta_0)/gamma_0,
    rho_l = ((z - theta_{l-1}) rho_{l-1} - mu_{l-2} rho_{l-2}) / gamma_{l-1}."""
    v = np.asarray(v, dtype=np.float64)
    cols = np.empty((v.size, nlev + 1))
    cols[:, 0] = v
    for l in range(1, nlev + 1):
        y = A @ cols[:, l - 1] - theta[l - 1] * cols[:, l - 1]
        if l >= 2:
            y = y - mu[l - 2] * cols[:, l - 2]
        cols[:, l] = y / gamma[l - 1]
    return cols


def sstep_basis(A, p, r, s: int, params) -> np.ndarray:
    """Y_{k,s} = [P_{k,s}, R_{k,s}] of (2.2): s+1 columns from p, s from r."""
    theta, gamma, mu = params
    P = polynomial_columns(A, p, s, theta, gamma, mu)
    R = polynomial_columns(A, r, s - 1, theta, gamma, mu)
    return np.concatenate([P, R], axis=1)


def _B_block(i: int, theta, gamma, mu) -> np.ndarray:
    """B_i of (2.5): column j (j <= i-2) holds theta_j on the diagonal,
    gamma_j below it and mu_{j-1} above it; the last column is zero."""
    B = np.zeros((i, i))
    for j in range(i - 1):
        B[j, j] = theta[j]
        B[j + 1, j] = gamma[j]
        if j >= 1:
            B[j - 1, j] = mu[j - 1]
    return B


def change_of_basis(s: int, params) -> np.ndarray:
    """The (2s+1) x (2s+1) matrix blkdiag(B_{s+1}, B_s) of (2.5).

    Reading: for a basis restricted to s < sbar levels the same parameter
    sequence is used, and the last P column and last R column are zero (the
    underlined Y zeroes columns s+1 and 2s+1)."""
    theta, gamma, mu = params
    n = 2 * s + 1
    B = np.zeros((n, n))
    B[: s + 1, : s + 1] = _B_block(s + 1, theta, gamma, mu)
    B[s + 1:, s + 1:] = _B_block(s, theta, gamma, mu)
    return B


def sub_indices(sbar: int, l: int) -> np.ndarray:
    """Columns of Y_{k,l} = [P_{k,l}, R_{k,l}] inside Y_{k,sbar} (paper
    order, (2.2) and Section 3): P_0..P_l are columns 0..l, R_0..R_{l-1} are
    sbar+1..sbar+l.

    Reading: the "leading principal submatrices" of G used for kappa(Y_{k,l})
    are the principal submatrices on exactly these columns."""
    return np.concatenate([np.arange(l + 1), sbar + 1 + np.arange(l)]).astype(np.int64)
