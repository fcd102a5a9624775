"""Improved adaptive s-step CG, Algorithm 5 of the paper (Section 4).
Oracle: test infrastructure only.

Everything is FP64 numpy, in the paper's column order Y = [P, R].  The
places where the paper is silent or inconsistent follow these readings
(each also marked in the code):

* unit roundoff eps = 2^-53 (Section 5 states eps ~ 2^-53), c_1 = eps^{-1/2};
* residual norms in the s-selection condition (3.2) and the break test
  (4.7) are relative, ||r||/||b||, as is the tolerance eps* (Section 3);
* s~ is the largest l reached by scanning l = 1..sbar upward until (3.2)
  first fails, and at least 1; a sub-Gram matrix whose smallest eigenvalue
  is not positive counts as kappa = inf;
* gamma_l = kappa(Y_{k,l+1}) as in Algorithm 5 (the break after inner step j
  tests gamma_{j+1});
* the Ritz estimates start at global iteration 0 and are stepped for
  m+j+1 > 1; the current c (c_1 until the first update) is used in (3.2)
  and in the break test;
* convergence: when the updated relative residual (r'^T G r')^{1/2}/||b||
  reaches eps* the inner loop ends (s_k = j+1); after recovery the true
  relative residual ||b - A x||/||b|| decides.  Five failed confirmations
  in a row without a 10% improvement of the best true residual stop the
  solve as STAGNATED;
* quadratic forms r'^T G r' are clamped at 0 (G may be numerically
  indefinite); p'^T G B p' <= 0 is a BREAKDOWN, non-finite values DIVERGED;
* basis parameters switch from monomial once m > 1 and are regenerated after
  every outer loop from the latest estimates, unless lambda_max - lambda_min
  is not positive and finite (then the previous ones are kept).

Comparison variants of Section 5 (``variant``):

* "improved": Algorithm 5 as above, c = xi~ of (4.6);
* "improved_c_ratio": Algorithm 5 with c = lambda~max / lambda~min, updated
  with the estimates every iteration (Section 5.1; c_1 until the first
  update);
* "improved_c_one": Algorithm 5 with the constant c = 1 (Section 5.1);
* "old": the adaptive s-step CG of Algorithm 2 with the monomial basis
  throughout and a constant c_k = ``c_const`` (the algorithm leaves c_k to
  the user; 1 by default): s~ by (3.2), gamma = kappa(Y_{k,s~}) of the
  selected basis, break after step j when gamma >= eps* / (c_k eps rho_{j+1})
  with the current relative residual rho_{j+1};
* "fixed": fixed s-step CG, monomial basis, s_k = s-bar = sigma in every
  outer loop (no selection, no break); the stopping test is the same.

Pins (tests/pins.py) fix the solve as a whole (HSCG at sigma = 1, the
monomial basis against HSCG's coefficients, convergence against a dense
Cholesky solve), the Ritz estimates, the basis recurrences, B, psi and
c >= 1, and the adaptive control of each run against quantities computed
without this code: kappa against an SVD of the recorded basis, the
relative-residual reading by exact power-of-two scaling of b, the Ritz
estimates after every inner step against explicit Rayleigh-Ritz problems on
T, psi and c against the recovered vectors, the basis of every loop against
the Chebyshev closed form of the previous loop's estimates, every (4.7)
decision of a run where the break fires in many loops (index, phi and
eps = 2^-53 included), and the first-failure rule of the s~ scan.
"""
from __future__ import annotations

import math

import numpy as np

from .basis import change_of_basis, make_params, sstep_basis, sub_indices
from .outcome import Outcome
from .ritz import MaxRitzEstimate, MinRitzEstimate, psi_update

UNIT_ROUNDOFF = 2.0 ** -53


def select_stilde(kappa, thr) -> int:
    """s~ of (3.2): the largest l in 1..sbar for which kappa(Y_{k,l}) <=
    thr (``kappa[l-1]`` = kappa(Y_{k,l})).

    Reading: the scan runs upward and stops at the first l that fails, with
    s~ >= 1 even when l = 1 fails.  Y_{k,l} is a column subset of
    Y_{k,l+1}, so by interlacing kappa(Y_{k,l}) is nondecreasing in l in
    exact arithmetic and this is the largest passing l; computed values can
    break that order only through rounding on a numerically singular G, and
    then no sub-basis past the first failure is taken."""
    stilde = 1
    for l in range(1, len(kappa) + 1):
        if kappa[l - 1] <= thr:
            stilde = l
        else:
            break
    return stilde


def _kappa_sub(G, idx) -> float:
    """sqrt(kappa(G_sub)) ~ kappa(Y_sub) (Section 3), from the eigenvalues of
    the principal submatrix of G on ``idx``."""
    ev = np.linalg.eigvalsh(G[np.ix_(idx, idx)])
    lo, hi = ev[0], ev[-1]
    if not (lo > 0.0 and np.isfinite(lo) and np.isfinite(hi)):
        return math.inf
    return math.sqrt(hi / lo)


VARIANTS = ("improved", "improved_c_ratio", "improved_c_one", "old", "fixed")


def adaptive_sstep_cg(A, b, x0=None, s_max=10, s_init=None, growth=None, tol=1e-10,
                      basis="chebyshev", max_outer=None, max_iters=None, record=True,
                      record_gram=False, record_basis=False, variant="improved",
                      c_const=1.0):
    """Solve A x = b by the improved adaptive s-step CG (Algorithm 5).

    Parameters follow the algorithm's inputs: sigma = ``s_max``,
    s-bar_0 = ``s_init`` (default sigma), f = ``growth`` (default sigma),
    eps* = ``tol``; ``basis`` is "chebyshev", "newton" or "monomial" (the
    last keeps the monomial basis throughout).
    Returns (x, info); ``info["trace"]`` has one record per outer loop.
    With ``record_gram`` each record also keeps G (paper order), the carried
    state at the start of the loop and, per inner step, the scalars and the
    coordinate vectors after the step (for step-by-step comparisons); with
    ``record_basis`` it keeps the basis Y itself (small problems only).
    """
    if variant not in VARIANTS:
        raise ValueError(f"unknown variant {variant!r}")
    improved = variant.startswith("improved")
    if not improved:
        basis = "monomial"
    A = A.tocsr() if hasattr(A, "tocsr") else A
    b = np.asarray(b, dtype=np.float64)
    N = b.size
    sigma = int(s_max)
    sbar0 = sigma if s_init is None else int(s_init)
    f = sigma if growth is None else int(growth)
    if max_iters is None:
        max_iters = 10 * N
    if max_outer is None:
        max_outer = max_iters
    u = UNIT_ROUNDOFF
    nb = float(np.linalg.norm(b))
    x = np.zeros(N) if x0 is None else np.array(x0, dtype=np.float64)
    info = {"outcome": Outcome.MAX_ITER, "outer": 0, "iters": 0, "relres_true": np.nan,
            "relres_updated": np.nan, "lmin": np.nan, "lmax": np.nan, "c": np.nan,
            "trace": [], "alphas": [], "betas": []}
    if nb == 0.0:
        x[:] = 0.0
        info.update(outcome=Outcome.CONVERGED, relres_true=0.0, relres_updated=0.0)
        return x, info

    r = b - A @ x
    p = r.copy()
    psi = 1.0
    c = {"improved_c_one": 1.0, "old": float(c_const)}.get(variant, u ** -0.5)
    m = 0
    params = make_params("monomial", sigma)
    mt_max = mt_min = None
    lmin = lmax = math.nan
    alpha_prev = beta_prev = None
    s_prev = None
    best, streak = math.inf, 0
    outcome = None
    k = 0
    while outcome is None:
        sbar = sbar0 if k == 0 else min(s_prev + f, sigma)
        Y = sstep_basis(A, p, r, sbar, params)
        G = Y.T @ Y
        rec = {"k": k, "sbar": sbar, "m": m, "c_in": c}
        if record_basis:
            rec["Y"] = Y.copy()
        if record_gram:
            rec["G"] = G.copy()
            rec["steps"] = []
            rec["state_in"] = {
                "m": m, "c": c, "psi": psi, "alpha_prev": alpha_prev, "beta_prev": beta_prev,
                "mt_max": None if mt_max is None else (mt_max.omega, mt_max.h, mt_max.zeta),
                "mt_min": None if mt_min is None else (mt_min.omega, mt_min.a, mt_min.d,
                                                       mt_min.g, mt_min.h),
                "lmin": lmin, "lmax": lmax,
                "params": tuple(np.array(q, dtype=np.float64) for q in params),
            }
        if not np.all(np.isfinite(G)):
            outcome = Outcome.DIVERGED
            info["trace"].append(rec)
            break
        r_idx = sbar + 1                        # column of R_0 = r_m
        rho_m = math.sqrt(max(G[r_idx, r_idx], 0.0)) / nb
        thr = tol / (c * u * rho_m) if rho_m > 0.0 else math.inf
        kappa = [math.nan] + [_kappa_sub(G, sub_indices(sbar, l)) for l in range(1, sbar + 1)]
        stilde = select_stilde(kappa[1:], thr)
        if variant == "fixed":
            stilde = sbar
        gam = {l: kappa[l + 1] for l in range(1, stilde)}
        idx = sub_indices(sbar, stilde)
        Gs = G[np.ix_(idx, idx)]
        B = change_of_basis(stilde, params)
        n = 2 * stilde + 1
        pc = np.zeros(n); pc[0] = 1.0
        rc = np.zeros(n); rc[stilde + 1] = 1.0
        xc = np.zeros(n)
        rGr = max(float(rc @ Gs @ rc), 0.0)
        phi = math.sqrt(rGr) / nb
        candidate = False
        broke = False
        sk = 0
        rec.update(thr=thr, kappa=kappa[1:], stilde=stilde, rho_m=rho_m)
        for j in range(stilde):
            sk = j + 1
            Bp = B @ pc
            den = float(pc @ (Gs @ Bp))
            if not np.isfinite(den):
                outcome = Outcome.DIVERGED
                break
            if den <= 0.0 or rGr <= 0.0:
                outcome = Outcome.BREAKDOWN
                break
            alpha = rGr / den
            q = alpha * pc
            xc = xc + q
            rc_new = rc - B @ q
            rGr_new = max(float(rc_new @ Gs @ rc_new), 0.0)
            beta = rGr_new / rGr
            pc = rc_new + beta * pc
            rc = rc_new
            rGr = rGr_new
            rho = math.sqrt(rGr) / nb
            phi = max(phi, rho)
            psi = psi_update(psi, beta)
            i = m + j                           # global index of this iteration
            zeta = 1.0 / math.sqrt(alpha)
            if i == 0:
                mt_max = MaxRitzEstimate(zeta)
                mt_min = MinRitzEstimate(zeta)
            else:
                eta = math.sqrt(beta_prev / alpha_prev)
                lmax = mt_max.step(eta, zeta)
                lmin = mt_min.step(eta, zeta)
                if variant == "improved":
                    c = max(1.0, lmax * math.sqrt(psi / lmin))          # (4.6)
                elif variant == "improved_c_ratio":
                    c = lmax / lmin
            alpha_prev, beta_prev = alpha, beta
            info["alphas"].append(alpha)
            info["betas"].append(beta)
            if record_gram:
                rec["steps"].append({"alpha": alpha, "beta": beta, "rho": rho, "phi": phi,
                                     "psi": psi, "c": c, "lmin": lmin, "lmax": lmax,
                                     "rc": rc.copy(), "pc": pc.copy()})
            if not (np.isfinite(alpha) and np.isfinite(beta)):
                outcome = Outcome.DIVERGED
                break
            if rho <= tol:
                candidate = True
                break
            if improved:
                if j < stilde - 1 and gam[j + 1] >= tol / (c * u * phi):   # (4.7)
                    broke = True
                    break
            elif variant == "old":
                if j < stilde - 1 and kappa[stilde] >= tol / (c * u * rho):
                    broke = True
                    break
        rec.update(sk=sk, phi=phi, c=c, lmin=lmin, lmax=lmax, psi=psi,
                   relres_updated=math.sqrt(rGr) / nb, candidate=candidate, broke=broke)
        if record_gram:
            rec.update(xc=xc.copy(), rc=rc.copy(), pc=pc.copy(),
                       alphas=info["alphas"][m:m + sk], betas=info["betas"][m:m + sk])
        if outcome is not None and outcome != Outcome.CONVERGED:
            info["trace"].append(rec)
            break
        # recovery (2.6): x += Y x', r = Y r', p = Y p'
        Ys = Y[:, idx]
        x = x + Ys @ xc
        r = Ys @ rc
        p = Ys @ pc
        m += sk
        s_prev = sk
        if improved and m > 1 and np.isfinite(lmax) and np.isfinite(lmin) and lmax - lmin > 0.0:
            params = make_params(basis, sigma, lmin, lmax) if basis != "monomial" \
                else make_params("monomial", sigma)
        k += 1
        info["relres_updated"] = math.sqrt(rGr) / nb
        if candidate:
            true_rel = float(np.linalg.norm(b - A @ x)) / nb
            rec["relres_true"] = true_rel
            info["relres_true"] = true_rel
            if true_rel <= tol:
                outcome = Outcome.CONVERGED
            elif true_rel < 0.9 * best:
                best, streak = true_rel, 0
            else:
                streak += 1
                if streak >= 5:
                    outcome = Outcome.STAGNATED
        info["trace"].append(rec)
        if outcome is None and (m >= max_iters or k >= max_outer):
            outcome = Outcome.MAX_ITER
    info.update(outcome=outcome, outer=k, iters=m, lmin=lmin, lmax=lmax, c=c)
    if outcome != Outcome.CONVERGED or np.isnan(info["relres_true"]):
        info["relres_true"] = float(np.linalg.norm(b - A @ x)) / nb
    return x, info
