"""Hestenes-Stiefel CG, Algorithm 1 of the paper (Section 1).  Oracle: test
infrastructure only."""
from __future__ import annotations

import numpy as np

from .outcome import Outcome


def hscg(A, b, x0=None, tol=1e-10, max_iters=None, record=False, record_vectors=False):
    """Solve A x = b with HSCG (Algorithm 1).

    One SpMV w = A p per iteration; alpha = r'r / p'w; x += alpha p;
    r -= alpha w; beta = r_new'r_new / r'r; p = r_new + beta p.

    Stopping (the paper says only "until convergence"; Reading: the same
    rule as the s-step method): when the updated relative residual
    ||r||/||b|| drops to ``tol`` the true relative residual ||b - A x||/||b||
    is computed; the solve ends when that is <= tol.  Returns (x, info) with
    the iteration count and, with ``record``, the alpha/beta sequences and the
    residual vectors' norms; with ``record_vectors`` (small systems only) the
    residual vectors r_0, r_1, ... themselves.
    """
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if max_iters is None:
        max_iters = 10 * n
    nb = float(np.linalg.norm(b))
    info = {"outcome": Outcome.MAX_ITER, "iters": 0, "relres_true": np.nan,
            "relres_updated": np.nan, "alphas": [], "betas": [], "rnorms": [], "pnorms": [],
            "rvecs": []}
    if nb == 0.0:
        x[:] = 0.0
        info.update(outcome=Outcome.CONVERGED, relres_true=0.0, relres_updated=0.0)
        return x, info
    r = b - A @ x
    p = r.copy()
    rr = float(r @ r)
    if record:
        info["rnorms"].append(np.sqrt(rr)); info["pnorms"].append(np.sqrt(rr))
    if record_vectors:
        info["rvecs"].append(r.copy())
    best, streak = np.inf, 0
    for i in range(max_iters):
        w = A @ p
        pw = float(p @ w)
        if not (pw > 0.0 and np.isfinite(pw)):
            info["outcome"] = Outcome.BREAKDOWN if np.isfinite(pw) else Outcome.DIVERGED
            info["iters"] = i
            break
        alpha = rr / pw
        q = alpha * p
        x += q
        r -= alpha * w
        rr_new = float(r @ r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        info["iters"] = i + 1
        if record:
            info["alphas"].append(alpha); info["betas"].append(beta)
            info["rnorms"].append(np.sqrt(rr)); info["pnorms"].append(float(np.linalg.norm(p)))
        if record_vectors:
            info["rvecs"].append(r.copy())
        rel = np.sqrt(rr) / nb
        info["relres_updated"] = rel
        if not np.isfinite(rel):
            info["outcome"] = Outcome.DIVERGED
            break
        if rel <= tol:
            true_rel = float(np.linalg.norm(b - A @ x)) / nb
            info["relres_true"] = true_rel
            if true_rel <= tol:
                info["outcome"] = Outcome.CONVERGED
                break
            if true_rel < 0.9 * best:
                best, streak = true_rel, 0
            else:
                streak += 1
                if streak >= 5:
                    info["outcome"] = Outcome.STAGNATED
                    break
    if np.isnan(info["relres_true"]) or info["outcome"] != Outcome.CONVERGED:
        info["relres_true"] = float(np.linalg.norm(b - A @ x)) / nb
    return x, info
