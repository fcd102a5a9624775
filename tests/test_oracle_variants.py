"""Pins of the oracle's comparison variants (Section 5): fixed s-step CG,
the adaptive s-step CG of Algorithm 2 with a constant c_k, and Algorithm 5
with c = 1 or c = lambda~max / lambda~min.  Each variant is tied to another
computation it must reduce to, and the qualitative outcomes the paper
reports for the monomial basis at large s are reproduced."""
import numpy as np

import oracle as O
import spd_problems as P


def _pr():
    return P.make_config("poisson2d_64", size=24)


def test_fixed_s1_is_hscg():
    """s = 1: one CG step per outer loop (Section 2), the iterates of HSCG."""
    pr = _pr()
    xh, ih = O.hscg(pr.A, pr.b, pr.x0, tol=1e-10)
    xf, jf = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=1, tol=1e-10, variant="fixed")
    assert jf["outcome"] == O.Outcome.CONVERGED
    assert jf["iters"] == ih["iters"] and jf["outer"] == ih["iters"]
    assert np.linalg.norm(xf - xh) <= 1e-10 * np.linalg.norm(xh)


def test_fixed_runs_full_blocks():
    pr = _pr()
    _, info = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=6, tol=1e-10, variant="fixed")
    tr = info["trace"]
    assert all(t["stilde"] == t["sbar"] == 6 for t in tr)
    assert all(t["sk"] == 6 for t in tr[:-1])


def test_old_with_negligible_c_never_limits_s():
    """c_k -> 0 puts the threshold of (3.2) and of Algorithm 2's break test
    out of reach: s~ is the largest l whose leading blocks all have a
    positive definite Gram matrix (kappa finite; the first loop has p = r,
    so only l = 1... fails there), and every loop but the last runs all s~
    steps."""
    pr = _pr()
    _, jo = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=5, tol=1e-10, variant="old",
                                c_const=1e-200)
    assert jo["outcome"] == O.Outcome.CONVERGED
    for t in jo["trace"]:
        fin = np.isfinite(t["kappa"])
        expect = max(1, int(np.argmin(fin)) if not fin.all() else len(fin))
        assert t["stilde"] == expect, (t["k"], t["stilde"], t["kappa"])
    assert all(t["sk"] == t["stilde"] for t in jo["trace"][:-1])


def test_old_with_huge_c_takes_single_steps():
    """c_k -> inf fails (3.2) for every l: s~ = 1 in every loop, CG one step
    per outer loop."""
    pr = _pr()
    xh, ih = O.hscg(pr.A, pr.b, pr.x0, tol=1e-10)
    xo, jo = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=8, tol=1e-10, variant="old",
                                 c_const=1e300)
    assert all(t["stilde"] == 1 and t["sk"] == 1 for t in jo["trace"])
    assert jo["iters"] == ih["iters"]
    assert np.linalg.norm(xo - xh) <= 1e-9 * np.linalg.norm(xh)


def test_improved_c_choices():
    pr = _pr()
    _, one = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10,
                                 variant="improved_c_one")
    assert all(t["c"] == 1.0 and t["c_in"] == 1.0 for t in one["trace"])
    _, rat = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=10, tol=1e-10,
                                 variant="improved_c_ratio")
    for t in rat["trace"]:
        if np.isfinite(t["lmax"]):
            assert t["c"] == t["lmax"] / t["lmin"]


def test_monomial_variants_fail_at_large_s_where_improved_converges():
    """The pattern of the paper's tables: with s = 15 the monomial basis
    breaks fixed s-step CG down and slows or stops the old adaptive method,
    while Algorithm 5 converges in about HSCG's iteration count."""
    pr = P.make_config("poisson2d_64")
    _, ih = O.hscg(pr.A, pr.b, pr.x0, tol=1e-10)
    _, jf = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=15, tol=1e-10, variant="fixed")
    _, jo = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=15, tol=1e-10, variant="old")
    _, ji = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, s_max=15, tol=1e-10, basis="chebyshev")
    assert jf["outcome"] != O.Outcome.CONVERGED
    assert jo["outcome"] != O.Outcome.CONVERGED or jo["iters"] > 2 * ih["iters"]
    assert ji["outcome"] == O.Outcome.CONVERGED
    assert abs(ji["iters"] - ih["iters"]) <= 0.05 * ih["iters"]
    assert ji["outer"] < ih["iters"] / 8
