"""Helpers shared by the GPU tests (no tests here)."""
import json
import math
import os

import numpy as np

import oracle as O
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def interleave_perm(s: int) -> np.ndarray:
    """perm[c] = paper-order ([P, R]) index of interleaved column c
    ([p0, r0, p1, r1, ..., p_s])."""
    perm = np.empty(2 * s + 1, dtype=np.int64)
    for c in range(2 * s + 1):
        perm[c] = c // 2 if c % 2 == 0 else s + 1 + (c - 1) // 2
    return perm


def to_interleaved_matrix(G, s):
    p = interleave_perm(s)
    return G[np.ix_(p, p)]


def to_interleaved_vec(v, s):
    return np.asarray(v)[interleave_perm(s)]


def block_state_from_oracle(L, st):
    """assg_block_state_t from an oracle trace record's state_in."""
    S = L.AssgBlockState()
    nan = math.nan
    S.m = st["m"]
    S.c = st["c"]
    S.psi = st["psi"]
    S.alpha_prev = nan if st["alpha_prev"] is None else st["alpha_prev"]
    S.beta_prev = nan if st["beta_prev"] is None else st["beta_prev"]
    mx = st["mt_max"] or (nan, nan, nan)
    mn = st["mt_min"] or (nan, nan, nan, nan, nan)
    S.mt_max_omega, S.mt_max_h, S.mt_max_zeta = mx
    S.mt_min_omega, S.mt_min_a, S.mt_min_d, S.mt_min_g, S.mt_min_h = mn
    S.lmin = st["lmin"]
    S.lmax = st["lmax"]
    th, ga, mu = st["params"]
    for l in range(L.MAX_S):
        S.theta[l] = th[l] if l < th.size else 0.0
        S.gamma[l] = ga[l] if l < ga.size else 1.0
        S.mu[l] = mu[l] if l < mu.size else 0.0
    return S


def first_divergence(tg, to, tol):
    """Index of the first outer loop in which the GPU trace ``tg`` and the
    oracle trace ``to`` take a different decision: s-bar, s~, s_k, the
    stopping candidate, or (both checked) the true-residual confirmation;
    the shorter length when one trace is a prefix of the other."""
    for k, (a, b) in enumerate(zip(tg, to)):
        if (a["sbar"], a["stilde"], a["sk"], bool(a["candidate"])) != \
                (b["sbar"], b["stilde"], b["sk"], bool(b["candidate"])):
            return k
        if a["candidate"] and "relres_true" in b and a["relres_true"] >= 0:
            if (a["relres_true"] <= tol) != (b["relres_true"] <= tol):
                return k
    return min(len(tg), len(to))


def _log_fallback(entry):
    path = os.environ.get("ASSG_PARITY_LOG")
    if path:
        with open(path, "a") as f:
            f.write(json.dumps(entry) + "\n")
    print("outer-loop fallback:", json.dumps(entry))


def check_outer_parity(torch, L, h, pr, ig, xo, io, opts, tg=None, case=""):
    """The outer-loop bar: the GPU's count within +-1 of the oracle's.

    Algorithm 5 compares kappa(Y_{k,l}) and residual norms against thresholds
    ((3.2), (4.7), the stopping test), so where one of these sits within
    rounding of its threshold two correct implementations that sum in
    different orders part ways.  When the counts differ by more than one:

    * the decision logic is cleared on identical input: the device
      controller, fed the oracle's G and carried state of the first loop in
      which the two traces differ, takes the oracle's decision there
      (Algorithm 5 only; the comparison methods have no controller replay);
    * the arithmetic is cleared along the oracle's whole trajectory: the GPU,
      replaying the oracle's s_k schedule (assg_solve_forced_schedule),
      converges at the end of the schedule, or (where the last loop's
      residual lands just above the tolerance: late in a run two roundings
      of CG give residual histories a few per cent apart) one loop later,
      with the solution within 1e-8 of the oracle's;
    * the case, the two counts and the loop where the trajectories part are
      reported (printed, and appended to $ASSG_PARITY_LOG when set)."""
    dk = ig["outer_iters"] - io["outer"]
    if abs(dk) <= 1:
        return
    tol = opts["tol"]
    variant = opts.get("variant", "improved")
    entry = {"case": case, "gpu_outer": ig["outer_iters"], "oracle_outer": io["outer"]}
    nb = float(np.linalg.norm(pr.b))
    # the oracle again with G and the carried state of every loop
    _, ir = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, record_gram=True, **_oracle_kw(opts))
    to = ir["trace"]
    assert ir["outer"] == io["outer"]
    if tg is not None:
        k = first_divergence(tg, to, tol)
        entry["first_divergence"] = k
        if k < min(len(tg), len(to)):
            a, b = tg[k], to[k]
            entry["gpu"] = {"stilde": a["stilde"], "sk": a["sk"], "candidate": a["candidate"]}
            entry["oracle"] = {"stilde": b["stilde"], "sk": b["sk"],
                               "candidate": bool(b["candidate"])}
            if a["stilde"] != b["stilde"]:
                l = min(a["stilde"], b["stilde"]) + 1
                if l <= b["sbar"]:
                    entry["kappa_over_thr"] = {"gpu": a["kappa"][l - 1] / a["thr"],
                                               "oracle": b["kappa"][l - 1] / b["thr"]}
            if variant == "improved" and b["sbar"] == a["sbar"]:
                sbar = b["sbar"]
                S = block_state_from_oracle(L, b["state_in"])
                res = L.assg_block_controller(h, to_interleaved_matrix(b["G"], sbar), sbar, nb,
                                              tol, opts.get("basis", "chebyshev"),
                                              opts["s_max"], S)
                assert (res.stilde, res.sk, bool(res.candidate)) == \
                    (b["stilde"], b["sk"], bool(b["candidate"])), (case, k, res.stilde, res.sk)
    sk = np.array([rec["sk"] for rec in to], dtype=np.int32)
    Ad = L.csr_to_device(pr.A)
    L.assg_analyze(h, Ad)
    b = torch.from_numpy(pr.b).cuda()
    x = torch.from_numpy(pr.x0.copy()).cuda()
    fi = L.assg_solve_forced_schedule(h, Ad, b, x, sk, L.assg_default_opts(record_trace=1, **opts))
    ft = L.assg_get_trace(h)
    xf = x.cpu().numpy()
    entry["forced"] = {"outcome": fi["outcome_name"], "outer": fi["outer_iters"],
                       "err_vs_oracle": float(np.linalg.norm(xf - xo) / np.linalg.norm(xo))}
    _log_fallback(entry)
    assert fi["outcome"] == L.CONVERGED, (case, fi)
    assert fi["outer_iters"] in (io["outer"], io["outer"] + 1), (case, fi)
    assert [t["sk"] for t in ft[:len(sk)]] == list(sk)
    assert entry["forced"]["err_vs_oracle"] <= 1e-8, entry


def _oracle_kw(opts):
    keys = ("s_max", "s_init", "growth", "tol", "basis", "max_outer", "max_iters", "variant",
            "c_const")
    return {k: v for k, v in opts.items() if k in keys}
