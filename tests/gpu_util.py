"""Helpers shared by the GPU tests (no tests here)."""
import math

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


def oracle_outer_spread(pr, seeds=12, **kw):
    """Range of the oracle's outer-loop count when every basis entry it builds
    carries one extra relative rounding error (normal noise of size 2^-53,
    fixed seeds).  The GPU sums in another order than the host BLAS, so on a
    problem whose s-selection sits near a threshold this is the spread any
    correct implementation can land in."""
    import oracle.sstep as S
    base = S.sstep_basis
    outs = []
    try:
        for seed in range(seeds):
            rng = np.random.default_rng(seed)

            def noisy(*a, _rng=rng, **k):
                Y = base(*a, **k)
                return Y * (1.0 + 2.0 ** -53 * _rng.standard_normal(Y.shape))

            S.sstep_basis = noisy
            _, info = O.adaptive_sstep_cg(pr.A, pr.b, pr.x0, **kw)
            outs.append(info["outer"])
    finally:
        S.sstep_basis = base
    return min(outs), max(outs)
