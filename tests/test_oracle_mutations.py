"""Plant plausible mistakes in the oracle (CPU only) and check that at least
one pin fails for each: evidence that the pins constrain every part."""
import math

import numpy as np
import pytest

import oracle as O
import oracle.basis as OB
import oracle.ritz as OR
import oracle.sstep as OS
import pins


def _mut_alg3_wrong_zeta(mp):
    orig = OR.MaxRitzEstimate.step

    def step(self, eta, zeta_next):
        return orig(self, eta, self.zeta)          # a = eta^2 + zeta_l^2 instead of zeta_{l+1}
    mp.setattr(OR.MaxRitzEstimate, "step", step)


def _mut_alg4_sign(mp):
    orig = OR.MinRitzEstimate.step

    def step(self, eta, zeta_next):
        self.d = -self.d                              # coupling sign lost
        return orig(self, eta, zeta_next)
    mp.setattr(OR.MinRitzEstimate, "step", step)


def _mut_alg4_drop_one(mp):
    def step(self, eta, zeta_next):
        d = -(eta / zeta_next) * (self.g * self.d + self.h * self.a)
        a = (eta * eta * self.a) / (zeta_next * zeta_next)    # "+1" dropped
        chi = math.sqrt((self.omega - a) ** 2 + 4.0 * d * d)
        h = math.sqrt(max(0.0, 0.5 * (1.0 - (self.omega - a) / chi))) if chi else 0.0
        self.omega += chi * h * h
        self.g = math.sqrt(max(0.0, 1.0 - h * h)); self.h = abs(h) * (1 if d >= 0 else -1)
        self.d, self.a = d, a
        return 1.0 / self.omega
    mp.setattr(OR.MinRitzEstimate, "step", step)


def _mut_cheb_printed_mu(mp):
    def cheb(lmin, lmax, s):
        c, d = 0.5 * (lmin + lmax), lmax - lmin
        g = np.full(s, 0.5 * d); g[0] = d
        return np.full(s, c), g, np.full(max(s - 1, 0), 2.0 * d)
    mp.setattr(O, "params_chebyshev", cheb); mp.setattr(OB, "params_chebyshev", cheb)


def _mut_drop_mu_term(mp):
    def cols(A, v, nlev, theta, gamma, mu):
        out = np.empty((v.size, nlev + 1)); out[:, 0] = v
        for l in range(1, nlev + 1):
            out[:, l] = (A @ out[:, l - 1] - theta[l - 1] * out[:, l - 1]) / gamma[l - 1]
        return out
    mp.setattr(O, "polynomial_columns", cols); mp.setattr(OB, "polynomial_columns", cols)


def _mut_B_transposed(mp):
    orig = OB.change_of_basis
    f = lambda s, prm: orig(s, prm).T
    mp.setattr(O, "change_of_basis", f); mp.setattr(OB, "change_of_basis", f)
    mp.setattr(OS, "change_of_basis", f)


def _mut_sub_prefix(mp):
    f = lambda sbar, l: np.arange(2 * l + 1)
    mp.setattr(O, "sub_indices", f); mp.setattr(OB, "sub_indices", f); mp.setattr(OS, "sub_indices", f)


def _mut_psi_sign(mp):
    f = lambda psi, beta: psi / (psi - beta)
    mp.setattr(O, "psi_update", f); mp.setattr(OR, "psi_update", f); mp.setattr(OS, "psi_update", f)


def _mut_T_diag(mp):
    def T(alphas, betas, i=None):
        i = len(alphas) if i is None else i
        M = np.zeros((i, i))
        for j in range(i):
            M[j, j] = 1.0 / alphas[j]                  # beta_{j-1}/alpha_{j-1} dropped
            if j + 1 < i:
                M[j, j + 1] = M[j + 1, j] = math.sqrt(betas[j]) / alphas[j]
        return M
    mp.setattr(O, "lanczos_tridiagonal", T); mp.setattr(OR, "lanczos_tridiagonal", T)


def _mut_leja_tie_max(mp):
    orig = OB.leja_reference_points

    def f(count):
        t = orig(count).copy()
        if count > 3:
            t[3] = -t[3]                                # tie broken the other way
        return t
    mp.setattr(O, "leja_reference_points", f); mp.setattr(OB, "leja_reference_points", f)


def _mut_newton_swap(mp):
    orig = OB.params_newton

    def f(lmin, lmax, s):
        th, g, m = orig(lmin, lmax, s)
        th = th.copy(); th[0], th[1] = th[1], th[0]
        return th, g, m
    mp.setattr(O, "params_newton", f); mp.setattr(OB, "params_newton", f)


def _mut_alpha_without_B(mp):
    f = lambda s, prm: np.eye(2 * s + 1)
    mp.setattr(OS, "change_of_basis", f)


def _mut_hscg_beta(mp):
    orig = O.hscg

    def f(A, b, x0=None, tol=1e-10, max_iters=None, record=False, record_vectors=False):
        x, info = orig(A, b, x0, tol, max_iters, record, record_vectors)
        info["betas"] = [bb * 1.001 for bb in info["betas"]]
        return x, info
    mp.setattr(O, "hscg", f)


def _mut_source(mp, old, new):
    """Replaces a line of the oracle's s-step loop (for decision rules that
    are written inline rather than as functions of their own)."""
    import inspect
    src = inspect.getsource(OS)
    assert old in src
    ns = {"__name__": OS.__name__, "__package__": "oracle", "__file__": OS.__file__}
    exec(compile(src.replace(old, new), OS.__file__, "exec"), ns)
    mp.setattr(OS, "adaptive_sstep_cg", ns["adaptive_sstep_cg"])
    mp.setattr(O, "adaptive_sstep_cg", ns["adaptive_sstep_cg"])


def _mut_c_without_max(mp):
    _mut_source(mp, "c = max(1.0, lmax * math.sqrt(psi / lmin))",
                "c = lmax * math.sqrt(psi / lmin)")


def _mut_c_estimates_swapped(mp):
    _mut_source(mp, "c = max(1.0, lmax * math.sqrt(psi / lmin))",
                "c = max(1.0, lmin * math.sqrt(psi / lmax))")


def _mut_kappa_without_sqrt(mp):
    _mut_source(mp, "    return math.sqrt(hi / lo)", "    return hi / lo")


def _mut_absolute_residual_in_condy(mp):
    _mut_source(mp, "rho_m = math.sqrt(max(G[r_idx, r_idx], 0.0)) / nb",
                "rho_m = math.sqrt(max(G[r_idx, r_idx], 0.0))")


def _mut_absolute_phi(mp):
    _mut_source(mp, "phi = math.sqrt(rGr) / nb", "phi = math.sqrt(rGr)")


def _mut_ritz_start_at_one(mp):
    _mut_source(mp, "            if i == 0:\n                mt_max = MaxRitzEstimate(zeta)",
                "            if i <= 1:\n                mt_max = MaxRitzEstimate(zeta)")


def _mut_no_basis_update(mp):
    _mut_source(mp, "if improved and m > 1 and np.isfinite(lmax)",
                "if False and m > 1 and np.isfinite(lmax)")


def _mut_no_break(mp):
    _mut_source(mp, "if j < stilde - 1 and gam[j + 1] >= tol / (c * u * phi):   # (4.7)",
                "if False:")


def _mut_break_wrong_index(mp):
    _mut_source(mp, "if j < stilde - 1 and gam[j + 1] >= tol / (c * u * phi):   # (4.7)",
                "if j < stilde - 1 and kappa[j + 1] >= tol / (c * u * phi):")


def _mut_break_current_residual(mp):
    _mut_source(mp, "if j < stilde - 1 and gam[j + 1] >= tol / (c * u * phi):   # (4.7)",
                "if j < stilde - 1 and gam[j + 1] >= tol / (c * u * rho):")


def _mut_eps_double(mp):
    _mut_source(mp, "UNIT_ROUNDOFF = 2.0 ** -53", "UNIT_ROUNDOFF = 2.0 ** -52")


def _mut_stilde_largest_passing(mp):
    def f(kappa, thr):
        ok = [l for l in range(1, len(kappa) + 1) if kappa[l - 1] <= thr]
        return max(ok) if ok else 1
    mp.setattr(OS, "select_stilde", f)
    mp.setattr(O, "select_stilde", f)


MUTATIONS = {
    "alg3_wrong_zeta": _mut_alg3_wrong_zeta,
    "alg4_coupling_sign": _mut_alg4_sign,
    "alg4_drop_one": _mut_alg4_drop_one,
    "chebyshev_printed_mu": _mut_cheb_printed_mu,
    "basis_drop_mu_term": _mut_drop_mu_term,
    "B_transposed": _mut_B_transposed,
    "sub_indices_prefix": _mut_sub_prefix,
    "psi_sign": _mut_psi_sign,
    "T_diag_term": _mut_T_diag,
    "leja_tie_other_way": _mut_leja_tie_max,
    "newton_first_two_swapped": _mut_newton_swap,
    "alpha_without_B": _mut_alpha_without_B,
    "hscg_beta_scaled": _mut_hscg_beta,
    "c_without_max": _mut_c_without_max,
    "c_estimates_swapped": _mut_c_estimates_swapped,
    "kappa_without_sqrt": _mut_kappa_without_sqrt,
    "absolute_residual_in_condy": _mut_absolute_residual_in_condy,
    "absolute_phi_in_break": _mut_absolute_phi,
    "ritz_start_at_one": _mut_ritz_start_at_one,
    "no_basis_update": _mut_no_basis_update,
    "no_break": _mut_no_break,
    "break_index_kappa_j1": _mut_break_wrong_index,
    "stilde_largest_passing": _mut_stilde_largest_passing,
    "break_current_residual": _mut_break_current_residual,
    "eps_2_pow_52": _mut_eps_double,
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    MUTATIONS[name](monkeypatch)
    for pin in pins.ALL_PINS:
        try:
            pin()
        except (AssertionError, FloatingPointError, ValueError, ZeroDivisionError, KeyError,
                IndexError, np.linalg.LinAlgError):
            return                                  # caught by this pin
    pytest.fail(f"no pin caught mutation {name}")
