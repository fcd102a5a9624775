"""Ritz-value machinery of Section 4 (oracle; test infrastructure only).

* ``lanczos_tridiagonal``   -- T_i written in terms of the CG coefficients,
  equation (1.1).
* ``lanczos_cholesky_factor`` -- the upper bidiagonal L_i^T with
  zeta_j = alpha_j^{-1/2}, eta_j = (beta_j/alpha_j)^{1/2}, equation (4.1).
* ``MaxRitzEstimate``       -- Algorithm 3: incremental estimate of
  ||L_i||^2 = lambda_max(T_i), one 2x2 Rayleigh-Ritz step per CG iteration.
* ``MinRitzEstimate``       -- Algorithm 4: incremental estimate of
  ||L_i^{-1}||^2, whose inverse estimates lambda_min(T_i) (equation (4.2)).
* ``psi_update``            -- equation (4.5).
"""
from __future__ import annotations

import math

import numpy as np


def lanczos_tridiagonal(alphas, betas, i=None) -> np.ndarray:
    """T_i of equation (1.1): diagonal 1/alpha_0, 1/alpha_j + beta_{j-1}/alpha_{j-1};
    off-diagonal sqrt(beta_j)/alpha_j."""
    alphas = np.asarray(alphas, dtype=np.float64)
    betas = np.asarray(betas, dtype=np.float64)
    i = alphas.size if i is None else i
    T = np.zeros((i, i))
    for j in range(i):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < i:
            T[j, j + 1] = T[j + 1, j] = math.sqrt(betas[j]) / alphas[j]
    return T


def lanczos_cholesky_factor(alphas, betas, i=None) -> np.ndarray:
    """L_i^T of equation (4.1) (upper bidiagonal): zeta_j on the diagonal,
    eta_j on the superdiagonal."""
    alphas = np.asarray(alphas, dtype=np.float64)
    betas = np.asarray(betas, dtype=np.float64)
    i = alphas.size if i is None else i
    U = np.zeros((i, i))
    for j in range(i):
        U[j, j] = 1.0 / math.sqrt(alphas[j])
        if j + 1 < i:
            U[j, j + 1] = math.sqrt(betas[j] / alphas[j])
    return U


def _sign(v: float) -> float:
    # Reading: sign(0) is taken as +1 (the paper does not define it).
    return -1.0 if v < 0.0 else 1.0


class MaxRitzEstimate:
    """Algorithm 3 (incremental estimate of ||L_i||^2).

    Reading: the printed update a_l = eta_l^2 + xi_{l+1}^2 uses zeta_{l+1}
    (xi is the error/residual ratio of (4.4) and has no role here): a_l is
    then the new diagonal entry T_{l+1,l+1} of (1.1), and each step is exactly
    a 2x2 Rayleigh-Ritz problem on T.
    """

    def __init__(self, zeta0: float):
        self.omega = zeta0 * zeta0
        self.h = 1.0
        self.zeta = zeta0          # zeta_l of the last row added

    def step(self, eta: float, zeta_next: float) -> float:
        z, e = self.zeta, eta
        d = z * z * e * e * self.h
        a = e * e + zeta_next * zeta_next
        chi = math.sqrt((self.omega - a) ** 2 + 4.0 * d)
        if chi == 0.0:
            # Reading: degenerate 2x2 problem (omega == a and no coupling);
            # the estimate and the weight are left unchanged.
            h = 0.0
        else:
            h = 0.5 * (1.0 - (self.omega - a) / chi)
        self.omega = self.omega + chi * h
        self.h = h
        self.zeta = zeta_next
        return self.omega

    @property
    def value(self) -> float:
        return self.omega


class MinRitzEstimate:
    """Algorithm 4 (incremental estimate of ||L_i^{-1}||^2; its inverse
    estimates lambda_min(T_i)).

    Reading: the Ensure line's "||L_i||^{-2}" means ||L_i^{-1}||^{-2}
    (equation (4.2)).  Radicands are clamped at 0; a vanishing chi leaves the
    estimate unchanged (h = 0, g = 1); sign(0) = +1.
    """

    def __init__(self, zeta0: float):
        self.omega = 1.0 / (zeta0 * zeta0)
        self.a = self.omega
        self.d = 0.0
        self.g = 0.0
        self.h = 1.0

    def step(self, eta: float, zeta_next: float) -> float:
        d = -(eta / zeta_next) * (self.g * self.d + self.h * self.a)
        a = (eta * eta * self.a + 1.0) / (zeta_next * zeta_next)
        chi = math.sqrt((self.omega - a) ** 2 + 4.0 * d * d)
        if chi == 0.0:
            h = 0.0
        else:
            h = math.sqrt(max(0.0, 0.5 * (1.0 - (self.omega - a) / chi)))
        self.omega = self.omega + chi * h * h
        self.g = math.sqrt(max(0.0, 1.0 - h * h))
        self.h = abs(h) * _sign(d)
        self.d = d
        self.a = a
        return 1.0 / self.omega

    @property
    def value(self) -> float:
        return 1.0 / self.omega


def psi_update(psi: float, beta: float) -> float:
    """Equation (4.5): psi_{i+1} = psi_i / (psi_i + beta_i), psi_0 = 1
    (psi_i = ||r_i||^2 / ||p_i||^2)."""
    return psi / (psi + beta)
