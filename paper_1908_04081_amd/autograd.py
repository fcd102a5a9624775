"""Differentiable solve x = A^{-1} b through the adaptive s-step CG.

Forward: one assg_solve.  Backward: the adjoint solve lambda = A^{-1} g for
the incoming gradient g = dL/dx (A is symmetric positive definite, so the
adjoint system has the same matrix and the same solver applies), then
dL/db = lambda and dL/dval_k = -lambda[row(k)] * x[col(k)] for every stored
entry, written by the library's pattern kernel.  Every stored value is its
own variable: for a symmetric perturbation of A (a_ij and a_ji together) the
directional derivative is the sum over both entries.

A solve that ends STAGNATED (the true residual stopped improving above the
tolerance: the attainable accuracy of the recurrence for that right-hand
side, which plain CG shares) still returns its iterate and emits a
SolveStagnated warning; DIVERGED, BREAKDOWN and MAX_ITER raise.  The outcome and residuals of the last forward
and adjoint solves are kept in ``last_info``.

PyTorch supplies the tensors and the autograd graph only; both solves and the
gradient scatter run in the HIP library.
"""
from __future__ import annotations

import warnings

import torch

from . import (CONVERGED, OUTCOME_NAMES, STAGNATED, DeviceCSR, Handle, assg_analyze,
               assg_create, assg_csr_outer_on_pattern, assg_default_opts, assg_solve)

last_info: dict = {}


class SolveError(RuntimeError):
    pass


class SolveStagnated(UserWarning):
    """A forward or adjoint solve stopped above its tolerance (STAGNATED)."""


def _accept(info, what, tol):
    last_info[what] = info
    if info["outcome"] not in (CONVERGED, STAGNATED):
        raise SolveError(f"{what} solve: {OUTCOME_NAMES.get(info['outcome'])}")
    if info["outcome"] == STAGNATED:
        warnings.warn(f"{what} solve stagnated at relative residual {info['relres_true']:.3e} "
                      f"above tol {tol:.1e}; its iterate is used", SolveStagnated, stacklevel=3)


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, val, b, pattern, handle, opts):
        A = DeviceCSR(pattern.row_ptr, pattern.col_idx, val.detach().contiguous(), pattern.n,
                      pattern.nnz)
        x = torch.zeros_like(b)
        _accept(assg_solve(handle, A, b.detach().contiguous(), x, opts), "forward", opts.tol)
        ctx.A, ctx.handle, ctx.opts = A, handle, opts
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        A, h = ctx.A, ctx.handle
        lam = torch.zeros_like(x)
        g = gx.detach().contiguous()
        if torch.count_nonzero(g).item() > 0:
            _accept(assg_solve(h, A, g, lam, ctx.opts), "adjoint", ctx.opts.tol)
        gval = None
        if ctx.needs_input_grad[0]:
            gval = torch.empty_like(A.val)
            assg_csr_outer_on_pattern(h, A, lam, x, -1.0, gval)
        gb = lam if ctx.needs_input_grad[1] else None
        return gval, gb, None, None, None


def solve(pattern: DeviceCSR, val: torch.Tensor, b: torch.Tensor, handle: Handle | None = None,
          **opts) -> torch.Tensor:
    """x = A^{-1} b with A = (pattern, val); differentiable in ``val`` and ``b``.
    ``pattern`` supplies row_ptr/col_idx (its own values are not used); options
    are those of assg_default_opts (e.g. tol=1e-12, s_max=10, basis=...)."""
    if handle is None:
        handle = assg_create()
        assg_analyze(handle, pattern)
    o = assg_default_opts(**opts)
    return _Solve.apply(val, b, pattern, handle, o)
