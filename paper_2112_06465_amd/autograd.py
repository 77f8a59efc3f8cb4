"""torch.autograd wrappers around the solve and its adjoint.

``helmholtz_solve(row_ptr, col_idx, vals, b)`` returns x = A^{-1} b
(zbicgstab_solve); its backward runs one adjoint solve (zbicgstab_adjoint)
and returns grad_b = lambda and grad_vals = -lambda_i conj(x_j), in torch's
real-pair convention for complex gradients.  ``helmholtz_solve_batched`` does
the same for B systems on one pattern (zbicgstab_solve_batched /
zbicgstab_adjoint_batched).  ``entry_map`` expresses matrix
entries as an affine function vals = vals0 + Phi beta of parameters beta
(Phi sparse, nnz x m, held as CSR together with Phi^H); its backward is
the rectangular SpMV Phi^H grad_vals (csr_zspmv_rect).  All arithmetic runs
in the library's kernels.
"""

from __future__ import annotations

from dataclasses import dataclass

import torch

from . import binding as B


@dataclass(frozen=True)
class SolveOptions:
    rtol: float = 1e-10
    maxiter: int = 20000
    jacobi: bool = True
    symmetric: bool = False  # caller asserts A = A^T (bitwise) for every vals passed

    @property
    def flags(self) -> int:
        return (B.PRECOND_JACOBI if self.jacobi else B.PRECOND_NONE) | (B.SYMMETRIC if self.symmetric else 0)


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, row_ptr, col_idx, opts: SolveOptions):
        x, info = B.zbicgstab_solve(row_ptr, col_idx, vals.detach(), b.detach().contiguous(), rtol=opts.rtol,
                                    maxiter=opts.maxiter, flags=opts.flags & B.PRECOND_JACOBI)
        if info["status"] != B.OK:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.save_for_backward(vals.detach(), x, row_ptr, col_idx)
        ctx.opts = opts
        ctx.info = info
        return x

    @staticmethod
    def backward(ctx, gx):
        vals, x, row_ptr, col_idx = ctx.saved_tensors
        opts = ctx.opts
        need_vals = ctx.needs_input_grad[0]
        grad_b, grad_vals, info = B.zbicgstab_adjoint(row_ptr, col_idx, vals, x, gx.to(torch.complex128).contiguous(),
                                                      rtol=opts.rtol, maxiter=opts.maxiter, flags=opts.flags,
                                                      want_grad_vals=need_vals)
        if info["status"] != B.OK:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        return grad_vals, (grad_b if ctx.needs_input_grad[1] else None), None, None, None


def helmholtz_solve(row_ptr, col_idx, vals, b, opts: SolveOptions | None = None):
    """Differentiable x = A^{-1} b on the GPU."""
    return HelmholtzSolve.apply(vals, b, row_ptr, col_idx, opts or SolveOptions())


class HelmholtzSolveBatched(torch.autograd.Function):
    """x[:, j] = A_j^{-1} b[:, j] for B systems on one pattern (vals (nnz, B), b (n, B))."""

    @staticmethod
    def forward(ctx, vals, b, row_ptr, col_idx, opts: SolveOptions):
        x, infos = B.zbicgstab_solve_batched(row_ptr, col_idx, vals.detach().contiguous(), b.detach().contiguous(),
                                             rtol=opts.rtol, maxiter=opts.maxiter, flags=opts.flags & B.PRECOND_JACOBI)
        bad = [i for i in infos if i["status"] != B.OK]
        if bad:
            raise RuntimeError(f"forward solve did not converge: {bad[0]}")
        ctx.save_for_backward(vals.detach().contiguous(), x, row_ptr, col_idx)
        ctx.opts = opts
        return x

    @staticmethod
    def backward(ctx, gx):
        vals, x, row_ptr, col_idx = ctx.saved_tensors
        opts = ctx.opts
        need_vals = ctx.needs_input_grad[0]
        grad_b, grad_vals, infos = B.zbicgstab_adjoint_batched(row_ptr, col_idx, vals, x,
                                                               gx.to(torch.complex128).contiguous(), rtol=opts.rtol,
                                                               maxiter=opts.maxiter, flags=opts.flags,
                                                               want_grad_vals=need_vals)
        bad = [i for i in infos if i["status"] != B.OK]
        if bad:
            raise RuntimeError(f"adjoint solve did not converge: {bad[0]}")
        return grad_vals, (grad_b if ctx.needs_input_grad[1] else None), None, None, None


def helmholtz_solve_batched(row_ptr, col_idx, vals, b, opts: SolveOptions | None = None):
    """Differentiable X = [A_j^{-1} b_j] for B systems sharing one pattern."""
    return HelmholtzSolveBatched.apply(vals, b, row_ptr, col_idx, opts or SolveOptions())


class EntryMap(torch.autograd.Function):
    @staticmethod
    def forward(ctx, beta, vals0, phi, phi_h):
        # phi = (row_ptr, col_idx, vals) of Phi (nnz x m); phi_h likewise for Phi^H (m x nnz)
        v = B.csr_zspmv_rect(*phi, beta.detach().contiguous())
        ctx.phi_h = phi_h
        return vals0 + v

    @staticmethod
    def backward(ctx, g):
        gb = B.csr_zspmv_rect(*ctx.phi_h, g.to(torch.complex128).contiguous())
        return gb, g, None, None


def entry_map(beta, vals0, phi, phi_h):
    """vals = vals0 + Phi beta, differentiable in beta and vals0."""
    return EntryMap.apply(beta, vals0, phi, phi_h)
