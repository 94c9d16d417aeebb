"""torch.autograd.Function wrappers over the hand-written adjoint kernels.

Gradients follow PyTorch's complex convention for a real loss, dL/dRe + i dL/dIm, so for
out = Op psi the backward is grad_psi = Op^dagger grad_out and grad_U is the link gradient of
Re <grad_out, Op psi> computed by grid_dhop_backward (HMC's fermion force, Section 4 of the
paper, is its su(3) projection; ``force=True`` returns that instead).
"""
from __future__ import annotations

import torch

from . import api


class DhopFn(torch.autograd.Function):
    """out = Op(U) psi with Op = H ("hop"), D ("wilson") or M ("dwf"); differentiable in U and psi."""

    @staticmethod
    def forward(ctx, U, psi, kind="hop", dag=False, mass=0.0, M5=1.8, mf=0.01):
        ctx.save_for_backward(U, psi)
        ctx.cfg = dict(kind=kind, dag=dag, mass=mass, M5=M5, mf=mf)
        return api.dhop(U, psi, **ctx.cfg)

    @staticmethod
    def backward(ctx, grad_out):
        U, psi = ctx.saved_tensors
        g = grad_out.contiguous()
        gp, gu = api.dhop_backward(U, psi, g, want_psi=ctx.needs_input_grad[1], want_U=ctx.needs_input_grad[0],
                                   **ctx.cfg)
        return gu, gp, None, None, None, None, None


class PseudofermionActionFn(torch.autograd.Function):
    """S = Re phi^dagger (Op^dagger Op)^-1 phi (Op = D, M or the Moebius M, FP64), differentiable in U and phi.

    The library computes S (a fixed-order FP64 reduction) and, in backward, dS/dU = -2 G(Op X, X)
    and dS/dphi = 2 X scaled by the upstream gradient (grid_pseudofermion_action); the solve X is
    recomputed there instead of being stored.
    """

    @staticmethod
    def forward(ctx, U, phi, kind="wilson", mass=0.1, M5=1.8, mf=0.01, tol=1e-12, sloppy="f64", b5=1.0, c5=0.0):
        ctx.save_for_backward(U, phi)
        ctx.cfg = dict(kind=kind, mass=mass, M5=M5, mf=mf, tol=tol, sloppy=sloppy, b5=b5, c5=c5)
        S, _, _, _, _ = api.pseudofermion_action(U, phi, **ctx.cfg)
        return torch.tensor(S, dtype=torch.float64, device=phi.device)

    @staticmethod
    def backward(ctx, gS):
        U, phi = ctx.saved_tensors
        want_U, want_phi = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_U or want_phi):
            return None, None, None, None, None, None, None, None, None, None
        _, _, gU, gphi, _ = api.pseudofermion_action(U, phi, grad_scale=float(gS), want_S=False, want_U=want_U,
                                                     want_phi=want_phi, **ctx.cfg)
        return gU, gphi, None, None, None, None, None, None, None, None
