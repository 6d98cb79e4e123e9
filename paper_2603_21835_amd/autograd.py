"""torch.autograd binding of the grid density.

``gint_rho(plan, D, R)`` returns rho(r_g) (Sec. 3.3.1, rho(r_g) equation) for
density matrix D (device, norb x norb) and atom positions R (natom x 3); its
backward pass is the hand-written adjoint of the library:

  dL/dD_mu,nu = sum_g (dL/drho_g) phit_mu(r_g) phit_nu(r_g)   -> gint_build_H_weighted
  dL/dR_I     = sum_g (dL/drho_g) d rho_g / dR_I               -> gint_force_weighted

so that E = dV * (V * rho).sum() followed by E.backward() yields the grid
force of the F^{loc,Pulay} equation (as dE/dR).  Marshalling only: the
positions go to the plan as host doubles; all arithmetic runs in the
library's kernels.
"""
from __future__ import annotations

import torch


class GintRho(torch.autograd.Function):
    @staticmethod
    def forward(ctx, D, R, plan):
        pos = R.detach().to("cpu", torch.float64).contiguous().numpy()
        plan.set_positions(pos)
        rho = plan.build_rho(D.detach().contiguous())
        ctx.plan = plan
        ctx.pos = pos
        ctx.save_for_backward(D, R)
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        D, R = ctx.saved_tensors
        plan = ctx.plan
        plan.set_positions(ctx.pos)
        g = grad_rho.contiguous()
        grad_D = grad_R = None
        if ctx.needs_input_grad[0]:
            grad_D = plan.build_H(g, weighted=True)
        if ctx.needs_input_grad[1]:
            grad_R = plan.force(g, D.detach().contiguous(), weighted=True).to(R.device, R.dtype)
        return grad_D, grad_R, None


def gint_rho(plan, D, R):
    """rho on the mesh, differentiable in D and in the positions R."""
    return GintRho.apply(D, R, plan)
