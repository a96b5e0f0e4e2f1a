"""torch.autograd.Function around the hand-written adjoint of the mechanical
equilibrium: J(E) for a per-voxel Young's modulus field E, with the gradient
from fgcg_mech_adjoint (forward strain recomputed in backward, no CG history
kept).  Objectives: "energy" (total elastic energy W) and "C11" (effective
<sigma_11>/eps_11 under the applied macro strain)."""
import torch

from . import fgcg

_OBJ = {"energy": fgcg.J_ENERGY, "C11": fgcg.J_C11}


class MechObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E_field, context, nu, eps_mac, objective, tol, maxit):
        # the objective as the library evaluates it (forward solve only)
        _, J, _, _ = context.mech_adjoint(E_field.detach().contiguous(), nu, eps_mac, objective=_OBJ[objective],
                                          tol=tol, maxit=maxit, want_grad=False)
        ctx.save_for_backward(E_field)
        ctx.args = (context, nu, tuple(eps_mac), objective, tol, maxit)
        return torch.tensor(J, dtype=torch.float64, device=E_field.device)

    @staticmethod
    def backward(ctx, grad_out):
        (E_field,) = ctx.saved_tensors
        context, nu, eps_mac, objective, tol, maxit = ctx.args
        g, _, _, _ = context.mech_adjoint(E_field.detach().contiguous(), nu, eps_mac, objective=_OBJ[objective],
                                          tol=tol, maxit=maxit)
        return grad_out * g, None, None, None, None, None, None


def mech_objective(E_field, context, nu, eps_mac, objective="energy", tol=1e-12, maxit=50000):
    return MechObjective.apply(E_field, context, nu, eps_mac, objective, tol, maxit)
