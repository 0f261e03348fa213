"""torch.autograd binding of the exchange energy (argument marshalling only).

``exchange_energy(plan, C, V, D, precision)`` returns E_x per system (FP64 or
mixed forward); its backward calls the library's binary64 exchange_backward
kernels for dE/dC, dE/dV and dE/dD with each system's upstream gradient,
reusing the forward K for dE/dD and, after a binary64 forward whose workspace
no other call has overwritten, the forward's intermediates E and H'.
``spin_exchange_energy(plan, C, V, D)`` is the same for the collinear-spin
energy (two density matrices, binary64; the forward's E and H' likewise).
``exchange_forces(plan, C, V, D)`` returns -dE_x/dR for the synthetic
exp(-r/1.5) / exp(-r^2/8) position dependence of C and V.
"""
import torch

from ._lib import PREC_FP64


class _ExchangeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C, V, D, plan, precision):
        K = torch.empty(plan.info["d_size"], dtype=torch.float64, device=C.device)
        Ex = torch.empty(plan.n_systems, dtype=torch.float64, device=C.device)
        plan.build_K(C, V, D, K, Ex, precision=precision)
        ctx.save_for_backward(C, V, D, K)
        ctx.plan = plan
        # the workspace generation of this build: the backward takes its E and H' if no
        # other call has written the workspace since (binary64 builds only)
        ctx.build_id = plan.build_id() if precision == PREC_FP64 else None
        return Ex

    @staticmethod
    def backward(ctx, gEx):
        C, V, D, K = ctx.saved_tensors
        gE = gEx.detach().to(torch.float64).contiguous()   # one upstream gradient per system
        need = ctx.needs_input_grad
        dC = torch.empty_like(C) if need[0] else None
        dV = torch.empty_like(V) if need[1] else None
        dD = torch.empty_like(D) if need[2] else None
        if dC is not None or dV is not None or dD is not None:
            # binary64 gradient kernels; dE/dD = -K/2 reuses the forward K (of either precision)
            ctx.plan.exchange_backward(C, V, D, gE, dC=dC, dV=dV, dD=dD, K=K, build_id=ctx.build_id)
        return dC, dV, dD, None, None


class _SpinExchangeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, C, V, D, plan):
        K = torch.empty(2 * plan.info["d_size"], dtype=torch.float64, device=C.device)
        Ex = torch.empty(plan.n_systems, dtype=torch.float64, device=C.device)
        plan.build_K_spin(C, V, D, K, Ex)
        ctx.save_for_backward(C, V, D, K)
        ctx.plan = plan
        ctx.build_id = plan.build_id()
        return Ex

    @staticmethod
    def backward(ctx, gEx):
        C, V, D, K = ctx.saved_tensors
        gE = gEx.detach().to(torch.float64).contiguous()
        need = ctx.needs_input_grad
        dC = torch.empty_like(C) if need[0] else None
        dV = torch.empty_like(V) if need[1] else None
        dD = torch.empty_like(D) if need[2] else None
        if dC is not None or dV is not None or dD is not None:
            ctx.plan.exchange_backward_spin(C, V, D, gE, dC=dC, dV=dV, dD=dD, K=K, build_id=ctx.build_id)
        return dC, dV, dD, None


def spin_exchange_energy(plan, C, V, D):
    """Collinear-spin E_x = -1/2 sum_s <K^s, D^s> of every system (D: spin 0 then
    spin 1, 2 d_size), differentiable in C, V and both density matrices."""
    return _SpinExchangeEnergy.apply(C, V, D, plan)


def exchange_energy(plan, C, V, D, precision=PREC_FP64):
    """E_x of every system of the plan (differentiable in C, V and D)."""
    return _ExchangeEnergy.apply(C, V, D, plan, precision)


def exchange_forces(plan, C, V, D, c_decay=1.5, v_2s2=8.0, gE=1.0):
    """Atomic forces -d(gE E_x)/dR, shape (n_atoms, 3)."""
    F = torch.empty(plan.n_atoms * 3, dtype=torch.float64, device=C.device)
    plan.exchange_backward(C, V, D, gE, forces=F, c_decay=c_decay, v_2s2=v_2s2)
    return F.view(-1, 3)
