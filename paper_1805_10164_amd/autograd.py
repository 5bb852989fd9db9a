"""torch.autograd entries to the DIRECT and Monte Carlo currents and their gradients (HIP
library calls only).

`direct_current(system, onsite, gamma, energies, weights)` returns the current
I = sum_k w_k T_eff(E_k) (Sec. III C, the probe system of Eq. (8) solved per energy) as a
0-d float64 CUDA tensor that is differentiable in `onsite` (V_i = H_ii) and `gamma`
(Sigma_s,ii = -(i/2) gamma_i, Sec. III A, Eq. (77)).  The derivatives come from the
library's hand-written adjoint (mc_negf_grad), computed in the forward pass together with
I whenever either input requires a gradient, so the O(N^3) probe solve runs once; the
backward pass only scales them by the incoming gradient.  A scalar dephasing eta enters as
gamma = eta * ones(N), and autograd gives dI/deta = sum_i dI/dgamma_i.

`mc_current(system, onsite, gamma, energies, weights, n_walkers, seed)` is the Monte Carlo
current of Eq. (66) from n_walkers walks per energy, differentiable by the score function of
its walks (mc_negf_walk_counts + mc_negf_grad_mc): the gradient is itself an unbiased
estimate of dI/dV_i and dI/dgamma_i from the same walks.
"""
from __future__ import annotations

import torch

from . import mcnegf as M


class DirectCurrent(torch.autograd.Function):
    @staticmethod
    def forward(ctx, onsite, gamma, system, energies, weights, inject_lead):
        onsite = onsite.detach().contiguous()
        gamma = gamma.detach().contiguous()
        nE = int(energies.numel())
        # no alias tables: only the DIRECT current and its adjoint read this workspace
        sysd = M.System(system.W, system.L, system.t, system.lead_model, system.gamma_l,
                        system.delta_lead, system.flags | M.BUILD_NO_ALIAS)
        ws = M.allocate_workspace(sysd, nE, onsite.device)
        k = M.mc_negf_build_kernel(sysd, onsite, gamma, energies, ws)
        if ctx.needs_input_grad[0] or ctx.needs_input_grad[1]:
            gws = torch.empty(M.mc_negf_grad_workspace_bytes(k), dtype=torch.uint8,
                              device=onsite.device)
            dV = torch.empty_like(onsite)
            dg = torch.empty_like(gamma)
            _, I = M.mc_negf_grad(k, inject_lead, weights, gws, dV, dg)
            ctx.save_for_backward(dV, dg)
        else:
            T = torch.empty(nE, dtype=torch.float64, device=onsite.device)
            sg = torch.empty_like(T)
            _, I, _ = M.mc_negf_current(k, 1, inject_lead, None, weights, T, sg)
        return torch.tensor(I, dtype=torch.float64, device=onsite.device)

    @staticmethod
    def backward(ctx, grad_I):
        dV, dg = ctx.saved_tensors
        gV = grad_I * dV if ctx.needs_input_grad[0] else None
        gG = grad_I * dg if ctx.needs_input_grad[1] else None
        return gV, gG, None, None, None, None


def direct_current(system, onsite, gamma, energies, weights, inject_lead: int = 0):
    """I(onsite, gamma) with gradients through the library's adjoint (see the module doc)."""
    return DirectCurrent.apply(onsite, gamma, system, energies, weights, inject_lead)


class MonteCarloCurrent(torch.autograd.Function):
    @staticmethod
    def forward(ctx, onsite, gamma, system, energies, weights, n_walkers, seed, inject_lead):
        onsite = onsite.detach().contiguous()
        gamma = gamma.detach().contiguous()
        nE = int(energies.numel())
        dev = onsite.device
        sysm = M.System(system.W, system.L, system.t, system.lead_model, system.gamma_l,
                        system.delta_lead, system.flags | M.BUILD_NO_DIRECT)
        ws = M.allocate_workspace(sysm, nE, dev)
        k = M.mc_negf_build_kernel(sysm, onsite, gamma, energies, ws)
        tal = torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=dev)
        need = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        if need:
            cnt = torch.zeros(M.mc_negf_walk_counts_bytes(k) // 4, dtype=torch.int32,
                              device=dev)
            M.mc_negf_walk_counts(k, seed, 0, inject_lead, 0, n_walkers, 1_000_000, cnt, tal)
        else:
            M.mc_negf_walk(k, seed, 0, inject_lead, 0, n_walkers, 1_000_000, tal)
        T = torch.empty(nE, dtype=torch.float64, device=dev)
        sg = torch.empty_like(T)
        _, I, _ = M.mc_negf_current(k, 0, inject_lead, tal, weights, T, sg)
        if need:
            gws = torch.empty(M.mc_negf_grad_workspace_bytes(k), dtype=torch.uint8, device=dev)
            dV = torch.empty_like(onsite)
            dg = torch.empty_like(gamma)
            M.mc_negf_grad_mc(k, inject_lead, cnt, tal, weights, gws, dV, dg)
            ctx.save_for_backward(dV, dg)
        return torch.tensor(I, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, grad_I):
        dV, dg = ctx.saved_tensors
        gV = grad_I * dV if ctx.needs_input_grad[0] else None
        gG = grad_I * dg if ctx.needs_input_grad[1] else None
        return gV, gG, None, None, None, None, None, None


def mc_current(system, onsite, gamma, energies, weights, n_walkers: int, seed: int,
               inject_lead: int = 0):
    """Monte Carlo I(onsite, gamma) from n_walkers walks per energy, with score-function
    gradients (see the module doc)."""
    return MonteCarloCurrent.apply(onsite, gamma, system, energies, weights, n_walkers, seed,
                                   inject_lead)
