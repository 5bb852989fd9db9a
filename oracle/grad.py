"""Derivatives of the DIRECT current with respect to the onsite potentials and the dephasing rates.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Never called by the HIP library.

The current is I = sum_k w_k T_eff(E_k) (Sec. III C) with T_eff the current collected by lead
R per unit f_L - f_R when the Buttiker probes float (Sec. II A, Eqs. (8), (15); Sec. III C,
Eq. (79), read as the diagonal of Eq. (8), as in dense.py).  Two independent evaluations of
dI/dV_i (V_i = H_ii) and dI/dgamma_i (Sigma_s,ii = -(i/2) gamma_i):

  adjoint()   reverse-mode differentiation (torch autograd on the CPU, float64/complex128) of
              a plain dense evaluation of T_eff written again in torch: G = (E - H - Sigma)^{-1}
              by a dense solve, the probe occupations from the diagonal of Eq. (8), the lead
              current of Eq. (15) (dense.py supplies only H and the lead self-energies).  The
              tests pin it to
  central_differences()  of dense.py's current (the plain definition), and to the closed
              form of a single site between wide-band leads.
"""
from __future__ import annotations

import numpy as np
import torch

from . import dense as D


def _current_torch(W, L, t, V, gam, energies, weights, lead_model, delta_lead, gamma_l):
    """I(V, gamma) as a torch scalar (V, gam: float64 tensors with requires_grad)."""
    N = W * L
    H0 = torch.from_numpy(D.hamiltonian(W, L, t, np.zeros(N))).to(torch.complex128)
    s0, s1 = D.slice_sites(0, W), D.slice_sites(L - 1, W)
    eye = torch.eye(N, dtype=torch.complex128)
    total = torch.zeros((), dtype=torch.float64)
    for E, w in zip(energies, weights):
        SL = torch.from_numpy(D.lead_self_energy(E, W, t, lead_model, delta_lead, gamma_l))
        GamL = 1j * (SL - SL.conj().T)
        GamL_full = torch.zeros((N, N), dtype=torch.complex128)
        GamR_full = torch.zeros((N, N), dtype=torch.complex128)
        GamL_full[s0, s0] = GamL
        GamR_full[s1, s1] = GamL  # identical leads
        Sig = torch.zeros((N, N), dtype=torch.complex128)
        Sig[s0, s0] += SL
        Sig[s1, s1] += SL  # both leads on one slice when L = 1
        A = E * eye - H0 - torch.diag(V.to(torch.complex128)) - Sig \
            + torch.diag((0.5j * gam).to(torch.complex128))
        G = torch.linalg.solve(A, eye)
        Gd = G.conj().T
        Adiag = torch.real(torch.diagonal(1j * (G - Gd)))
        P = torch.abs(G) ** 2
        wL = torch.real(torch.diagonal(G @ GamL_full @ Gd))
        # diagonal of Eq. (8) with f_L = 1, f_R = 0: A_jj n_j - sum_i |G_ji|^2 gamma_i n_i = wL_j
        Mp = torch.diag(Adiag) - P * gam[None, :]
        n = torch.linalg.solve(Mp, wL)
        # lead current collected by R, Eq. (15) with f_R = 0: Tr Gamma_R (-i G^<)
        S = GamL_full + torch.diag((gam * n).to(torch.complex128))
        T = torch.real(torch.trace(GamR_full @ G @ S @ Gd))
        total = total + w * T
    return total


def adjoint(W, L, t, onsite, gamma, energies, weights, lead_model=0, delta_lead=1e-10,
            gamma_l=0.0):
    """(I, dI/dV [N], dI/dgamma [N]) by reverse-mode differentiation of the dense current."""
    V = torch.tensor(np.asarray(onsite, dtype=np.float64), requires_grad=True)
    g = torch.tensor(np.asarray(gamma, dtype=np.float64), requires_grad=True)
    I = _current_torch(W, L, t, V, g, energies, weights, lead_model, delta_lead, gamma_l)
    I.backward()
    return float(I.detach()), V.grad.numpy().copy(), g.grad.numpy().copy()


def central_differences(W, L, t, onsite, gamma, energies, weights, h=1e-6, lead_model=0,
                        delta_lead=1e-10, gamma_l=0.0, which="V", sites=None):
    """dI/dV_i (which = "V") or dI/dgamma_i ("gamma") by (I(x + h) - I(x - h)) / 2h of the
    plain definition (dense.solve_workload / dense.current), for the listed sites."""
    onsite = np.asarray(onsite, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    N = W * L
    sites = range(N) if sites is None else sites
    out = []
    for i in sites:
        vals = []
        for sgn in (1.0, -1.0):
            V, g = onsite.copy(), gamma.copy()
            if which == "V":
                V[i] += sgn * h
            else:
                g[i] += sgn * h
            sols = D.solve_workload(W, L, t, V, g, energies, lead_model, delta_lead, gamma_l)
            vals.append(D.current(sols, weights))
        out.append((vals[0] - vals[1]) / (2.0 * h))
    return np.array(out)
