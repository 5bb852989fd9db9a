"""Gradient of the Monte Carlo transmission estimator by the score function (the derivative of
a reweighted path estimator).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Never called by the HIP library.

A walk injected at lead p scores X = c_p [exit at q] (Eq. (66)); its mean is T = c_p P(exit
at q).  Reweighting a walk drawn at parameters theta0 by its likelihood ratio
prod p_theta(s -> o) / p_theta0(s -> o) keeps the estimator unbiased at theta, so
    dT/dtheta = E[ X ( sum over the walk's steps of d log p(s -> o)/dtheta ) ] + E[X] dc_p/dtheta / c_p.
With C[o][s] the number of steps s -> o taken by the walks that reach q (out of N_w walks),
p(s -> o) = K_so / S_s (K the kernel weights of Eqs. (75), (76) and of the marginalised
injection rows, S_s the row totals: A_ss for a probe, c_p for the injection row), the
injection row's normaliser cancels the c_p term and
    estimate = (c_p / N_w) d/dtheta [ sum_so C_so K_so(theta) / K_so(theta0)
                                      - sum_{s probe} n_s A_ss(theta) / A_ss(theta0) ],
n_s = sum_o C_so, evaluated at theta0 (V_i = H_ii, gamma_i).  The oracle writes K, A and
c_p again in torch (complex128 on the CPU, dense G by a solve) and differentiates this
expression by reverse mode.

expected_counts() gives E[C] / N_w exactly (visits v_s, transition probabilities p_so and the
absorption probabilities h_o at q: E[C_so] / N_w = v_s p_so h_o); with it the estimate is the
exact derivative of T_eff (a pin of the formula, independent of sampling).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import dense as D
from . import walker as OW


def kernel_torch(W, L, t, V, gam, E, lead_model=0, delta_lead=1e-10, gamma_l=0.0):
    """(K [n][n] real torch tensor, A_jj [N], c_L, c_R) as functions of V, gamma (float64
    tensors), following dense.EnergySolution.transition_kernel: probe row j weighs outcome i
    by gamma_i |G_ij|^2 and lead r by <G_{:,j}|Gamma_r|G_{:,j}>; injection row r weighs probe
    i by gamma_i (G Gamma_r G^+)_ii and lead r' by Tr Gamma_r' G Gamma_r G^+."""
    N = W * L
    H0 = torch.from_numpy(D.hamiltonian(W, L, t, np.zeros(N))).to(torch.complex128)
    s0, s1 = D.slice_sites(0, W), D.slice_sites(L - 1, W)
    eye = torch.eye(N, dtype=torch.complex128)
    SL = torch.from_numpy(D.lead_self_energy(E, W, t, lead_model, delta_lead, gamma_l))
    Gam = 1j * (SL - SL.conj().T)
    GL = torch.zeros((N, N), dtype=torch.complex128)
    GR = torch.zeros((N, N), dtype=torch.complex128)
    GL[s0, s0] = Gam
    GR[s1, s1] = Gam  # identical leads
    Sig = torch.zeros((N, N), dtype=torch.complex128)
    Sig[s0, s0] += SL
    Sig[s1, s1] += SL
    A = E * eye - H0 - torch.diag(V.to(torch.complex128)) - Sig \
        + torch.diag((0.5j * gam).to(torch.complex128))
    G = torch.linalg.solve(A, eye)
    Gd = G.conj().T
    Adiag = torch.real(torch.diagonal(1j * (G - Gd)))
    n = N + 2
    K = torch.zeros((n, n), dtype=torch.float64)
    # probe rows: row j is psi = G[:, j]
    P = torch.abs(G) ** 2                                   # P[i, j] = |G_ij|^2
    K[:N, :N] = (P * gam[:, None]).T                        # K[j, i] = gamma_i |G_ij|^2
    K[:N, N] = torch.real(torch.diagonal(Gd @ GL @ G))      # <psi_j|Gamma_L|psi_j>
    K[:N, N + 1] = torch.real(torch.diagonal(Gd @ GR @ G))
    for row, Gp in ((N, GL), (N + 1, GR)):
        K[row, :N] = gam * torch.real(torch.diagonal(G @ Gp @ Gd))
        K[row, N] = torch.real(torch.trace(GL @ G @ Gp @ Gd))
        K[row, N + 1] = torch.real(torch.trace(GR @ G @ Gp @ Gd))
    cL = torch.real(torch.trace(GL @ (1j * (G - Gd))))
    cR = torch.real(torch.trace(GR @ (1j * (G - Gd))))
    return K, Adiag, cL, cR


def score_gradient(W, L, t, onsite, gamma, E, counts, n_walkers, inject_lead=0, lead_model=0,
                   delta_lead=1e-10, gamma_l=0.0):
    """(dT/dV [N], dT/dgamma [N]) estimated from the transition counts C[o][s] of the walks
    that reached q among n_walkers walks at energy E (see the module docstring).  Counts may
    be any non-negative reals (e.g. expected counts)."""
    N = W * L
    n = N + 2
    C = torch.as_tensor(np.asarray(counts, dtype=np.float64)).T   # C[s][o]
    with torch.no_grad():
        K0, A0, cL0, cR0 = kernel_torch(W, L, t, torch.tensor(np.asarray(onsite, float)),
                                        torch.tensor(np.asarray(gamma, float)), E, lead_model,
                                        delta_lead, gamma_l)
    lam = torch.where(C > 0, C / torch.where(K0 > 0, K0, torch.ones_like(K0)),
                      torch.zeros_like(C))
    mu = C[:N].sum(dim=1) / A0                                     # n_s / A_ss over probes
    V = torch.tensor(np.asarray(onsite, dtype=np.float64), requires_grad=True)
    g = torch.tensor(np.asarray(gamma, dtype=np.float64), requires_grad=True)
    K, A, _, _ = kernel_torch(W, L, t, V, g, E, lead_model, delta_lead, gamma_l)
    F = (lam * K).sum() - (mu * A).sum()
    F.backward()
    c = float(cL0 if inject_lead == 0 else cR0)
    scale = c / float(n_walkers)
    return scale * V.grad.numpy().copy(), scale * g.grad.numpy().copy()


def expected_counts(K, inject_lead=0):
    """E[C[o][s]] per walker for the walks that reach q, from the rows of K: the expected
    number of visits v_s (1 for the injection row; v = r + Q^T v over the probes), the
    transition probabilities p_so and the probability h_o of reaching q from outcome o."""
    K = np.asarray(K, dtype=np.float64)
    n = K.shape[0]
    N = n - 2
    p_row = N + inject_lead
    q = N + 1 - inject_lead
    P = K / K.sum(axis=1, keepdims=True)
    Q = P[:N, :N]
    hR = D.absorption_probabilities(K)          # P(exit at R | state)
    h = hR if q == N + 1 else 1.0 - hR
    h = h.copy()
    h[q] = 1.0
    h[N + inject_lead] = 0.0                    # lead p absorbs without reaching q
    v = np.zeros(n)
    v[p_row] = 1.0
    v[:N] = np.linalg.solve(np.eye(N) - Q.T, P[p_row, :N])
    Ecount = np.zeros((n, n))                   # [o][s]
    for s in list(range(N)) + [p_row]:
        for o in list(range(N)) + [q]:
            Ecount[o, s] = v[s] * P[s, o] * h[o]
    return Ecount


def walk_counts_cdf(K, seed, realization, inject_lead, walker_begin, n_walkers,
                    max_steps=1_000_000):
    """(tallies [nE][5], counts [nE][n][n] int64) of the C walker with the paper's sampler."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    if K.ndim == 2:
        K = K[None]
    nE, n, _ = K.shape
    tal = np.zeros((nE, 5), dtype=np.int64)
    cnt = np.zeros((nE, n, n), dtype=np.int64)
    f = OW.lib().oracle_walk_counts_cdf
    vp, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    f.argtypes = [vp, i32, i32, u64, u32, u32, u64, u64, u32, vp, vp]
    f.restype = ctypes.c_int
    if f(K.ctypes.data, nE, n, seed, realization, inject_lead, walker_begin, n_walkers,
         max_steps, tal.ctypes.data, cnt.ctypes.data) != 0:
        raise ValueError("oracle_walk_counts_cdf rejected its arguments")
    return tal, cnt


def walk_counts_alias(thr, alias, seed, realization, inject_lead, walker_begin, n_walkers,
                      max_steps=1_000_000):
    """(tallies, counts) of the C walker on alias tables thr/alias [nE][n][pitch]."""
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    alias = np.ascontiguousarray(alias, dtype=np.int32)
    if thr.ndim == 2:
        thr, alias = thr[None], alias[None]
    nE, n, pitch = thr.shape
    tal = np.zeros((nE, 5), dtype=np.int64)
    cnt = np.zeros((nE, n, n), dtype=np.int64)
    f = OW.lib().oracle_walk_counts_alias
    vp, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    f.argtypes = [vp, vp, ctypes.c_int64, i32, i32, u64, u32, u32, u64, u64, u32, vp, vp]
    f.restype = ctypes.c_int
    if f(thr.ctypes.data, alias.ctypes.data, pitch, nE, n, seed, realization, inject_lead,
         walker_begin, n_walkers, max_steps, tal.ctypes.data, cnt.ctypes.data) != 0:
        raise ValueError("oracle_walk_counts_alias rejected its arguments")
    return tal, cnt
