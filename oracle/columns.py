"""Single columns of G^r and single rows of the walker's kernel, by a sparse LU, for systems
too large for the dense oracle (N in the thousands to 16 000).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Never called by the HIP library.

The definitions are those of dense.py:
  G^r = (E - H - Sigma^r)^{-1}                                    Sec. II A, Eq. (7)
  Sigma^r = Sigma_L + Sigma_R + Sigma_s, Sigma_s,ii = -(i/2) gamma_i    Eq. (9); Sec. III A, Eq. (77)
  walker step 6' from psi = G|j>: weight gamma_i |psi_i|^2 to probe i and <psi|Gamma_r|psi>
  to lead r                                                       Sec. II F, Eqs. (75), (76)
  injection from lead p: eigen-channel c of Gamma_p drawn with weight lambda_c <c|A|c>,
  then the step-6' weights of psi = G|c>                          Sec. II D, Eq. (39)
E - H - Sigma^r is sparse (five nonzeros per row and the two W x W lead blocks); column j of
G^r solves (E - H - Sigma^r) x = e_j, here with SuperLU (scipy.sparse.linalg.splu) instead of
the dense oracle's LAPACK solve against the identity.  Pinned to dense.py on small systems.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import dense as D


def inverse_green_sparse(E: float, W: int, L: int, t: float, onsite, gamma, SL, SR):
    """E - H - Sigma_L - Sigma_R - Sigma_s as a sparse complex matrix (CSC)."""
    N = W * L
    onsite = np.asarray(onsite, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    rows, cols, vals = [], [], []
    for x in range(L):
        for y in range(W):
            i = D.site(x, y, W)
            # diagonal: E - V_i - (-(i/2) gamma_i)
            rows.append(i)
            cols.append(i)
            vals.append(E - onsite[i] + 0.5j * gamma[i])
            # -H_ij = +t between nearest neighbours (across the slice and along the wire)
            for j in ([D.site(x, y + 1, W)] if y + 1 < W else []) + \
                     ([D.site(x + 1, y, W)] if x + 1 < L else []):
                rows += [i, j]
                cols += [j, i]
                vals += [t, t]
    for x, S in ((0, SL), (L - 1, SR)):
        for a in range(W):
            for b in range(W):
                rows.append(D.site(x, a, W))
                cols.append(D.site(x, b, W))
                vals.append(-S[a, b])
    return sp.csc_matrix((np.array(vals, dtype=np.complex128), (rows, cols)), shape=(N, N))


class SparseEnergy:
    """G^r at one energy through a sparse LU of E - H - Sigma^r (columns on demand)."""

    def __init__(self, E, W, L, t, onsite, gamma, lead_model=0, delta_lead=1e-10, gamma_l=0.0):
        self.E, self.W, self.L, self.t = float(E), W, L, t
        self.N = W * L
        self.gamma = np.asarray(gamma, dtype=np.float64)
        self.SL = D.lead_self_energy(E, W, t, lead_model, delta_lead, gamma_l)
        self.SR = D.lead_self_energy(E, W, t, lead_model, delta_lead, gamma_l)
        self.GamL = D.broadening(self.SL)
        self.GamR = D.broadening(self.SR)
        self.lu = spla.splu(inverse_green_sparse(self.E, W, L, t, onsite, self.gamma,
                                                 self.SL, self.SR))

    def solve(self, rhs) -> np.ndarray:
        return self.lu.solve(np.asarray(rhs, dtype=np.complex128))

    def columns(self, cols) -> np.ndarray:
        """[N][len(cols)] columns of G^r."""
        B = np.zeros((self.N, len(cols)), dtype=np.complex128)
        for c, j in enumerate(cols):
            B[j, c] = 1.0
        return self.solve(B)

    def step6_weights(self, psi) -> np.ndarray:
        """Weights of the N + 2 outcomes from psi: probes, then lead L, lead R."""
        N, W, L = self.N, self.W, self.L
        out = np.zeros(N + 2, dtype=np.float64)
        out[:N] = self.gamma * np.abs(psi) ** 2
        pL = psi[D.slice_sites(0, W)]
        pR = psi[D.slice_sites(L - 1, W)]
        out[N] = float(np.real(np.vdot(pL, self.GamL @ pL)))
        out[N + 1] = float(np.real(np.vdot(pR, self.GamR @ pR)))
        return out

    def kernel_row(self, r: int) -> np.ndarray:
        """Row r of the (N+2) x (N+2) transition kernel (probe r < N, lead L = N, lead R)."""
        N, W, L = self.N, self.W, self.L
        if r < N:
            return self.step6_weights(self.columns([r])[:, 0])
        Gam, x = (self.GamL, 0) if r == N else (self.GamR, L - 1)
        lam, vec = np.linalg.eigh(Gam)
        row = np.zeros(N + 2, dtype=np.float64)
        for c in range(W):
            if lam[c] <= 0.0:
                continue
            ket = np.zeros(N, dtype=np.complex128)
            ket[D.slice_sites(x, W)] = vec[:, c]
            row += lam[c] * self.step6_weights(self.solve(ket))
        return row

    def effective_transmission(self) -> float:
        """T_eff = T_RL + sum_j T_Rj f_j with (diag(gamma_j A_jj) - T_PP) f = T_PL: the
        probe-conservation system in transmission form (Sec. III C, Eq. (79), with
        T_ab = Tr Gamma_a G Gamma_b G^+ and Gamma_j = gamma_j |j><j|), from all N columns
        of G.  Needs gamma_i > 0 on every site."""
        N, W, L = self.N, self.W, self.L
        g = self.gamma
        if not (g > 0.0).all():
            raise ValueError("effective_transmission needs gamma_i > 0 on every site")
        G = self.columns(list(range(N)))
        s0, s1 = D.slice_sites(0, W), D.slice_sites(L - 1, W)
        A = -2.0 * np.imag(np.diag(G))
        P = np.abs(G) ** 2
        Gc0 = G[:, s0]                                   # columns of slice 0
        T_PL = g * np.real(np.einsum("ja,ab,jb->j", Gc0, self.GamL, Gc0.conj()))
        Gr1 = G[s1, :]                                   # rows of the last slice
        T_RP = g * np.real(np.einsum("aj,ab,bj->j", Gr1.conj(), self.GamR, Gr1))
        G10 = G[s1, s0]
        T_RL = float(np.real(np.trace(self.GamR @ G10 @ self.GamL @ G10.conj().T)))
        M = np.diag(g * A) - g[:, None] * P * g[None, :]
        f = np.linalg.solve(M, T_PL)
        return T_RL + float(T_RP @ f)
