"""Dense FP64 oracle: direct NEGF with elastic Buttiker dephasing, written out plainly.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Never called by the HIP library.

Notation follows the paper (Musland, Bergli, Flage-Larsen):
  G = G^r = (E - H - Sigma^r)^{-1}                                  Sec. II A, Eq. (7)
  Sigma^r = Sigma_L + Sigma_R + Sigma_s                             Sec. II A, Eq. (9)
  Gamma_p = i (Sigma_p - Sigma_p^dagger)                            Sec. II A, Eq. (11)
  A = i (G - G^dagger) = G Gamma G^dagger                           Sec. II A, Eqs. (5), (14)
  Buttiker: Sigma_s diagonal, sigma_i = -(i/2) gamma_i              Sec. II F, Eq. (67); Sec. III A, Eq. (77)
  G^< = G Sigma^< G^dagger                                          Sec. II A, Eq. (8)
  lead current i_q = -(i/h) Tr Gamma_q (G^< - i A f_q)              Sec. II A, Eq. (15)
  direct method: the diagonal of Eq. (8) with Buttiker Sigma^<_s     Sec. III C, Eq. (79)
  walker step 6': p_i ~ gamma_i |<i|psi>|^2, p_r ~ <psi|Gamma_r|psi> Sec. II F, Eqs. (75), (76)
  estimator X_pq = Tr Gamma_p A delta_rq                            Sec. II E, Eq. (66)
  midpoint energy quadrature                                        Sec. III C

Readings of the paper taken here (each one is listed in the design notes):
  * sites i = x*W + y (slice-major), H_ii = V_i, H_ij = -t between nearest neighbours, hard
    wall across the wire; leads are clean semi-infinite copies of the wire's cross-section
    coupled by -t to the first and last slice (lead_model 0), or the paper's wide-band model
    Sigma_p = -(i/2) Gamma_l P_p (lead_model 1, Sec. III A, Eq. (78));
  * the lead surface Green's function is taken at z = E + i*delta_lead; the device itself
    is at real E;
  * Eq. (79) is read as the diagonal of Eq. (8) with Sigma^<_{s,ii} = gamma_i n_i and
    -i G^<_{jj} = A_jj n_j, n_j being the probe occupation (linear response, f_L = 1, f_R = 0);
  * injection from lead p draws the eigen-channel of Gamma_p (steps 3-4, Eq. (39)) and then
    the first step 6' draw; the oracle forms this marginal channel by channel.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------------------------------
# Energy grid (Sec. III C: midpoint rule on a regular grid)
# ----------------------------------------------------------------------------------------
def midpoint_grid(emin: float, emax: float, n: int):
    """Midpoint nodes E_k = emin + (k + 1/2) dE and weights w_k = dE, dE = (emax - emin)/n."""
    dE = (emax - emin) / n
    E = np.array([emin + (k + 0.5) * dE for k in range(n)], dtype=np.float64)
    w = np.full(n, dE, dtype=np.float64)
    return E, w


# ----------------------------------------------------------------------------------------
# Hamiltonian (tight binding, nearest neighbours)
# ----------------------------------------------------------------------------------------
def site(x: int, y: int, W: int) -> int:
    return x * W + y


def hamiltonian(W: int, L: int, t: float, onsite) -> np.ndarray:
    """Dense real symmetric H of the W x L wire, slice-major site order, hard wall in y."""
    N = W * L
    H = np.zeros((N, N), dtype=np.float64)
    for x in range(L):
        for y in range(W):
            i = site(x, y, W)
            H[i, i] = onsite[i]
            if y + 1 < W:
                j = site(x, y + 1, W)
                H[i, j] = H[j, i] = -t
            if x + 1 < L:
                j = site(x + 1, y, W)
                H[i, j] = H[j, i] = -t
    return H


# ----------------------------------------------------------------------------------------
# Lead self-energies (Sec. II A, Eqs. (9)-(11); wide-band model Sec. III A, Eq. (78))
# ----------------------------------------------------------------------------------------
def transverse_modes(W: int, t: float):
    """Eigenmodes of the lead cross-section (an open chain of W sites, hopping -t).

    chi[:, m-1](y) = sqrt(2/(W+1)) sin(m pi y/(W+1)) for y, m = 1..W, eigenvalue
    eps_m = -2 t cos(m pi/(W+1)).
    """
    y = np.arange(1, W + 1)
    chi = np.zeros((W, W), dtype=np.float64)
    eps = np.zeros(W, dtype=np.float64)
    for m in range(1, W + 1):
        chi[:, m - 1] = np.sqrt(2.0 / (W + 1)) * np.sin(m * np.pi * y / (W + 1))
        eps[m - 1] = -2.0 * t * np.cos(m * np.pi / (W + 1))
    return chi, eps


def chain_surface_sigma(z: complex, eps: float, t: float) -> complex:
    """t^2 g_s for a semi-infinite chain with onsite eps and hopping -t, at complex z.

    g_s solves g = 1/(z - eps - t^2 g).  With w = (z - eps)/(2t) the retarded (decaying)
    root is t (w - sqrt(w-1) sqrt(w+1)) using principal square roots.
    """
    w = (z - eps) / (2.0 * t)
    return t * (w - np.sqrt(w - 1.0 + 0j) * np.sqrt(w + 1.0 + 0j))


def lead_self_energy(E: float, W: int, t: float, lead_model: int = 0,
                     delta_lead: float = 1e-10, gamma_l: float = 0.0) -> np.ndarray:
    """W x W retarded self-energy of one lead on its end slice of the wire."""
    if lead_model == 1:
        return -0.5j * gamma_l * np.eye(W, dtype=np.complex128)
    if lead_model != 0:
        raise ValueError("lead_model must be 0 or 1")
    z = E + 1j * delta_lead * t
    chi, eps = transverse_modes(W, t)
    S = np.zeros((W, W), dtype=np.complex128)
    for m in range(W):
        S += chain_surface_sigma(z, eps[m], t) * np.outer(chi[:, m], chi[:, m])
    return S


def broadening(S: np.ndarray) -> np.ndarray:
    """Gamma = i (Sigma - Sigma^dagger), Eq. (11)."""
    return 1j * (S - S.conj().T)


# ----------------------------------------------------------------------------------------
# Retarded Green's function, Eq. (7), dense
# ----------------------------------------------------------------------------------------
def slice_sites(x: int, W: int) -> slice:
    return slice(x * W, (x + 1) * W)


def inverse_green(E: float, H: np.ndarray, W: int, L: int, SL: np.ndarray, SR: np.ndarray,
                  gamma) -> np.ndarray:
    """E - H - Sigma_L - Sigma_R - Sigma_s with Sigma_s = diag(-(i/2) gamma_i), Eq. (77)."""
    N = W * L
    M = E * np.eye(N, dtype=np.complex128) - H.astype(np.complex128)
    M[slice_sites(0, W), slice_sites(0, W)] -= SL
    M[slice_sites(L - 1, W), slice_sites(L - 1, W)] -= SR
    M -= np.diag(-0.5j * np.asarray(gamma, dtype=np.float64))
    return M


def retarded_green(E, H, W, L, SL, SR, gamma) -> np.ndarray:
    """G^r = (E - H - Sigma^r)^{-1} by LAPACK (zgesv against the identity)."""
    M = inverse_green(E, H, W, L, SL, SR, gamma)
    return sla.solve(M, np.eye(M.shape[0], dtype=np.complex128))


# ----------------------------------------------------------------------------------------
# Per-energy solve: transmissions, probe system, lead current
# ----------------------------------------------------------------------------------------
class EnergySolution:
    """Everything the oracle knows at one energy (all FP64 / complex128)."""

    def __init__(self, E, W, L, t, onsite, gamma, lead_model=0, delta_lead=1e-10,
                 gamma_l=0.0, H=None):
        self.E, self.W, self.L, self.t = float(E), W, L, t
        self.N = W * L
        self.gamma = np.asarray(gamma, dtype=np.float64)
        H = hamiltonian(W, L, t, onsite) if H is None else H
        self.SL = lead_self_energy(E, W, t, lead_model, delta_lead, gamma_l)
        self.SR = lead_self_energy(E, W, t, lead_model, delta_lead, gamma_l)
        self.GamL = broadening(self.SL)
        self.GamR = broadening(self.SR)
        self.G = retarded_green(E, H, W, L, self.SL, self.SR, self.gamma)
        N = self.N
        s0, s1 = slice_sites(0, W), slice_sites(L - 1, W)
        # Full-size lead broadenings (zero outside the end slices).
        self.GL_full = np.zeros((N, N), dtype=np.complex128)
        self.GR_full = np.zeros((N, N), dtype=np.complex128)
        self.GL_full[s0, s0] = self.GamL
        self.GR_full[s1, s1] = self.GamR
        G = self.G
        Gd = G.conj().T
        self.A = 1j * (G - Gd)                                   # Eq. (5)
        self.Adiag = np.real(np.diag(self.A))
        # Terminal transmissions T_ab = Tr Gamma_a G Gamma_b G^dagger; the probes are
        # terminals with Gamma_j = gamma_j |j><j|.
        g = self.gamma
        self.P = np.abs(G) ** 2
        self.T_PP = g[:, None] * self.P * g[None, :]             # T_ij = gamma_i gamma_j |G_ij|^2
        self.T_PL = g * np.real(np.diag(G @ self.GL_full @ Gd))  # T_jL = gamma_j (G Gamma_L G^+)_jj
        self.T_PR = g * np.real(np.diag(G @ self.GR_full @ Gd))  # T_jR
        self.T_LP = g * np.real(np.diag(Gd @ self.GL_full @ G))  # T_Lj = gamma_j (G^+ Gamma_L G)_jj
        self.T_RP = g * np.real(np.diag(Gd @ self.GR_full @ G))  # T_Rj
        self.T_RL = float(np.real(np.trace(self.GR_full @ G @ self.GL_full @ Gd)))
        self.T_LR = float(np.real(np.trace(self.GL_full @ G @ self.GR_full @ Gd)))
        self.T_LL = float(np.real(np.trace(self.GL_full @ G @ self.GL_full @ Gd)))
        self.T_RR = float(np.real(np.trace(self.GR_full @ G @ self.GR_full @ Gd)))
        self.trGLA = float(np.real(np.trace(self.GL_full @ self.A)))  # Tr Gamma_L A
        self.trGRA = float(np.real(np.trace(self.GR_full @ self.A)))
        self._solve_probes()

    # Eq. (79) read as the diagonal of Eq. (8): with Sigma^< = i(Gamma_L f_L + Gamma_R f_R
    # + diag(gamma_i n_i)) and -i G^<_jj = A_jj n_j,
    #   A_jj n_j = (G Gamma_L G^+)_jj f_L + (G Gamma_R G^+)_jj f_R + sum_i |G_ji|^2 gamma_i n_i.
    def probe_occupations(self, fL: float, fR: float) -> np.ndarray:
        G, g = self.G, self.gamma
        Gd = G.conj().T
        src = (np.real(np.diag(G @ self.GL_full @ Gd)) * fL
               + np.real(np.diag(G @ self.GR_full @ Gd)) * fR)
        M = np.diag(self.Adiag) - self.P * g[None, :]
        return np.linalg.solve(M, src)

    def lesser_times_minus_i(self, fL: float, fR: float, n: np.ndarray) -> np.ndarray:
        """-i G^< = G (Gamma_L f_L + Gamma_R f_R + diag(gamma n)) G^dagger, from Eq. (8)."""
        G = self.G
        S = self.GL_full * fL + self.GR_full * fR + np.diag(self.gamma * n)
        return G @ S @ G.conj().T

    def lead_current(self, Gam_full, fq, mGl) -> float:
        """h i_q = -i Tr Gamma_q (G^< - i A f_q) = Tr Gamma_q (-i G^<) - f_q Tr Gamma_q A, Eq. (15)."""
        return float(np.real(np.trace(Gam_full @ mGl) - fq * np.trace(Gam_full @ self.A)))

    def _solve_probes(self):
        # Linear response around equilibrium: f_L = 1, f_R = 0 (Sec. II E, Eq. (62)).
        self.n = self.probe_occupations(1.0, 0.0)
        mGl = self.lesser_times_minus_i(1.0, 0.0, self.n)
        self.i_L = self.lead_current(self.GL_full, 1.0, mGl)
        self.i_R = self.lead_current(self.GR_full, 0.0, mGl)
        # Effective transmission L -> R: the current collected by lead R per unit f_L - f_R.
        self.T_eff = self.i_R
        # Net current into every probe (must vanish: the probes float).
        self.i_probe = (np.real(np.diag(mGl)) * self.gamma - self.gamma * self.Adiag * self.n)

    # ------------------------------------------------------------------------------------
    # The walker's transition kernel (Sec. II F, step 6'; injection by steps 3-4)
    # ------------------------------------------------------------------------------------
    def transition_kernel(self) -> np.ndarray:
        """(N+2) x (N+2) weights; row = current state, column = outcome.

        States 0..N-1 are probe sites, N is lead L, N+1 is lead R.  Row j (a walker at
        probe j): psi = G|j> (step 5, Eq. (40)); weight gamma_i |psi_i|^2 to probe i and
        <psi|Gamma_r|psi> to lead r (Eqs. (75), (76)).  Row N (injection from L): for each
        eigen-channel c of Gamma_L with eigenvalue lambda_c, psi_c = G|c> and the channel
        is drawn with probability lambda_c <c|A|c> / Tr Gamma_L A (Eq. (39)), so the
        marginal weight of outcome o is sum_c lambda_c * (step-6' weight of o from psi_c).
        Row N+1 is the same for lead R.
        """
        N, W, L = self.N, self.W, self.L
        G, g = self.G, self.gamma
        K = np.zeros((N + 2, N + 2), dtype=np.float64)

        def step6_weights(psi):
            out = np.zeros(N + 2, dtype=np.float64)
            out[:N] = g * np.abs(psi) ** 2
            out[N] = float(np.real(np.vdot(psi, self.GL_full @ psi)))
            out[N + 1] = float(np.real(np.vdot(psi, self.GR_full @ psi)))
            return out

        for j in range(N):
            K[j] = step6_weights(G[:, j])
        for row, Gam, x in ((N, self.GamL, 0), (N + 1, self.GamR, L - 1)):
            lam, vec = np.linalg.eigh(Gam)
            for c in range(W):
                if lam[c] <= 0.0:
                    continue
                ket = np.zeros(N, dtype=np.complex128)
                ket[slice_sites(x, W)] = vec[:, c]
                K[row] += lam[c] * step6_weights(G @ ket)
        return K


def absorption_probabilities(K: np.ndarray) -> np.ndarray:
    """Exact Markov-chain absorption probabilities of the walk defined by the rows of K.

    Rows are normalised to transition probabilities; columns N (lead L) and N+1 (lead R)
    absorb.  Returns h with h[s] = P(absorbed at R | current state s) for every row s,
    from the first-step equations h = Q h + r over the probe states (dense LAPACK solve).
    """
    n = K.shape[0]
    N = n - 2
    Pm = K / K.sum(axis=1, keepdims=True)
    Q = Pm[:N, :N]
    r = Pm[:N, N + 1]
    h_probe = np.linalg.solve(np.eye(N) - Q, r)
    h = np.zeros(n)
    h[:N] = h_probe
    h[N] = Pm[N, :N] @ h_probe + Pm[N, N + 1]
    h[N + 1] = Pm[N + 1, :N] @ h_probe + Pm[N + 1, N + 1]
    return h


# ----------------------------------------------------------------------------------------
# Whole workload
# ----------------------------------------------------------------------------------------
def solve_workload(W, L, t, onsite, gamma, energies, lead_model=0, delta_lead=1e-10,
                   gamma_l=0.0):
    H = hamiltonian(W, L, t, onsite)
    return [EnergySolution(E, W, L, t, onsite, gamma, lead_model, delta_lead, gamma_l, H=H)
            for E in energies]


def current(sols, weights) -> float:
    """I = sum_k w_k T_eff(E_k) in units of (e/h) per unit of f_L - f_R (Sec. III C)."""
    return float(sum(w * s.T_eff for s, w in zip(sols, weights)))


# ----------------------------------------------------------------------------------------
# Alias tables (Walker's method with Vose's two-stack construction), fixed-point format
# ----------------------------------------------------------------------------------------
TWO32 = 4294967296.0


def alias_vose(weights):
    """Alias table for the discrete distribution proportional to `weights`.

    Returns (thr, alias) with thr uint32 and alias int32: bucket c (drawn uniformly) keeps
    outcome c when a uniform 32-bit word r satisfies r < thr[c], else takes alias[c].
    A bucket whose kept mass is the whole bucket has thr = 2^32 - 1 and alias = c.
    Construction: scale to mean one; pair each small bucket with a large one, which gives
    up the small one's deficit (Vose, IEEE TSE 17 (1991)).
    """
    w = np.asarray(weights, dtype=np.float64)
    n = len(w)
    total = float(w.sum())
    q = w * n / total
    alias = np.arange(n, dtype=np.int32)
    prob = np.ones(n, dtype=np.float64)
    small = [i for i in range(n) if q[i] < 1.0]
    large = [i for i in range(n) if q[i] >= 1.0]
    while small and large:
        s = small.pop()
        l = large.pop()
        prob[s] = q[s]
        alias[s] = l
        q[l] = (q[l] + q[s]) - 1.0
        if q[l] < 1.0:
            small.append(l)
        else:
            large.append(l)
    for i in small + large:
        prob[i] = 1.0
        alias[i] = i
    thr = np.empty(n, dtype=np.uint32)
    for i in range(n):
        if prob[i] >= 1.0:
            thr[i] = 0xFFFFFFFF
            alias[i] = i
        else:
            thr[i] = np.uint32(int(prob[i] * TWO32))
    return thr, alias


def alias_distribution(thr, alias) -> np.ndarray:
    """The exact distribution an alias table (uint32 thresholds) samples."""
    n = len(thr)
    p = np.zeros(n, dtype=np.float64)
    for c in range(n):
        keep = float(thr[c]) / TWO32
        p[c] += keep / n
        p[int(alias[c])] += (1.0 - keep) / n
    return p
