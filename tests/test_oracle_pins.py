"""Pins of the dense oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something other than itself: closed forms, invariants
proved in the paper, a brute-force route, or a library routine.  A dropped term, a wrong sign
or index, or a transposed operand anywhere in oracle/dense.py fails at least one of them.
"""
import numpy as np
import pytest

from oracle import dense as D


def sol(W, L, E, eta, V=None, **kw):
    N = W * L
    V = np.zeros(N) if V is None else V
    g = np.full(N, eta) if np.isscalar(eta) else eta
    return D.EnergySolution(E, W, L, 1.0, V, g, **kw)


# ------------------------------------------------------------------ quadrature (Sec. III C)
def test_midpoint_grid_exact_error_on_quadratic():
    # Midpoint rule on x^2 over [a, b] with n cells errs by exactly -(b-a) h^2 f'' / 24, f'' = 2.
    a, b, n = -1.9, 1.9, 64
    E, w = D.midpoint_grid(a, b, n)
    h = (b - a) / n
    assert np.allclose(np.diff(E), h) and np.isclose(E[0], a + h / 2) and np.allclose(w, h)
    exact = (b ** 3 - a ** 3) / 3
    assert abs(np.sum(w * E ** 2) - (exact - (b - a) * h * h / 12)) < 1e-13


# ------------------------------------------------------------------ lead self-energy
def test_lead_sigma_chain_band_centre():
    # Semi-infinite chain at E = 0: Sigma = t^2 g_s = -i t, Gamma = 2t (textbook result).
    S = D.lead_self_energy(0.0, 1, 1.0, 0, 1e-10)
    assert abs(S[0, 0] - (-1j)) < 1e-9
    assert abs(D.broadening(S)[0, 0] - 2.0) < 1e-9


def test_lead_sigma_chain_outside_band_is_real_and_decaying():
    for E in (2.5, -3.0, 4.2):
        s = D.lead_self_energy(E, 1, 1.0, 0, 1e-10)[0, 0]
        w = E / 2
        ref = w - np.sign(w) * np.sqrt(w * w - 1)      # |t g_s| < 1 root
        assert abs(s.imag) < 1e-8 and abs(s.real - ref) < 1e-9 and abs(s) < 1


@pytest.mark.parametrize("W", [1, 3, 5])
def test_lead_sigma_matches_finite_lead_brute_force(W):
    # A finite lead of M slices at z = E + i*delta approaches the semi-infinite one as
    # exp(-M delta / v); with delta = 0.05 and M = 800 the difference is ~1e-12.
    delta, M = 0.05, 800
    for E in (-2.7, -0.4, 0.9, 3.3):
        S = D.lead_self_energy(E, W, 1.0, 0, delta)
        Hl = D.hamiltonian(W, M, 1.0, np.zeros(W * M))
        z = E + 1j * delta
        # surface slice = slice 0; Sigma = t^2 G_00 of the isolated lead
        G00 = np.linalg.inv(z * np.eye(W * M) - Hl)[:W, :W]
        assert np.abs(S - G00).max() < 1e-10


@pytest.mark.parametrize("W", [1, 4, 7])
def test_lead_sigma_dyson_fixed_point_and_retarded(W):
    # g_s = (z - H00 - t^2 g_s)^{-1} and -Im Sigma positive semidefinite (retarded branch).
    H00 = D.hamiltonian(W, 1, 1.0, np.zeros(W))
    for E in np.linspace(-3.9, 3.9, 17):
        S = D.lead_self_energy(E, W, 1.0, 0, 1e-10)
        z = E + 1e-10j
        resid = S - np.linalg.inv(z * np.eye(W) - H00 - S)
        assert np.abs(resid).max() < 1e-8 * max(1.0, np.abs(S).max())
        assert np.linalg.eigvalsh(D.broadening(S)).min() > -1e-12


def test_wide_band_lead():
    S = D.lead_self_energy(0.3, 4, 1.0, 1, gamma_l=0.2)
    assert np.allclose(S, -0.1j * np.eye(4)) and np.allclose(D.broadening(S), 0.2 * np.eye(4))


# ------------------------------------------------------------------ clean wire, eta = 0
@pytest.mark.parametrize("W", [1, 3, 5])
def test_clean_wire_integer_transmission(W):
    _, eps = D.transverse_modes(W, 1.0)
    for E in np.linspace(-3.7, 3.7, 13):
        s = sol(W, 6, E, 0.0)
        nopen = int(np.sum(np.abs(E - eps) < 2.0))
        assert abs(s.T_RL - nopen) < 1e-8
        assert abs(s.T_eff - nopen) < 1e-8
        # reflectionless: the L-row splits Tr Gamma_L A evenly between the leads
        assert abs(s.T_LL + s.T_RL - s.trGLA) < 1e-10


def test_chain_transmission_is_one_in_band():
    for E in np.linspace(-1.9, 1.9, 9):
        assert abs(sol(1, 50, E, 0.0).T_eff - 1.0) < 1e-8


# ------------------------------------------------------------------ closed forms with dephasing
@pytest.mark.parametrize("E,eps,GL,GR,gam", [(0.0, 0.0, 0.2, 0.2, 0.05), (0.3, -0.1, 0.4, 0.1, 0.3),
                                             (-0.7, 0.2, 1.0, 0.5, 0.0)])
def test_single_site_closed_form(E, eps, GL, GR, gam):
    # One site, wide-band leads on both sides (lead_model 1 puts Gamma_l on both, so use
    # GL = GR here) and one probe: T_eff = G_L G_R |G|^2 G_t / (G_L + G_R).
    GR = GL
    s = D.EnergySolution(E, 1, 1, 1.0, np.array([eps]), np.array([gam]), lead_model=1,
                         gamma_l=GL)
    Gt = GL + GR + gam
    G2 = 1.0 / ((E - eps) ** 2 + Gt * Gt / 4)
    assert abs(s.T_eff - GL * GR * G2 * Gt / (GL + GR)) < 1e-13
    assert abs(s.Adiag[0] - Gt * G2) < 1e-13


# ------------------------------------------------------------------ invariants from the paper
def disordered(W=3, L=7, E=0.4, eta=0.1, seed=1, **kw):
    V = np.random.default_rng(seed).uniform(-0.3, 0.3, W * L)
    return sol(W, L, E, eta, V, **kw)


@pytest.mark.parametrize("lead_model", [0, 1])
def test_current_conservation_leads_and_probes(lead_model):
    # Charge conservation (App. A, assumption (iv)): lead currents cancel, probes float.
    for E in (-2.1, 0.4, 1.3):
        s = disordered(E=E, lead_model=lead_model, gamma_l=0.5)
        assert abs(s.i_L + s.i_R) < 1e-12 * max(1, abs(s.i_R))
        assert np.abs(s.i_probe).max() < 1e-12
        assert s.T_eff > 0


def test_spectral_identity_and_row_sums():
    # A = G Gamma G^dagger (Eq. (14)) => every terminal's outgoing transmissions sum to
    # Tr Gamma_a A; for a probe, gamma_j A_jj.
    s = disordered(W=4, L=5, eta=0.07)
    G = s.G
    Gam = s.GL_full + s.GR_full + np.diag(s.gamma)
    assert np.abs(s.A - G @ Gam @ G.conj().T).max() < 1e-12
    g = s.gamma
    rows = s.T_PP.sum(axis=0) + s.T_LP + s.T_RP            # sum over receivers of T_{b j}
    assert np.abs(rows - g * s.Adiag).max() < 1e-12
    assert abs(s.T_PL.sum() + s.T_LL + s.T_RL - s.trGLA) < 1e-12
    K = s.transition_kernel()
    N = s.N
    assert np.abs(K[:N].sum(axis=1) - s.Adiag).max() < 1e-12
    assert abs(K[N].sum() - s.trGLA) < 1e-12 and abs(K[N + 1].sum() - s.trGRA) < 1e-12
    assert (K >= 0).all()


def test_reciprocity():
    s = disordered(W=3, L=6, eta=0.2)
    assert np.abs(s.T_PP - s.T_PP.T).max() < 1e-14
    assert np.abs(s.T_PL - s.T_LP).max() < 1e-13
    assert np.abs(s.T_PR - s.T_RP).max() < 1e-13
    assert abs(s.T_RL - s.T_LR) < 1e-13


def test_lead_row_channel_marginal_equals_trace_formula():
    # Injection (steps 3-4 then step 6'): summing over the eigen-channels of Gamma_L gives
    # gamma_i (G Gamma_L G^dagger)_ii to probe i and T_RL, T_LL to the leads.
    s = disordered(W=4, L=4, eta=0.15, seed=5)
    K = s.transition_kernel()
    N = s.N
    assert np.abs(K[N, :N] - s.T_PL).max() < 1e-13
    assert abs(K[N, N] - s.T_LL) < 1e-13 and abs(K[N, N + 1] - s.T_RL) < 1e-13
    assert np.abs(K[:N, :N] * s.gamma[:, None] - s.T_PP).max() < 1e-13


def neumann_T(s, q_full, p_full, nmax=2000):
    """sum_n Tr Gamma_q Xi^n A_p with Xi X = G diag(lambda_i X_ii) G^+, lambda_i = gamma_i/A_ii."""
    G = s.G
    Gd = G.conj().T
    lam = s.gamma / s.Adiag
    X = G @ p_full @ Gd
    tot = 0.0
    for _ in range(nmax):
        term = float(np.real(np.trace(q_full @ X)))
        tot += term
        if abs(term) < 1e-18:
            break
        X = G @ np.diag(lam * np.real(np.diag(X))) @ Gd
    return tot


def test_neumann_series_equals_probe_solve():
    # Sec. II E, Eq. (60): T_qp = sum_n Tr Gamma_q Xi^n A_p; the probe solve must agree.
    for E, eta in ((0.4, 0.2), (-1.1, 0.05)):
        s = disordered(W=2, L=5, E=E, eta=eta, seed=3)
        assert abs(neumann_T(s, s.GR_full, s.GL_full) - s.T_eff) < 1e-11


def test_appendix_b_spectral_expansion():
    # App. B, Eq. (B11): Tr A Gamma_q = sum_n sum_p Tr Gamma_q Xi^n A_p.
    s = disordered(W=2, L=4, eta=0.3, seed=7)
    rhs = neumann_T(s, s.GL_full, s.GL_full) + neumann_T(s, s.GL_full, s.GR_full)
    assert abs(rhs - s.trGLA) < 1e-11


def test_markov_absorption_equals_probe_solve():
    # E[X_LR] = Tr Gamma_L A * P(walker exits at R): the exact absorption probability of
    # the walk (a dense Markov-chain solve) times the lead-row total is T_eff.
    for seed in (1, 2):
        s = disordered(W=3, L=6, eta=0.08, seed=seed, E=0.9)
        K = s.transition_kernel()
        h = D.absorption_probabilities(K)
        N = s.N
        assert abs(K[N].sum() * h[N] - s.T_eff) < 1e-11
        assert abs(K[N + 1].sum() * (1 - h[N + 1]) - s.T_eff) < 1e-11   # reciprocity


def test_eta_to_zero_continuity():
    V = np.random.default_rng(4).uniform(-0.25, 0.25, 12)
    s0 = sol(3, 4, 0.5, 0.0, V)
    s1 = sol(3, 4, 0.5, 1e-7, V)
    assert abs(s1.T_eff - s0.T_RL) < 1e-5


def test_linear_in_length_resistance_strong_dephasing():
    # Sec. IV A: resistance grows linearly with length; the slope scales with the
    # dephasing rate (Sec. IV B: mean free path ~ 1/gamma).
    slopes = []
    for eta in (0.15, 0.3):
        Ls = np.array([20, 40, 80, 160])
        R = np.array([1.0 / sol(1, L, 0.3, eta).T_eff for L in Ls])
        p = np.polyfit(Ls, R, 1)
        assert np.abs(np.polyval(p, Ls) - R).max() / R.min() < 0.01
        slopes.append(p[0])
    assert abs(slopes[1] / slopes[0] - 2.0) < 0.3


def test_current_is_weighted_sum():
    E, w = D.midpoint_grid(-1.9, 1.9, 8)
    sols = D.solve_workload(1, 10, 1.0, np.zeros(10), np.full(10, 0.05), E)
    assert abs(D.current(sols, w) - sum(wk * s.T_eff for s, wk in zip(sols, w))) < 1e-15


# ------------------------------------------------------------------ alias tables
@pytest.mark.parametrize("n,seed", [(2, 0), (7, 1), (52, 2), (1002, 3)])
def test_alias_reconstructs_distribution(n, seed):
    rng = np.random.default_rng(seed)
    w = rng.exponential(size=n) * (rng.uniform(size=n) > 0.2)
    w[0] = 0.0
    w[-1] += 0.5
    thr, al = D.alias_vose(w)
    p = D.alias_distribution(thr, al)
    assert np.abs(p - w / w.sum()).max() <= 2.0 * n * 2.0 ** -32 / n + 1e-15
    assert p[0] == 0.0 or thr[0] == 0
