"""Pins of the oracle's energy-sampled walks and their constant estimator (CPU).

A walker draws its energy index k with probability w_k / W (W = sum of the weights) and
then walks at that energy; the variable X = W c_p(E_k) for an exit at the collecting lead
(0 otherwise) has mean sum_k w_k T_eff(E_k) (Eq. (66) with the energy density proportional
to the weights; with w_k = Th(E_k) dE this is the paper's constant estimator of Sec. II G).
"""
import numpy as np
from scipy import stats

from oracle import dense as D
from oracle import walker as OW


def system(W, L, eta, E, disorder=0.0, seed=3):
    V = np.random.default_rng(seed).uniform(-disorder, disorder, W * L) if disorder else np.zeros(W * L)
    g = np.full(W * L, eta)
    sols = D.solve_workload(W, L, 1.0, V, g, E)
    K = np.stack([s.transition_kernel() for s in sols])
    n = K.shape[1]
    c = K[:, n - 2, :].sum(axis=1)  # total weight of the injection row of lead L
    return sols, K, c


def thermal_weights(E, mu, kT):
    """Th(E) dE on a midpoint grid: -df/dE = 1 / (4 kT cosh^2((E - mu) / 2kT))."""
    dE = E[1] - E[0]
    return dE / (4.0 * kT * np.cosh((E - mu) / (2.0 * kT)) ** 2)


def test_energy_draws_follow_the_weights():
    E = np.linspace(-1.0, 1.0, 6)
    sols, K, c = system(2, 3, 0.1, E)
    w = np.array([0.5, 0.0, 1.5, 0.25, 0.0, 2.0])
    N = 200_000
    t = OW.walk_sampled_cdf(K, w, 17, 0, 0, 0, N)
    counts = t[:, :3].sum(axis=1)
    assert counts.sum() == N
    assert counts[1] == 0 and counts[4] == 0  # zero weight: never drawn
    p = w / w.sum()
    nz = p > 0
    chi2 = float((((counts[nz] - N * p[nz]) ** 2) / (N * p[nz])).sum())
    assert stats.chi2.sf(chi2, int(nz.sum()) - 1) > 1e-3


def test_clean_chain_constant_estimator_closed_form():
    # eta = 0 chain, energies in the band: T = 1, c_L = Tr Gamma_L A = 2 and half of the
    # walkers exit at R, so X is 0 or 2W with probability 1/2 each: I -> W, sigma_I -> W/sqrt(N).
    E = np.linspace(-1.5, 1.5, 5)
    sols, K, c = system(1, 12, 0.0, E)
    assert np.allclose(c, 2.0, atol=1e-9)
    w = thermal_weights(E, 0.2, 0.5)
    W = w.sum()
    N = 100_000
    t = OW.walk_sampled_cdf(K, w, 5, 0, 0, 0, N)
    I, s = OW.sampled_current(t, c, w)
    assert abs(I - W) < 4.0 * s
    assert abs(s / (W / np.sqrt(N)) - 1.0) < 0.02


def test_sampled_estimator_is_unbiased_with_dephasing():
    # mean within 3 sigma of the exact current with the same weights (thermal window)
    E = (np.arange(24) + 0.5) / 24 * 5.0 - 2.5
    sols, K, c = system(3, 6, 0.08, E, disorder=0.3)
    w = thermal_weights(E, 0.4, 0.3)
    exact = D.current(sols, w)
    t = OW.walk_sampled_cdf(K, w, 23, 0, 0, 0, 300_000)
    I, s = OW.sampled_current(t, c, w)
    assert abs(I - exact) < 3.0 * s, (I, exact, s)
    # the stratified estimator of the same walks per energy is a different, also unbiased one
    assert s > 0.0


def test_sampled_split_ranges_add_up():
    E = np.linspace(-1.0, 1.0, 4)
    sols, K, c = system(2, 2, 0.2, E)
    w = np.array([1.0, 2.0, 0.5, 1.0])
    a = OW.walk_sampled_cdf(K, w, 9, 1, 0, 0, 3000)
    b = OW.walk_sampled_cdf(K, w, 9, 1, 0, 0, 1234)
    OW.walk_sampled_cdf(K, w, 9, 1, 0, 1234, 3000 - 1234, tallies=b)
    assert (a == b).all()
