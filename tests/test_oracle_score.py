"""Pins of the oracle's score-function gradient of the Monte Carlo estimator (CPU only).

The estimator is linear in the transition counts of the walks that reach q; with the exact
expected counts it must give the exact derivative of T_eff, which the dense adjoint of
oracle/grad.py (itself pinned to central differences) provides.  The counting walker must
walk the plain walker's paths, and its counts must average to the expected counts.
"""
import numpy as np
import pytest

from oracle import dense as D
from oracle import grad as OG
from oracle import score as SC
from oracle import walker as OW

SEED = 180510164


def wire(W, L, eta, seed, disorder=0.3):
    V = np.random.default_rng(seed).uniform(-disorder, disorder, W * L)
    return V, np.full(W * L, eta)


def test_torch_kernel_is_the_dense_kernel():
    W, L = 2, 4
    V, g = wire(W, L, 0.2, 1)
    g = g * np.linspace(0.5, 1.5, W * L)
    import torch
    s = D.EnergySolution(0.3, W, L, 1.0, V, g)
    K, A, cL, cR = SC.kernel_torch(W, L, 1.0, torch.tensor(V), torch.tensor(g), 0.3)
    Kd = s.transition_kernel()
    assert np.abs(K.numpy() - Kd).max() < 1e-12 * Kd.max()
    assert np.abs(A.numpy() - s.Adiag).max() < 1e-12 * s.Adiag.max()
    assert float(cL) == pytest.approx(s.trGLA, rel=1e-12)
    assert float(cR) == pytest.approx(s.trGRA, rel=1e-12)


@pytest.mark.parametrize("W,L,eta,E,lead", [(1, 5, 0.3, 0.4, 0), (2, 4, 0.2, -0.9, 0),
                                            (2, 4, 0.2, -0.9, 1), (3, 3, 0.25, 1.3, 0)])
def test_expected_counts_give_the_exact_gradient(W, L, eta, E, lead):
    V, g = wire(W, L, eta, W + L)
    g = g * np.linspace(0.7, 1.3, W * L)
    s = D.EnergySolution(E, W, L, 1.0, V, g)
    Ec = SC.expected_counts(s.transition_kernel(), lead)
    dV, dG = SC.score_gradient(W, L, 1.0, V, g, E, Ec, 1.0, lead)
    _, rV, rG = OG.adjoint(W, L, 1.0, V, g, [E], [1.0])
    assert np.abs(dV - rV).max() <= 1e-8 * np.abs(rV).max()
    assert np.abs(dG - rG).max() <= 1e-8 * np.abs(rG).max()


def test_expected_counts_by_enumeration():
    # a two-probe chain: E[C] from summing the probabilities of every path of up to 80 steps
    # that ends at q, step by step
    W, L = 1, 2
    V, g = wire(W, L, 0.5, 3)
    s = D.EnergySolution(0.2, W, L, 1.0, V, g)
    K = s.transition_kernel()
    P = K / K.sum(axis=1, keepdims=True)
    N, q = 2, 3
    h = D.absorption_probabilities(K)  # exit at R from each state
    ref = np.zeros((4, 4))
    front = {N: 1.0}  # probability of being at a state after n steps (injection row L)
    for _ in range(80):
        nxt = {}
        for sidx, pr in front.items():
            for o in (0, 1, q):
                w = pr * P[sidx, o]
                # this step lies on a walk that reaches q with probability h_o (1 at q)
                ref[o, sidx] += w * (1.0 if o == q else h[o])
                if o < N:
                    nxt[o] = nxt.get(o, 0.0) + w
        front = nxt
    assert np.abs(SC.expected_counts(K, 0) - ref).max() < 1e-12


@pytest.mark.parametrize("lead", [0, 1])
def test_counting_walker_walks_the_plain_paths(lead):
    W, L = 2, 3
    V, g = wire(W, L, 0.3, 7)
    s = D.EnergySolution(-0.5, W, L, 1.0, V, g)
    K = s.transition_kernel()
    n = K.shape[0]
    N = n - 2
    q = N + 1 - lead
    nw = 30_000
    tal, cnt = SC.walk_counts_cdf(K, SEED, 2, lead, 11, nw)
    assert np.array_equal(tal, OW.walk_cdf(K[None], SEED, 2, lead, 11, nw))
    c = cnt[0]
    hits = tal[0, 1 - lead]
    # every walk that reaches q leaves the injection row once and enters q once
    assert c[:, N + lead].sum() == hits and c[q, :].sum() == hits
    assert c[N + lead, :].sum() == 0 and c[:, q].sum() == 0  # nothing enters p or leaves q
    # the counts average to the expected counts (entries with >= 400 expected counts, 5 sigma)
    Ec = SC.expected_counts(K, lead) * nw
    big = Ec >= 400
    assert big.sum() >= 4
    assert (np.abs(c[big] - Ec[big]) <= 5 * np.sqrt(Ec[big])).all()


def test_sampled_score_gradient_is_unbiased():
    # d T / d eta (the sum over gamma_i) from 8 batches of counts: batch mean within 4 sigma
    W, L, E = 2, 5, 0.6
    V, g = wire(W, L, 0.2, 9)
    s = D.EnergySolution(E, W, L, 1.0, V, g)
    K = s.transition_kernel()
    _, rV, rG = OG.adjoint(W, L, 1.0, V, g, [E], [1.0])
    ests_eta, ests_v = [], []
    nw = 40_000
    for b in range(8):
        tal, cnt = SC.walk_counts_cdf(K, SEED, 0, 0, b * nw, nw)
        dV, dG = SC.score_gradient(W, L, 1.0, V, g, E, cnt[0], nw, 0)
        ests_eta.append(dG.sum())
        ests_v.append(dV[3])
    for est, ref in ((ests_eta, rG.sum()), (ests_v, rV[3])):
        m, sd = np.mean(est), np.std(est, ddof=1) / np.sqrt(len(est))
        assert abs(m - ref) < 4 * sd + 1e-12, (m, ref, sd)
