"""Pins of the oracle's Monte Carlo estimator of the transmission and its standard error
(oracle.walker.mc_current; Eq. (66), Sec. IV A), CPU only.

The estimator is pinned to (i) the textbook sample variance of the explicit per-walker
scores, computed by numpy from the scores themselves, (ii) the exact transmission of the
dense probe solve as the mean over many independent replicates, and the spread of those
replicates as the standard error the estimator states, and (iii) the clean chain at eta = 0,
whose scores are 0 or 2 with probability 1/2 each (closed form).
"""
import numpy as np
import pytest

from oracle import dense as D
from oracle import walker as OW


def scores_from_tallies(t, c, inject_lead):
    """The N scores of one energy's walkers: c for an exit at the collecting lead, else 0."""
    walkers = int(t[0] + t[1] + t[2])
    hits = int(t[1] if inject_lead == 0 else t[0])
    return np.concatenate([np.full(hits, c), np.zeros(walkers - hits)])


@pytest.mark.parametrize("inject_lead", [0, 1])
def test_standard_error_is_the_sample_variance_of_the_scores(inject_lead):
    # tallies with truncated walks: they score 0 and count as walkers
    t = np.array([[120, 75, 5, 0, 0], [3, 997, 0, 0, 0], [40, 40, 20, 0, 0], [0, 1, 0, 0, 0],
                  [7, 0, 0, 0, 0]], dtype=np.int64)
    c = np.array([1.7, 0.4, 2.5, 3.0, 0.9])
    w = np.array([0.1, 0.3, 0.05, 0.2, 0.7])
    T, sig, I, sI = OW.mc_current(t, c, w, inject_lead)
    for k in range(len(c)):
        X = scores_from_tallies(t[k], c[k], inject_lead)
        assert T[k] == pytest.approx(X.mean(), rel=1e-14, abs=1e-300)
        ref = np.sqrt(np.var(X, ddof=1) / len(X)) if len(X) > 1 else 0.0
        assert sig[k] == pytest.approx(ref, rel=1e-12, abs=1e-14 * c[k])
    assert I == pytest.approx(float(np.sum(w * T)), rel=1e-15)
    assert sI == pytest.approx(float(np.sqrt(np.sum((w * sig) ** 2))), rel=1e-15)


def test_no_walkers_gives_zero():
    T, sig, I, sI = OW.mc_current(np.zeros((2, 5), np.int64), [1.0, 2.0], [0.5, 0.5])
    assert (T == 0).all() and (sig == 0).all() and I == 0 and sI == 0


@pytest.mark.parametrize("inject_lead", [0, 1])
def test_replicates_center_on_the_exact_transmission_with_the_stated_spread(inject_lead):
    # 3 energies of a disordered W = 2, L = 3 wire; R independent replicates (disjoint walker
    # ranges of the counter-based streams) of n walkers each on the oracle's Vose tables
    W, L, eta = 2, 3, 0.4
    V = np.random.default_rng(3).uniform(-0.3, 0.3, W * L)
    Es = np.array([-1.3, 0.2, 1.9])
    w = np.array([0.25, 0.5, 0.25])
    sols = [D.EnergySolution(E, W, L, 1.0, V, np.full(W * L, eta)) for E in Es]
    n = W * L + 2
    thr = np.zeros((3, n, n), np.uint32)
    al = np.zeros((3, n, n), np.int32)
    for e, s in enumerate(sols):
        K = s.transition_kernel()
        for r in range(n):
            thr[e, r], al[e, r] = D.alias_vose(K[r])
    row = n - 2 + inject_lead
    c = np.array([s.transition_kernel()[row].sum() for s in sols])
    T_ref = np.array([s.T_eff for s in sols])  # T_RL = T_LR (reciprocity)
    I_ref = float(np.sum(w * T_ref))
    R, nw = 400, 2000
    Ts, sigs, Is, sIs = [], [], [], []
    for i in range(R):
        tal = OW.walk_alias(thr, al, 77, 0, inject_lead, i * nw, nw)
        T, sig, I, sI = OW.mc_current(tal, c, w, inject_lead)
        Ts.append(T)
        sigs.append(sig)
        Is.append(I)
        sIs.append(sI)
    Ts, sigs = np.array(Ts), np.array(sigs)
    # mean over R * n walkers: within 4 standard errors of the exact value
    assert np.all(np.abs(Ts.mean(0) - T_ref) < 4 * sigs.mean(0) / np.sqrt(R))
    assert abs(np.mean(Is) - I_ref) < 4 * np.mean(sIs) / np.sqrt(R)
    # the replicates' variance equals the stated sigma^2 (relative scatter sqrt(2/R) = 7%)
    ratio = Ts.var(0, ddof=1) / (sigs ** 2).mean(0)
    assert np.all(np.abs(ratio - 1.0) < 0.3), ratio
    ratio_I = np.var(Is, ddof=1) / np.mean(np.square(sIs))
    assert abs(ratio_I - 1.0) < 0.3, ratio_I


def test_clean_chain_scores_are_zero_or_two():
    # clean chain, eta = 0, inside the band: c_L = Tr Gamma_L A = 2, every walker leaves at
    # its injection draw, into R with probability T_RL / c_L = 1/2: T = 1, sigma = 1/sqrt(N)
    s = D.EnergySolution(0.3, 1, 4, 1.0, np.zeros(4), np.zeros(4))
    K = s.transition_kernel()
    n = K.shape[0]
    thr = np.zeros((1, n, n), np.uint32)
    al = np.zeros((1, n, n), np.int32)
    for r in range(n):
        thr[0, r], al[0, r] = D.alias_vose(K[r])
    c = K[n - 2].sum()
    assert c == pytest.approx(2.0, rel=1e-10)
    nw = 200_000
    tal = OW.walk_alias(thr, al, 5, 0, 0, 0, nw)
    assert tal[0, 3] == nw  # one step each
    T, sig, I, sI = OW.mc_current(tal, [c], [1.0])
    assert sig[0] == pytest.approx(1.0 / np.sqrt(nw), rel=1e-3)
    assert abs(T[0] - 1.0) < 4 * sig[0]
