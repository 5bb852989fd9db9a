"""Pins of the oracle's importance-sampled walks (Sec. V A, "Improved estimator"), CPU only.

The weighted estimator is pinned by what the mathematics fixes: with b = 1 it is the plain
walk, count for count; with b = the exact absorption probabilities every walk scores the
transmission exactly (zero variance), which is also the dense NEGF T_eff; for other biases
its mean is the absorption probability and its second moment the exact one, the latter
checked by brute-force path enumeration on a chain of two probes and two leads.
"""
import numpy as np
import pytest

from oracle import dense as D
from oracle import walker as OW
from oracle import weighted as WT

SEED = 180510164


def problem(W=2, L=6, eta=0.3, E=0.2, seed=0):
    V = np.random.default_rng(seed).uniform(-0.25, 0.25, W * L)
    s = D.EnergySolution(E, W, L, 1.0, V, np.full(W * L, eta))
    return s, s.transition_kernel()


def test_unit_bias_is_the_plain_walk():
    _, K = problem()
    n = K.shape[0]
    b = np.ones(n)
    for lead in (0, 1):
        plain = OW.walk_cdf(K[None], SEED, 0, lead, 0, 20000)
        t, ws = WT.walk_weighted_cdf(K, b, SEED, 0, lead, 0, 20000)
        assert np.array_equal(t, plain)
        hits = plain[0, 1 - lead]
        # every ratio is rho_i / 1 with rho_i = sum_j p_ij = 1 up to rounding
        assert ws[0, 0] == pytest.approx(hits, rel=1e-12)
        assert ws[0, 1] == pytest.approx(hits, rel=1e-12)
    rows = [D.alias_vose(r) for r in K]
    thr = np.array([r[0] for r in rows], dtype=np.uint32)[None]
    al = np.array([r[1] for r in rows], dtype=np.int32)[None]
    plain = OW.walk_alias(thr, al, SEED, 0, 0, 0, 20000)
    t, ws = WT.walk_weighted_alias(thr, al, WT.rho(K, b), b, SEED, 0, 0, 0, 20000)
    assert np.array_equal(t, plain)


@pytest.mark.parametrize("lead", [0, 1])
def test_exact_absorption_bias_has_zero_variance(lead):
    # b = P(exit at q | state): rho = b on every row, the ratios telescope to b(injection row)
    # and c_p b(injection row) is the dense NEGF transmission
    s, K = problem(W=2, L=5, eta=0.2, E=-0.7, seed=3)
    n = K.shape[0]
    N = n - 2
    h = D.absorption_probabilities(K)  # exit at R
    b = h if lead == 0 else 1.0 - h
    b = b.copy()
    b[N + lead] = 0.0   # never sample lead p: those walks score 0 anyway
    b[N + 1 - lead] = 1.0
    nw = 4000
    t, ws = WT.walk_weighted_cdf(K, b, SEED, 0, lead, 0, nw)
    assert t[0, lead] == 0 and t[0, 2] == 0 and t[0, 1 - lead] == nw
    x = ws[0, 0] / nw
    assert x == pytest.approx(h[N] if lead == 0 else 1.0 - h[N + 1], rel=1e-12)
    assert ws[0, 1] / nw == pytest.approx(x * x, rel=1e-12)
    c = K[N + lead].sum()
    T, sig, _, _ = WT.weighted_current(t, ws, [c], [1.0])
    # the effective two-terminal transmission is reciprocal in linear response
    assert T[0] == pytest.approx(s.T_eff, rel=1e-10)
    assert sig[0] < 1e-6 * T[0]


@pytest.mark.parametrize("a", [3.0, 6.0])
def test_ramp_bias_is_unbiased_and_matches_the_exact_second_moment(a):
    s, K = problem(W=2, L=12, eta=0.25, E=0.4, seed=5)
    n = K.shape[0]
    N = n - 2
    b = WT.ramp_bias(2, 12, 0, a=a, floor_p=1e-3)
    m2 = WT.second_moment(K, b, 0)
    assert np.isfinite(m2)
    p = D.absorption_probabilities(K)[N]
    nw = 400_000
    t, ws = WT.walk_weighted_cdf(K, b, SEED, 1, 0, 0, nw)
    mean = ws[0, 0] / nw
    sd = np.sqrt((m2 - p * p) / nw)
    assert abs(mean - p) < 4 * sd
    # sample second moment against the exact one (its own spread is far below 5% here)
    assert ws[0, 1] / nw == pytest.approx(m2, rel=0.05)
    # the ramp lowers the variance below the plain walk's p (1 - p)
    assert m2 - p * p < 0.5 * p * (1 - p)


def test_second_moment_by_path_enumeration():
    # a chain with one probe pair and both leads (n = 4): enumerate every path of up to 80
    # steps under p' and sum p'(path) X'(path) and p'(path) X'(path)^2
    rng = np.random.default_rng(2)
    K = rng.uniform(0.1, 1.0, (4, 4))
    K[2, 2] = K[3, 3] = 0.0
    b = np.array([0.4, 0.7, 0.05, 1.0])
    P = WT.normalised(K)
    Pp = WT.normalised(WT.modified_rows(K, b))
    r = WT.rho(K, b)
    N, q = 2, 3
    m1 = m2 = 0.0
    # state distribution over probes with (probability, score, score^2) carried along
    front = {2: (1.0, 1.0, 1.0)}  # injection row of lead L (row N)
    for _ in range(80):
        nxt = {}
        for i, (pp, x, x2) in front.items():
            for j in range(4):
                if Pp[i, j] == 0.0 or j == N:
                    continue
                f = r[i] / b[j]
                w = pp * Pp[i, j]
                if j == q:
                    m1 += w * x * f
                    m2 += w * x2 * f * f
                else:
                    a = nxt.get(j, (0.0, 0.0, 0.0))
                    # keep the probability-weighted mean score and squared score per state
                    nxt[j] = (a[0] + w, a[1] + w * x * f, a[2] + w * x2 * f * f)
        front = {j: (v[0], v[1] / v[0], v[2] / v[0]) for j, v in nxt.items() if v[0] > 0}
    h = D.absorption_probabilities(K)
    assert m1 == pytest.approx(h[N], rel=1e-10)
    assert m2 == pytest.approx(WT.second_moment(K, b, 0), rel=1e-10)
    # the plain walk (b = 1) has second moment = mean = P(exit at q)
    assert WT.second_moment(K, np.ones(4), 0) == pytest.approx(h[N], rel=1e-12)


def test_second_moment_reports_divergence():
    # a bias that starves the path to q makes the ratios explode
    _, K = problem(W=1, L=8, eta=0.4, E=0.1, seed=1)
    n = K.shape[0]
    b = np.full(n, 1.0)
    b[:n - 2] = 1e-3
    b[n - 3] = 1e-6
    assert WT.second_moment(K, b, 0) == float("inf")


def test_weighted_current_closed_form():
    # scores 0, 2, 2, 0 (times c = 3): mean 1, sample variance 4/3
    t = np.array([[2, 2, 0, 10, 30]])
    ws = np.array([[4.0, 8.0]])
    T, sig, I, sI = WT.weighted_current(t, ws, [3.0], [0.5])
    assert T[0] == pytest.approx(3.0)
    assert sig[0] == pytest.approx(3.0 * np.sqrt(4.0 / 3.0 / 4.0))
    assert I == pytest.approx(1.5) and sI == pytest.approx(0.5 * sig[0])


def test_ramp_bias_layout():
    b = WT.ramp_bias(3, 4, 0, a=1.0, floor_p=0.0)
    assert b.shape == (14,)
    assert b[0] == b[2] == pytest.approx(1.5 / 6.0) and b[11] == pytest.approx(4.5 / 6.0)
    assert b[12] == 0.0 and b[13] == 1.0
    b1 = WT.ramp_bias(3, 4, 1, a=1.0, floor_p=0.2)
    assert b1[0] == pytest.approx(4.5 / 6.0) and b1[12] == 1.0 and b1[13] == 0.2
