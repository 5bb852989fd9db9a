"""Pins of the oracle's inelastic walk (step 7', Sec. II F) on the CPU.

- With only the elastic line (offset 0) the chain is the elastic walk: exits at the injection
  energy with the elastic absorption probabilities (themselves pinned to T_eff), and the C
  walker's tallies equal the elastic walker's bit for bit (the energy words are a separate
  stream).
- The linear solve of the chain agrees with a plain step-by-step propagation of the walk's
  probability mass (the Neumann series of the same chain), and the exit probabilities sum to 1.
- The threshold table gives the normalised line probabilities to 2^-32; weightless lines are
  never drawn.
- The C walker (both samplers) reproduces the exact exit distribution within 5 sigma; with
  emission lines only, no walk ever gains energy.
"""
import numpy as np
import pytest

from oracle import dense as D
from oracle import inelastic as IN
from oracle import walker as OW

SEED = 180510164


def system(W, L, nE, eta=0.3, seed=3, emin=-1.4, emax=1.2):
    V = np.random.default_rng(seed).uniform(-0.3, 0.3, W * L)
    g = np.full(W * L, eta)
    E, _ = D.midpoint_grid(emin, emax, nE)
    sols = [D.EnergySolution(x, W, L, 1.0, V, g) for x in E]
    Ks = np.array([s.transition_kernel() for s in sols])
    A = np.array([s.Adiag for s in sols])
    return sols, Ks, A


def test_elastic_line_is_the_elastic_walk():
    sols, Ks, A = system(2, 3, 5)
    N = 6
    for lead in (0, 1):
        B = IN.exit_distribution(Ks, A, [0], [1.0], lead)
        for e0, s in enumerate(sols):
            h = D.absorption_probabilities(Ks[e0])        # P(exit at R | state)
            pR = h[N + lead]
            ref = np.zeros((2, 5))
            ref[0, e0], ref[1, e0] = 1.0 - pR, pR
            assert np.abs(B[e0] - ref).max() < 1e-12
            # the estimator's mean is the effective transmission (Eq. (66))
            c = s.trGLA if lead == 0 else s.trGRA
            q = 1 - lead
            assert c * B[e0, q, e0] == pytest.approx(s.T_eff, rel=1e-10)


def test_solve_equals_step_by_step_propagation():
    sols, Ks, A = system(1, 2, 4, eta=0.6)
    off, lam = [-1, 0, 2], [0.5, 1.0, 0.3]
    B = IN.exit_distribution(Ks, A, off, lam, 0)
    P = Ks / Ks.sum(axis=2, keepdims=True)
    pe = IN.energy_probabilities(A, off, lam)
    nE, N = 4, 2
    for e0 in range(nE):
        ref = np.zeros((2, nE))
        # mass[e][s]: probability of standing at row s of energy e; start at lead L's row
        mass = np.zeros((nE, N + 2))
        mass[e0, N] = 1.0
        for _ in range(2000):
            nxt = np.zeros((nE, N + 2))
            for e in range(nE):
                for s in range(N + 2):
                    m = mass[e, s]
                    if m == 0.0:
                        continue
                    ref[0, e] += m * P[e, s, N]
                    ref[1, e] += m * P[e, s, N + 1]
                    for i in range(N):
                        for k, d in enumerate(off):
                            if 0 <= e + d < nE:
                                nxt[e + d, i] += m * P[e, s, i] * pe[e, i, k]
            mass = nxt
        assert mass.sum() < 1e-14
        assert np.abs(B[e0] - ref).max() < 1e-12
        assert B[e0].sum() == pytest.approx(1.0, abs=1e-12)


def test_table_gives_the_line_probabilities():
    _, _, A = system(2, 2, 6)
    off, lam = [-2, 0, 1, 3], [0.4, 1.0, 0.0, 0.25]
    t = IN.energy_table(A, off, lam)
    p = IN.energy_probabilities(A, off, lam)
    assert t.dtype == np.uint64
    assert (np.diff(t.astype(np.int64), axis=2) >= 0).all()
    assert np.abs(IN.table_probabilities(t) - p).max() <= 1.0 / IN.TWO32
    assert (IN.table_probabilities(t)[:, :, 2] == 0).all()          # lambda = 0
    # lines off the grid: energy 0 cannot go down, energy 5 cannot go up by 1 or 3
    assert (IN.table_probabilities(t)[0, :, 0] == 0).all()
    assert (IN.table_probabilities(t)[5, :, 2:] == 0).all()
    assert (t[5, :, 1] == 2 ** 32).all()


def test_table_rejects_a_probe_with_nowhere_to_go():
    _, _, A = system(1, 2, 3)
    with pytest.raises(ValueError):
        IN.energy_table(A, [-3, 4], [1.0, 1.0])


@pytest.mark.parametrize("lead", [0, 1])
def test_elastic_limit_of_the_walker_is_the_elastic_walker(lead):
    _, Ks, A = system(2, 3, 4)
    t = IN.energy_table(A, [0], [1.0])
    nw = 20_000
    tal, hist, bad = IN.walk_cdf(Ks, t, [0], SEED, 1, lead, 5, nw)
    ref = OW.walk_cdf(Ks, SEED, 1, lead, 5, nw)
    assert not bad
    assert np.array_equal(tal, ref)
    for e0 in range(4):
        assert hist[0, e0, e0] == tal[e0, 0] and hist[1, e0, e0] == tal[e0, 1]
    assert hist.sum() == tal[:, 0].sum() + tal[:, 1].sum()


@pytest.mark.parametrize("mode", ["cdf", "alias"])
def test_walker_reproduces_the_exact_exit_distribution(mode):
    _, Ks, A = system(2, 2, 6, eta=0.5)
    off, lam = [-2, 0, 1], [0.6, 1.0, 0.3]
    t = IN.energy_table(A, off, lam)
    nw = 100_000
    if mode == "cdf":
        tal, hist, bad = IN.walk_cdf(Ks, t, off, SEED, 0, 0, 0, nw)
    else:
        n = Ks.shape[1]
        pitch = 16
        thr = np.zeros((6, n, pitch), dtype=np.uint32)
        al = np.zeros((6, n, pitch), dtype=np.int32)
        for e in range(6):
            for s in range(n):
                a, b = D.alias_vose(Ks[e, s])
                thr[e, s, :n], al[e, s, :n] = a, b
                al[e, s, n:] = s
        tal, hist, bad = IN.walk_alias(thr, al, t, off, SEED, 0, 0, 0, nw)
    assert not bad and tal[:, 2].sum() == 0
    B = IN.exit_distribution(Ks, A, off, lam, 0, p_energy=IN.table_probabilities(t))
    expect = B.transpose(1, 0, 2) * nw                    # [r][e0][e]
    big = expect >= 400
    assert big.sum() >= 20
    assert (np.abs(hist[big] - expect[big]) <= 5 * np.sqrt(expect[big])).all()
    small = ~big
    assert hist[small].sum() <= expect[small].sum() + 5 * np.sqrt(expect[small].sum()) + 5


def test_emission_only_never_gains_energy():
    _, Ks, A = system(1, 3, 8, eta=0.8)
    off, lam = [0, -1, -3], [0.2, 1.0, 1.0]
    t = IN.energy_table(A, off, lam)
    tal, hist, bad = IN.walk_cdf(Ks, t, off, SEED, 2, 1, 0, 20_000)
    assert not bad
    for e0 in range(8):
        assert hist[:, e0, e0 + 1:].sum() == 0
    assert hist[:, 5:, :].sum(axis=(0, 1))[:5].sum() > 0       # walks relax downwards


def test_spectrum_sums_to_the_current():
    sols, Ks, A = system(2, 2, 5)
    off, lam = [-1, 0, 1], [0.3, 1.0, 0.3]
    t = IN.energy_table(A, off, lam)
    tal, hist, _ = IN.walk_cdf(Ks, t, off, SEED, 0, 0, 0, 30_000)
    c = np.array([s.trGLA for s in sols])
    w = np.linspace(0.1, 0.2, 5)
    S = IN.spectrum(tal, hist, c, w, 0)
    _, _, I, _ = OW.mc_current(tal, c, w, 0)
    assert S[1].sum() == pytest.approx(I, rel=1e-12)


def test_truncated_walks_are_tallied():
    _, Ks, A = system(2, 3, 3, eta=1.0)
    t = IN.energy_table(A, [-1, 0, 1], [1.0, 1.0, 1.0])
    tal, hist, _ = IN.walk_cdf(Ks, t, [-1, 0, 1], SEED, 0, 0, 0, 5000, max_steps=3)
    assert tal[:, 2].sum() > 0
    assert (tal[:, :3].sum(axis=1) == 5000).all()
    assert hist.sum() == tal[:, 0].sum() + tal[:, 1].sum()
    assert (tal[:, 3] <= 3 * 5000).all()
