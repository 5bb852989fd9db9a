"""Pins of the oracle's C walker and its Philox4x32-10 (CPU only)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import dense as D
from oracle import walker

HERE = os.path.dirname(os.path.abspath(__file__))


def read_kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_published_known_answers():
    for ctr, key, out in read_kat():
        assert walker.philox4x32_10(ctr, key) == out


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available to build the rocRAND cross-check")
def test_philox_matches_rocrand_engine(tmp_path):
    # rocRAND's philox4x32_10_engine run on the host: counter = (offset/4, subsequence),
    # key = seed.  Counters are kept below 2^30 in word 1 so offset*4 fits 64 bits.
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    exe = str(tmp_path / "kat")
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", exe,
                           os.path.join(HERE, "philox_rocrand_kat.cpp")])
    rng = np.random.default_rng(11)
    cases = [([0, 0, 0, 0], [0, 0]), ([3, 12345, 77, 1], [180510164, 0])]
    for _ in range(30):
        ctr = [int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 30)),
               int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 32))]
        key = [int(rng.integers(0, 2 ** 32)), int(rng.integers(0, 2 ** 32))]
        cases.append((ctr, key))
    inp = "".join("%x %x %x %x %x %x\n" % (*c, *k) for c, k in cases)
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    got = [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    assert got == [walker.philox4x32_10(c, k) for c, k in cases]


def small_problem(W=1, L=3, eta=0.3, E=0.2, seed=0):
    V = np.random.default_rng(seed).uniform(-0.2, 0.2, W * L)
    s = D.EnergySolution(E, W, L, 1.0, V, np.full(W * L, eta))
    return s, s.transition_kernel()


@pytest.mark.parametrize("mode", ["cdf", "alias"])
def test_walker_absorption_probability_within_4_sigma(mode):
    s, K = small_problem()
    N = s.N
    h = D.absorption_probabilities(K)
    n = 400_000
    if mode == "cdf":
        t = walker.walk_cdf(K, seed=99, realization=0, inject_lead=0, walker_begin=0,
                            n_walkers=n)
    else:
        thr = np.zeros((N + 2, N + 2), np.uint32)
        al = np.zeros((N + 2, N + 2), np.int32)
        for r in range(N + 2):
            thr[r], al[r] = D.alias_vose(K[r])
        t = walker.walk_alias(thr, al, seed=99, realization=0, inject_lead=0, walker_begin=0,
                              n_walkers=n)
    t = t[0]
    assert t[0] + t[1] + t[2] == n and t[2] == 0
    p = h[N]
    sig = np.sqrt(p * (1 - p) / n)
    assert abs(t[1] / n - p) < 4 * sig


def test_walker_chi_square_of_first_exit_from_each_probe():
    # The injection draw alone (max_steps = 1): probes / lead L / lead R must follow the
    # normalised lead row (chi-square, p-value above 1e-4).
    from scipy.stats import chisquare
    s, K = small_problem(W=2, L=2, eta=0.5)
    N = s.N
    n = 200_000
    t = walker.walk_cdf(K, seed=5, realization=3, inject_lead=0, walker_begin=0,
                        n_walkers=n, max_steps=1)
    # max_steps = 1: walkers whose first draw is a probe are truncated
    obs = np.array([t[0, 2], t[0, 0], t[0, 1]], dtype=float)
    pr = K[N] / K[N].sum()
    exp = np.array([pr[:N].sum(), pr[N], pr[N + 1]]) * n
    assert chisquare(obs, exp).pvalue > 1e-4


def test_walker_batch_split_and_determinism():
    s, K = small_problem(W=2, L=3, eta=0.2)
    a = walker.walk_cdf(K, 7, 1, 0, 0, 30_000)
    b = walker.walk_cdf(K, 7, 1, 0, 0, 12_345)
    b = walker.walk_cdf(K, 7, 1, 0, 12_345, 30_000 - 12_345, tallies=b)
    c = walker.walk_cdf(K, 7, 1, 0, 0, 30_000)
    assert (a == b).all() and (a == c).all()
    d = walker.walk_cdf(K, 8, 1, 0, 0, 30_000)
    assert not (a == d).all()


def test_walker_single_site_exit_probability():
    # One site with wide-band leads and a probe: P(exit at R) = T_eff / Tr Gamma_L A.
    s = D.EnergySolution(0.1, 1, 1, 1.0, np.zeros(1), np.array([0.3]), lead_model=1,
                         gamma_l=0.4)
    K = s.transition_kernel()
    n = 300_000
    t = walker.walk_cdf(K, 3, 0, 0, 0, n)[0]
    p = s.T_eff / K[1].sum()
    assert abs(t[1] / n - p) < 4 * np.sqrt(p * (1 - p) / n)
    # mean number of steps of a geometric number of probe visits: 1 / (1 - P(probe->probe))
    q = K[0, 0] / K[0].sum()
    pin = K[1, 0] / K[1].sum()
    mean_steps = 1 + pin / (1 - q)
    assert abs(t[3] / n - mean_steps) < 5 * np.sqrt(t[4] / n - (t[3] / n) ** 2) / np.sqrt(n)


def test_golden_redraw_walkers_are_rejected_by_the_bucket_rule():
    # each listed walker's injection word a (word 0 of counter (0, w, 0, tag)) is rejected by
    # Lemire's rule (a * n mod 2^32 < 2^32 mod n); listed double redraws also have their
    # first redraw word (counter (0, w, 0, tag | 2^31), key (key0, key1 ^ 1)) rejected
    path = os.path.join(HERE, "golden", "lemire_redraws.txt")
    if not os.path.exists(path):
        pytest.skip("golden file not generated")
    rows = [tuple(int(x) for x in line.split()) for line in open(path)
            if line.strip() and not line.startswith("#")]
    assert rows
    for n, seed, real, lead, w, redraws, bucket in rows:
        tag = (real << 1) | lead
        key = [seed & 0xFFFFFFFF, seed >> 32]
        thresh = (1 << 32) % n
        a = walker.philox4x32_10([0, w, 0, tag], key)[0]
        assert (a * n) % (1 << 32) < thresh
        words = [a]
        for r in range(1, redraws + 1):
            words.append(walker.philox4x32_10([0, w, 0, tag | 0x80000000],
                                              [key[0], key[1] ^ r])[0])
        for x in words[:-1]:
            assert (x * n) % (1 << 32) < thresh
        assert (words[-1] * n) % (1 << 32) >= thresh
        assert (words[-1] * n) >> 32 == bucket
