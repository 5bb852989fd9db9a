"""Pins of the oracle's interpolated walks (Sec. V A, "Interpolation"), CPU only.

The interpolated rows are pinned to their ends (alpha = 0 and 1 give the exact transmission
of the dense probe solve at the nodes), to second-order accuracy in the node spacing on a
smooth problem, and the C walker's interpolated walks to the exact Markov expectation of the
mixed rows and to the mixture's first-step law.
"""
import numpy as np
import pytest
from scipy.stats import binom

from oracle import dense as D
from oracle import interp as OI
from oracle import walker as OW


def sols_at(Es, W=2, L=4, eta=0.3, seed=4):
    V = np.random.default_rng(seed).uniform(-0.2, 0.2, W * L)
    return [D.EnergySolution(E, W, L, 1.0, V, np.full(W * L, eta)) for E in Es]


def test_bracket():
    nodes = [-1.0, 0.0, 2.0]
    assert OI.bracket(nodes, 1.0) == (1, 0.5)
    assert OI.bracket(nodes, -1.0) == (0, 0.0)
    assert OI.bracket(nodes, 2.0) == (2, 0.0)
    lo, a = OI.bracket(nodes, -0.25)
    assert lo == 0 and a == pytest.approx(0.75)
    for bad in (-1.5, 2.5):
        with pytest.raises(ValueError):
            OI.bracket(nodes, bad)
    with pytest.raises(ValueError):
        OI.bracket([0.0, 0.0, 1.0], 0.5)
    assert OI.alpha_fixed32(0.5) == 1 << 31 and OI.alpha_fixed32(1.0) == 0xFFFFFFFF


@pytest.mark.parametrize("inject_lead", [0, 1])
def test_interpolated_transmission_reduces_to_the_nodes(inject_lead):
    a, b = sols_at([0.3, 0.5])
    Ka, Kb = a.transition_kernel(), b.transition_kernel()
    assert OI.interpolated_transmission(Ka, Kb, 0.0, inject_lead) == pytest.approx(a.T_eff, rel=1e-10)
    assert OI.interpolated_transmission(Ka, Kb, 1.0, inject_lead) == pytest.approx(b.T_eff, rel=1e-10)


def test_interpolation_error_is_second_order():
    # midpoint of [E - h, E + h]: the error of the interpolated transmission against the exact
    # one falls about four times when h halves
    E = 0.4
    errs = []
    for h in (0.08, 0.04):
        a, m, b = sols_at([E - h, E, E + h])
        T = OI.interpolated_transmission(a.transition_kernel(), b.transition_kernel(), 0.5)
        errs.append(abs(T - m.T_eff))
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_row_distance_and_refine():
    Es = [0.0, 0.02, 0.9]
    sols = sols_at(Es)
    Ks = [s.transition_kernel() for s in sols]
    d01 = OI.row_distances(Ks[0], Ks[1])
    assert d01.shape == (Ks[0].shape[0],) and d01.max() < 0.05
    assert OI.row_distances(Ks[0], Ks[0]).max() == 0.0
    fine = [0.0, 0.01, 0.02, 0.3, 0.6, 0.9]
    need, d = OI.refine(Es, Ks, fine)
    assert d[0] < 0.05 < d[1]
    assert need == [0.3, 0.6]


def nodes_tables(sols):
    n = sols[0].N + 2
    K = np.stack([s.transition_kernel() for s in sols])
    thr = np.zeros((len(sols), n, n), np.uint32)
    al = np.zeros((len(sols), n, n), np.int32)
    for e in range(len(sols)):
        for r in range(n):
            thr[e, r], al[e, r] = D.alias_vose(K[e, r])
    return K, thr, al


@pytest.mark.parametrize("inject_lead", [0, 1])
@pytest.mark.parametrize("sampler", ["cdf", "alias"])
def test_interpolated_walks_center_on_the_exact_mixture(inject_lead, sampler):
    nodes = [0.1, 0.35, 0.6]
    sols = sols_at(nodes, eta=0.4)
    K, thr, al = nodes_tables(sols)
    fine = [0.1, 0.2, 0.3, 0.35, 0.5, 0.6]
    br = [OI.bracket(nodes, E) for E in fine]
    lo = [b[0] for b in br]
    a32 = [OI.alpha_fixed32(b[1]) for b in br]
    nw = 200_000
    if sampler == "cdf":
        tal = OW.walk_interp_cdf(K, lo, a32, 123, 1, inject_lead, 0, nw)
    else:
        tal = OW.walk_interp_alias(thr, al, lo, a32, 123, 1, inject_lead, 0, nw)
    row = K.shape[1] - 2 + inject_lead
    for f, (l, a) in enumerate(br):
        hi = min(l + 1, len(nodes) - 1)
        alpha = a32[f] / 2.0 ** 32
        T_ref = OI.interpolated_transmission(K[l], K[hi], alpha, inject_lead)
        c = (1 - alpha) * K[l, row].sum() + alpha * K[hi, row].sum()
        T, sig, _, _ = OW.mc_current(tal[f:f + 1], [c], [1.0], inject_lead)
        assert abs(T[0] - T_ref) < 4 * sig[0], (f, T[0], T_ref, sig[0])
        assert tal[f, :3].sum() == nw


def test_first_step_is_the_mixture_of_the_two_rows():
    # max_steps = 1: a walk ends at its injection draw; it exits into L with probability
    # (1 - alpha) p_a(L | L) + alpha p_b(L | L)
    sols = sols_at([0.1, 0.9], eta=0.4)
    K, _, _ = nodes_tables(sols)
    N = K.shape[1] - 2
    alpha = 0.3
    a32 = OI.alpha_fixed32(alpha)
    nw = 400_000
    tal = OW.walk_interp_cdf(K, [0], [a32], 9, 0, 0, 0, nw, max_steps=1)
    pa = K[0, N, N] / K[0, N].sum()
    pb = K[1, N, N] / K[1, N].sum()
    p = (1 - alpha) * pa + alpha * pb
    lo_q, hi_q = binom.ppf([0.0005, 0.9995], nw, p)
    assert lo_q <= tal[0, 0] <= hi_q
    # the two pure rows give visibly different counts, so the test can tell them apart
    assert abs(pa - pb) * nw > 10 * np.sqrt(nw * p * (1 - p))
