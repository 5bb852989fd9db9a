"""Walker and Monte Carlo current on the GPU (through the C ABI) against the oracle.

The walker's tallies are integers: on alias tables handed to it, they must equal the
oracle walker's bit for bit (same Philox streams, bucket rule and thresholds).  MC currents
must lie within 3 sigma of the oracle's exact value, with the count of per-energy 3-sigma
exceedances at most the 99.9% binomial quantile.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import dense as D  # noqa: E402
from oracle import walker as OW  # noqa: E402
from paper_1805_10164_amd import inputs  # noqa: E402
from paper_1805_10164_amd import mcnegf as M  # noqa: E402
from test_gpu_parity import DEV, SEED, case, gpu_build, oracle_solve, single_site, chain_case  # noqa: E402


def oracle_alias_tables(sols, pitch):
    n = sols[0].N + 2
    thr = np.zeros((len(sols), n, pitch), np.uint32)
    al = np.zeros((len(sols), n, pitch), np.int32)
    for e, s in enumerate(sols):
        K = s.transition_kernel()
        for r in range(n):
            thr[e, r, :n], al[e, r, :n] = D.alias_vose(K[r])
    return thr, al


@pytest.mark.parametrize("inject", [0, 1])
def test_walker_bit_exact_on_given_tables(inject):
    # The GPU walker on alias tables built by the oracle must reproduce the oracle walker's
    # integer tallies exactly (same Philox streams, same bucket and threshold rule).
    c = case(W=3, L=4, eta=0.3, disorder=0.3, nE=3, emin=-1.5, emax=1.5)
    k = gpu_build(c)
    sols = oracle_solve(c)
    thr, al = oracle_alias_tables(sols, k.alias_pitch)
    k.set_alias_tables(thr, al)
    nw = 50_000
    tal = torch.zeros((3, 5), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, SEED, 7, inject, 1000, nw, 1_000_000, tal)
    ref = OW.walk_alias(thr, al, SEED, 7, inject, 1000, nw)
    assert (tal.cpu().numpy() == ref).all()


@pytest.mark.parametrize("max_steps", [1, 2])
def test_walker_truncation_and_max_steps(max_steps):
    # max_steps = 1: every walk ends at its injection step, at a lead or truncated at a probe
    c = case(W=2, L=6, eta=0.5, disorder=0.2, nE=2, emin=-1.0, emax=1.0)
    k = gpu_build(c)
    sols = oracle_solve(c)
    thr, al = oracle_alias_tables(sols, k.alias_pitch)
    k.set_alias_tables(thr, al)
    tal = torch.zeros((2, 5), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, 11, 0, 0, 0, 20_000, max_steps, tal)
    ref = OW.walk_alias(thr, al, 11, 0, 0, 0, 20_000, max_steps=max_steps)
    assert (tal.cpu().numpy() == ref).all() and ref[:, 2].sum() > 0
    w = torch.tensor(c["w"], dtype=torch.float64, device=DEV)
    T = torch.empty(2, dtype=torch.float64, device=DEV)
    sg = torch.empty(2, dtype=torch.float64, device=DEV)
    st, _, _ = M.mc_negf_current(k, 0, 0, tal, w, T, sg)
    assert st == M.WTRUNC


def test_walker_split_ranges_and_determinism():
    c = case(W=4, L=6, eta=0.1, disorder=0.3, nE=4, emin=-2.0, emax=2.0)
    k = gpu_build(c)
    a = torch.zeros((4, 5), dtype=torch.int64, device=DEV)
    b = torch.zeros_like(a)
    d = torch.zeros_like(a)
    M.mc_negf_walk(k, 5, 2, 0, 0, 100_000, 1_000_000, a)
    M.mc_negf_walk(k, 5, 2, 0, 0, 37_001, 1_000_000, b)
    M.mc_negf_walk(k, 5, 2, 0, 37_001, 100_000 - 37_001, 1_000_000, b)
    M.mc_negf_walk(k, 5, 2, 0, 0, 100_000, 1_000_000, d)
    assert torch.equal(a, b) and torch.equal(a, d)
    assert int(a[:, :3].sum()) == 4 * 100_000


def mc_run(c, k, n_walkers, inject=0, seed=SEED):
    nE = len(c["E"])
    tal = torch.zeros((nE, 5), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, seed, 0, inject, 0, n_walkers, 1_000_000, tal)
    w = torch.tensor(c["w"], dtype=torch.float64, device=DEV)
    T = torch.empty(nE, dtype=torch.float64, device=DEV)
    sg = torch.empty(nE, dtype=torch.float64, device=DEV)
    st, I, sI = M.mc_negf_current(k, 0, inject, tal, w, T, sg)
    return st, I, sI, T.cpu().numpy(), sg.cpu().numpy(), tal.cpu().numpy()


def binom_quantile_999(n, p=0.0027):
    from scipy.stats import binom
    return int(binom.ppf(0.999, n, p))


@pytest.mark.parametrize("inject", [0, 1])
def test_mc_current_within_3_sigma(inject):
    c = case(W=4, L=10, eta=0.08, disorder=0.3, nE=24, emin=-3.2, emax=3.2)
    k = gpu_build(c)
    sols = oracle_solve(c)
    st, I, sI, T, sg, tal = mc_run(c, k, 200_000, inject)
    assert st == M.OK
    Tref = np.array([s.T_eff for s in sols])
    Iref = D.current(sols, c["w"])
    assert abs(I - Iref) <= 3 * sI
    exceed = int(np.sum(np.abs(T - Tref) > 3 * sg))
    assert exceed <= binom_quantile_999(len(Tref))


def test_single_site_closed_form_mc():
    c, ref = single_site()
    k = gpu_build(c)
    st, I, sI, Tm, sgm, _ = mc_run(c, k, 400_000)
    assert (np.abs(Tm - ref) < 4 * sgm).all()


def test_clean_chain_eta0_mc():
    c = case(W=1, L=50, eta=0.0, disorder=0.0, nE=8, emin=-1.9, emax=1.9)
    k = gpu_build(c)
    st, I, sI, Tm, sgm, tal = mc_run(c, k, 100_000)
    # every walker leaves at once; half of them into R (c_L = 2)
    assert (tal[:, 3] == 100_000).all()
    assert (np.abs(Tm - 1.0) < 4 * sgm).all()


def test_full_size_chain_mc():
    wl, c = chain_case()
    k = gpu_build(c)
    sols = oracle_solve(c)
    st, I, sI, T, sg, tal = mc_run(c, k, wl.walkers_per_energy)
    Iref = D.current(sols, c["w"])
    assert abs(I - Iref) <= 3 * sI
    Tref = np.array([s.T_eff for s in sols])
    assert int(np.sum(np.abs(T - Tref) > 3 * sg)) <= binom_quantile_999(len(Tref))


def test_outside_band_walkers_exit_at_once():
    c = case(W=1, L=5, eta=0.1, disorder=0.0, nE=2, emin=2.2, emax=2.6)
    k = gpu_build(c)
    st, I, sI, Tm, sgm, tal = mc_run(c, k, 1000)
    assert (Tm == 0).all() and (tal[:, 0] == 1000).all() and (tal[:, 3] == 1000).all()


def test_more_energies_than_one_launch_holds():
    # 2100 energies are walked in many launches (one per round of energies, the last one
    # partial); the streams are keyed by the global energy index, so the oracle walker on the
    # same tables agrees.
    c = case(W=1, L=3, eta=0.2, disorder=0.0, nE=2100, emin=-1.5, emax=1.5)
    k = gpu_build(c)
    sols = oracle_solve(c)
    thr, al = oracle_alias_tables(sols, k.alias_pitch)
    k.set_alias_tables(thr, al)
    tal = torch.zeros((2100, 5), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, 3, 1, 0, 5, 200, 1_000_000, tal)
    ref = OW.walk_alias(thr, al, 3, 1, 0, 5, 200)
    assert (tal.cpu().numpy() == ref).all()


@pytest.mark.parametrize("inject,max_steps", [(0, 1_000_000), (1, 1_000_000), (0, 2), (1, 3)])
def test_mc_estimator_matches_oracle_estimator(inject, max_steps):
    # mode 0 of mc_negf_current against the oracle's estimator on the same tallies, element by
    # element: with the GPU's own row totals c_p (only the estimator's arithmetic differs,
    # 1e-12) and with the oracle's c_p from its dense solve (1e-10); small max_steps gives
    # truncated walks, which score 0 and count as walkers
    c = case(W=3, L=7, eta=0.15, disorder=0.3, nE=11, emin=-2.8, emax=2.8)
    k = gpu_build(c)
    sols = oracle_solve(c)
    nE = len(c["E"])
    tal = torch.zeros((nE, 5), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, SEED, 3, inject, 0, 30_000, max_steps, tal)
    w = torch.tensor(c["w"], dtype=torch.float64, device=DEV)
    T = torch.empty(nE, dtype=torch.float64, device=DEV)
    sg = torch.empty(nE, dtype=torch.float64, device=DEV)
    st, I, sI = M.mc_negf_current(k, 0, inject, tal, w, T, sg)
    t = tal.cpu().numpy()
    if max_steps < 10:
        assert t[:, 2].sum() > 0 and st == M.WTRUNC
    else:
        assert t[:, 2].sum() == 0 and st == M.OK
    T, sg = T.cpu().numpy(), sg.cpu().numpy()
    c_gpu = k.lead().cpu().numpy()[:, M.LEAD_CL if inject == 0 else M.LEAD_CR]
    To, so, Io, sIo = OW.mc_current(t, c_gpu, c["w"], inject)
    assert np.allclose(T, To, rtol=1e-12, atol=0) and np.allclose(sg, so, rtol=1e-12, atol=0)
    assert abs(I - Io) <= 1e-12 * abs(Io) and abs(sI - sIo) <= 1e-12 * sIo
    row = sols[0].N + inject
    c_ora = np.array([s.transition_kernel()[row].sum() for s in sols])
    To, so, Io, sIo = OW.mc_current(t, c_ora, c["w"], inject)
    assert np.allclose(T, To, rtol=1e-10, atol=0) and np.allclose(sg, so, rtol=1e-10, atol=0)
    assert abs(I - Io) <= 1e-10 * abs(Io) and abs(sI - sIo) <= 1e-10 * sIo


def test_zero_walkers_launch_nothing_and_estimate_zero():
    # n_walkers = 0 is a valid request: every walk entry returns OK without touching its
    # outputs, and the estimators of empty tallies give T = 0, sigma = 0 (no division by zero)
    c = case(W=2, L=3, eta=0.2, disorder=0.1, nE=4, emin=-1.2, emax=1.2)
    k = gpu_build(c)
    sentinel = 7
    tal = torch.full((4, M.TALLY_N), sentinel, dtype=torch.int64, device=DEV)
    assert M.mc_negf_walk(k, SEED, 0, 0, 0, 0, 1_000_000, tal) == M.OK
    w = torch.full((4,), 0.25, dtype=torch.float64, device=DEV)
    scratch = torch.empty(max(256, M.mc_negf_walk_sampled_bytes(k, 0)), dtype=torch.uint8,
                          device=DEV)
    assert M.mc_negf_walk_sampled(k, SEED, 0, 0, 0, 0, 1_000_000, w, tal, scratch) == M.OK
    assert M.mc_negf_walk_sampled_noalloc(k, SEED, 0, 0, 0, 0, 1_000_000, w, tal) == M.OK
    counts = torch.full((M.mc_negf_walk_counts_bytes(k) // 4,), sentinel, dtype=torch.int32,
                        device=DEV)
    assert M.mc_negf_walk_counts(k, SEED, 0, 0, 0, 0, 1_000_000, counts, tal) == M.OK
    et = torch.empty(M.mc_negf_energy_table_bytes(k, 1) // 8, dtype=torch.int64, device=DEV)
    M.mc_negf_energy_table(k, [0], [1.0], et)
    hist = torch.full((2, 4, 4), sentinel, dtype=torch.int64, device=DEV)
    assert M.mc_negf_walk_inelastic(k, [0], et, SEED, 0, 0, 0, 0, 1_000_000, tal, hist) == M.OK
    torch.cuda.synchronize()
    assert (tal == sentinel).all() and (hist == sentinel).all() and (counts == sentinel).all()
    tal.zero_()
    T = torch.full((4,), -1.0, dtype=torch.float64, device=DEV)
    sg = torch.full((4,), -1.0, dtype=torch.float64, device=DEV)
    st, I, sI = M.mc_negf_current(k, 0, 0, tal, w, T, sg)
    assert st == M.OK and I == 0.0 and sI == 0.0
    assert (T == 0).all() and (sg == 0).all()


def test_more_energies_than_the_reported_grid_height():
    # the alias build launches rows x energies; 70000 energies exceed the 65536 the runtime
    # reports as the grid's y extent: the tables beyond it must equal single-energy builds, and
    # the walker on all 70000 energies must replay in the oracle walker
    nE = 70_000
    sysm = M.make_system(1, 2)
    V = torch.zeros(2, dtype=torch.float64, device=DEV)
    g = torch.full((2,), 0.1, dtype=torch.float64, device=DEV)
    E, _ = inputs.energy_grid(-1.5, 1.5, nE)
    ws = M.allocate_workspace(sysm, nE)
    k = M.mc_negf_build_kernel(sysm, V, g, torch.tensor(E, device=DEV), ws)
    rows = list(range(k.n_out))
    for e in (0, 65535, 65536, nE - 1):
        thr, al = k.alias_rows(e, rows)
        ws1 = M.allocate_workspace(sysm, 1)
        k1 = M.mc_negf_build_kernel(sysm, V, g, torch.tensor(E[e:e + 1], device=DEV), ws1)
        thr1, al1 = k1.alias_rows(0, rows)
        assert (thr == thr1).all() and (al == al1).all(), e
    thr, al = k.alias_tables()
    tal = torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, SEED, 0, 0, 0, 50, 1_000_000, tal)
    assert (tal.cpu().numpy() == OW.walk_alias(thr, al, SEED, 0, 0, 0, 50)).all()


def test_graph_of_a_whole_step_matches_eager():
    # Capture: the kernel build, zeroed tallies (a fill kernel, no memset node), one walk and
    # both currents into device outputs (mc_negf_current_async).  Replay three times with eager
    # work and synchronisations between replays; every replay must equal the eager run.
    c = case(W=3, L=4, eta=0.3, disorder=0.3, nE=6, emin=-1.5, emax=1.5)
    sysm = M.make_system(3, 4)
    ws = M.allocate_workspace(sysm, 6)
    V = torch.tensor(c["V"], device=DEV)
    g = torch.tensor(c["g"], device=DEV)
    E = torch.tensor(c["E"], device=DEV)
    w = torch.tensor(c["w"], device=DEV)
    tal = torch.zeros((6, M.TALLY_N), dtype=torch.int64, device=DEV)
    T = torch.empty(6, dtype=torch.float64, device=DEV)
    sg = torch.empty_like(T)
    out = torch.zeros((2, 2), dtype=torch.float64, device=DEV)

    def step(stream):
        k = M.mc_negf_build_kernel(sysm, V, g, E, ws, stream)
        tal.zero_()
        M.mc_negf_walk(k, SEED, 0, 0, 0, 20_000, 1_000_000, tal, stream)
        M.mc_negf_current_async(k, 0, 0, tal, w, T, sg, out[0], stream)
        M.mc_negf_current_async(k, 1, 0, None, w, T, sg, out[1], stream)
        return k

    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        k = step(s)
    s.synchronize()
    n = k.n_out
    eager = [x.cpu().numpy().copy() for x in (tal, out, k.P(), k.alias_packed()[..., :n])]
    with torch.cuda.stream(s):
        M.mc_negf_graph_begin(s)
        step(s)
        gr = M.mc_negf_graph_end(s)
    try:
        for rep in range(3):
            tal.fill_(-1)
            out.fill_(float("nan"))
            k.P().fill_(float("nan"))
            k.alias_packed().fill_(-1)
            y = torch.randn(1 << 16, device=DEV, dtype=torch.float64)
            (y * y).sum().item()
            gr.launch(s)
            s.synchronize()
            for i, (x, e) in enumerate(zip((tal, out, k.P(), k.alias_packed()[..., :n]),
                                           eager)):
                assert (x.cpu().numpy() == e).all(), (rep, i)
    finally:
        gr.destroy()
