"""Inelastic walks (step 7', Sec. II F) on the GPU through the C ABI against the oracle
(oracle/inelastic.py, oracle/walker.c).

- Table: from the oracle's A_jj written into the handle, the GPU's thresholds equal the
  oracle's bit for bit (same FP64 operations in the same order); from the GPU's own A_jj they
  differ by at most one unit of 2^-32.
- Walks: on the oracle's alias and step-7' tables the GPU's tallies and exit-energy histogram
  equal the oracle walker's exactly (integers), for both leads, several line sets, truncated
  walks, a walker range that does not fill the last workgroup, up to 8 lines, and the largest
  energy grid (4096 energies).
- Elastic limit: with the single line at 0 the GPU's inelastic walks are mc_negf_walk's, tally
  for tally, on the GPU's own tables (also at the full wire size).
- Statistics: the GPU's exit distribution and current agree with the exact chain within 5
  sigma (bins) and 4 sigma (current); the energy-resolved current equals the oracle's from the
  same histogram and sums to the current of the tallies.
- The benchmark's configuration (full wire, phonon lines): properties that hold at any size.
- Graph capture: table, walks and spectrum captured once; every replay equals the eager run.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import inelastic as IN  # noqa: E402
from paper_1805_10164_amd import inputs  # noqa: E402
from paper_1805_10164_amd import mcnegf as M  # noqa: E402
from test_gpu_parity import DEV, SEED, case, gpu_build, oracle_solve  # noqa: E402
from test_gpu_walker import oracle_alias_tables  # noqa: E402


def gpu_table(k, offsets, lambdas):
    t = torch.empty(M.mc_negf_energy_table_bytes(k, len(offsets)) // 8, dtype=torch.int64,
                    device=DEV)
    M.mc_negf_energy_table(k, offsets, lambdas, t)
    torch.cuda.synchronize()
    return t


def to_device_table(t):
    return torch.from_numpy(np.ascontiguousarray(t, dtype=np.uint64).view(np.int64)).to(DEV)


def gpu_walk(k, offsets, table, nw, inject=0, begin=0, realization=0, max_steps=1_000_000):
    tal = torch.zeros((k.nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    hist = torch.zeros((2, k.nE, k.nE), dtype=torch.int64, device=DEV)
    M.mc_negf_walk_inelastic(k, offsets, table, SEED, realization, inject, begin, nw, max_steps,
                             tal, hist)
    torch.cuda.synchronize()
    return tal.cpu().numpy(), hist.cpu().numpy()


def host_table(t, k, n_lines):
    return t.cpu().numpy().view(np.uint64).reshape(k.nE, k.N, n_lines)


def test_table_equals_the_oracle_bit_for_bit():
    c = case(W=3, L=4, eta=0.3, disorder=0.3, nE=9, emin=-2.0, emax=1.5)
    k = gpu_build(c)
    sols = oracle_solve(c)
    A = np.array([s.Adiag for s in sols])
    off, lam = [-3, -1, 0, 2, 5], [0.3, 0.7, 1.0, 0.2, 0.05]
    # from the GPU's own A_jj: within one unit of the oracle's thresholds
    own = host_table(gpu_table(k, off, lam), k, 5).astype(np.int64)
    ref = IN.energy_table(A, off, lam)
    assert np.abs(own - ref.astype(np.int64)).max() <= 1
    # from the oracle's A_jj written into the handle: identical
    k.Adiag().copy_(torch.from_numpy(A).to(DEV))
    t = host_table(gpu_table(k, off, lam), k, 5)
    assert np.array_equal(t, ref)
    assert M.mc_negf_status(k) & M.FLAG_NONFINITE == 0


@pytest.mark.parametrize("inject,offsets,lambdas,nw,begin,max_steps", [
    (0, [-1, 0, 1], [0.5, 1.0, 0.5], 30_000, 0, 1_000_000),
    (1, [-1, 0, 1], [0.5, 1.0, 0.5], 30_000, 77, 1_000_000),
    (0, [0, -2, 3], [0.1, 1.0, 0.4], 4_099, 12_345, 1_000_000),   # a ragged last workgroup
    (1, [-4, -3, -2, -1, 1, 2, 3, 4], [1, 2, 3, 4, 4, 3, 2, 1], 20_000, 0, 1_000_000),
    (0, [-1, 0, 1], [1.0, 1.0, 1.0], 20_000, 5, 3),                # truncated walks
])
def test_walks_equal_the_oracle_walker(inject, offsets, lambdas, nw, begin, max_steps):
    c = case(W=3, L=4, eta=0.3, disorder=0.3, nE=10, emin=-1.8, emax=1.6)
    k = gpu_build(c)
    sols = oracle_solve(c)
    thr, al = oracle_alias_tables(sols, k.alias_pitch)
    k.set_alias_tables(thr, al)
    A = np.array([s.Adiag for s in sols])
    et = IN.energy_table(A, offsets, lambdas)
    tal, hist = gpu_walk(k, offsets, to_device_table(et), nw, inject, begin, 3, max_steps)
    rt, rh, bad = IN.walk_alias(thr, al, et, offsets, SEED, 3, inject, begin, nw, max_steps)
    assert not bad
    assert np.array_equal(tal, rt)
    assert np.array_equal(hist, rh)
    off_diag = hist.sum() - sum(hist[r, e, e] for r in (0, 1) for e in range(10))
    assert off_diag > 0                                # the walks do change energy
    if max_steps == 3:
        assert tal[:, 2].sum() > 0
        assert M.mc_negf_status(k) & M.FLAG_TRUNC
    else:
        assert M.mc_negf_status(k) & (M.FLAG_TRUNC | M.FLAG_RANGE) == 0


def test_off_grid_table_entry_ends_the_walk_and_flags_it():
    # a table whose thresholds are all 0 always draws the last line; from the top energy the
    # line +1 leaves the grid: the walker's bounds check ends such walks as truncated
    c = case(W=2, L=3, eta=0.4, disorder=0.2, nE=4, emin=-1.0, emax=1.0)
    k = gpu_build(c)
    et = np.zeros((4, 6, 2), dtype=np.uint64)
    tal, _ = gpu_walk(k, [0, 1], to_device_table(et), 5_000)
    assert tal[:, 2].sum() > 0
    assert M.mc_negf_status(k) & M.FLAG_RANGE
    assert (tal[:, :3].sum(axis=1) == 5_000).all()


@pytest.mark.parametrize("inject", [0, 1])
def test_elastic_line_is_the_elastic_walker(inject):
    c = case(W=4, L=6, eta=0.2, disorder=0.3, nE=6, emin=-2.5, emax=2.0, seed=4)
    k = gpu_build(c)
    t = gpu_table(k, [0], [1.0])
    nw = 100_000
    tal, hist = gpu_walk(k, [0], t, nw, inject, begin=11, realization=2)
    ref = torch.zeros((k.nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, SEED, 2, inject, 11, nw, 1_000_000, ref)
    torch.cuda.synchronize()
    assert np.array_equal(tal, ref.cpu().numpy())
    for e in range(k.nE):
        assert hist[0, e, e] == tal[e, 0] and hist[1, e, e] == tal[e, 1]
    assert hist.sum() == tal[:, :2].sum()


def test_elastic_line_at_the_wire_size():
    # the wire workload (W = 10, L = 100, 256 energies) with the single elastic line: the
    # inelastic walker repeats mc_negf_walk's tallies at every energy
    wl = inputs.WIRE_W10_L100
    c = case(W=wl.W, L=wl.L, eta=wl.eta, disorder=0.0, nE=wl.n_energies, emin=wl.emin,
             emax=wl.emax)
    c["V"] = inputs.onsite(wl)
    k = gpu_build(c)
    t = gpu_table(k, [0], [1.0])
    nw = 20_000
    tal, _ = gpu_walk(k, [0], t, nw)
    ref = torch.zeros((k.nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, SEED, 0, 0, 0, nw, 1_000_000, ref)
    torch.cuda.synchronize()
    assert np.array_equal(tal, ref.cpu().numpy())


def test_wire_table_at_sampled_energies():
    # full-size thresholds at three energies against the oracle's dense A_jj (within 1 unit)
    wl = inputs.WIRE_W10_L100
    c = case(W=wl.W, L=wl.L, eta=wl.eta, disorder=0.0, nE=wl.n_energies, emin=wl.emin,
             emax=wl.emax)
    c["V"] = inputs.onsite(wl)
    k = gpu_build(c)
    off, lam = list(inputs.PHONON_LINES), list(inputs.PHONON_WEIGHTS)
    t = host_table(gpu_table(k, off, lam), k, len(off)).astype(np.int64)
    nE = wl.n_energies
    for e in (0, 101, nE - 1):
        need = sorted({e + d for d in off if 0 <= e + d < nE})
        sols = oracle_solve(c, need)
        A = np.zeros((nE, wl.W * wl.L))
        for j, s in zip(need, sols):
            A[j] = s.Adiag
        A[A == 0] = 1.0  # energies this row does not read
        ref = IN.energy_table(A, off, lam)[e].astype(np.int64)
        assert np.abs(t[e] - ref).max() <= 1


def test_exit_distribution_and_current_match_the_exact_chain():
    c = case(W=2, L=3, eta=0.5, disorder=0.3, nE=8, emin=-1.6, emax=1.4, seed=7)
    k = gpu_build(c)
    sols = oracle_solve(c)
    Ks = np.array([s.transition_kernel() for s in sols])
    A = np.array([s.Adiag for s in sols])
    off, lam = [-2, 0, 1], [0.8, 1.0, 0.4]
    t = gpu_table(k, off, lam)
    nw = 400_000
    tal, hist = gpu_walk(k, off, t, nw)
    B = IN.exit_distribution(Ks, A, off, lam, 0)
    expect = B.transpose(1, 0, 2) * nw
    big = expect >= 400
    assert big.sum() >= 30
    assert (np.abs(hist[big] - expect[big]) <= 5 * np.sqrt(expect[big])).all()
    # current: walkers score c_L(e0) at an exit at R
    w = torch.tensor(c["w"], device=DEV)
    T = torch.empty(k.nE, dtype=torch.float64, device=DEV)
    sg = torch.empty_like(T)
    _, I, sI = M.mc_negf_current(k, 0, 0, torch.from_numpy(tal).to(DEV), w, T, sg)
    cL = np.array([s.trGLA for s in sols])
    I_exact = float(np.sum(c["w"] * cL * B[:, 1, :].sum(axis=1)))
    assert abs(I - I_exact) < 4 * sI
    # energy-resolved current: the oracle's from the same histogram, with the GPU's row totals
    # c_p (only the estimator's arithmetic differs) and with the oracle's; sums to I
    S = torch.empty((2, k.nE), dtype=torch.float64, device=DEV)
    M.mc_negf_spectrum(k, 0, torch.from_numpy(tal).to(DEV), torch.from_numpy(hist).to(DEV), w, S)
    torch.cuda.synchronize()
    Sg = S.cpu().numpy()
    c_gpu = k.lead().cpu().numpy()[:, M.LEAD_CL]
    Sref = IN.spectrum(tal, hist, c_gpu, c["w"], 0)
    assert np.abs(Sg - Sref).max() <= 1e-12 * np.abs(Sref).max()
    Sref = IN.spectrum(tal, hist, cL, c["w"], 0)
    assert np.abs(Sg - Sref).max() <= 1e-10 * np.abs(Sref).max()
    assert Sg[1].sum() == pytest.approx(I, rel=1e-12)
    assert Sg[1][Sg[1] > 0].size > 1                    # exits spread over several energies


def test_inelastic_argument_checks():
    c = case(W=2, L=3, eta=0.2, disorder=0.3, nE=3, emin=-1.0, emax=1.0)
    k = gpu_build(c)
    t = gpu_table(k, [-1, 0, 1], [1.0, 1.0, 1.0])
    with pytest.raises(M.McnegfError) as ei:
        M.mc_negf_walk_inelastic(k, [-1, 0, 3], t, SEED, 0, 0, 0, 10, 100,
                                 torch.zeros((3, M.TALLY_N), dtype=torch.int64, device=DEV),
                                 torch.zeros((2, 3, 3), dtype=torch.int64, device=DEV))
    assert ei.value.code == M.EINVAL
    small = torch.empty(4, dtype=torch.int64, device=DEV)
    with pytest.raises(M.McnegfError) as ei:
        M.mc_negf_energy_table(k, [-1, 0, 1], [1.0, 1.0, 1.0], small)
    assert ei.value.code == M.EWS


def test_wire_walks_with_the_phonon_lines():
    # the benchmark's configuration (W = 10, L = 100, 256 energies, lines 0 and -/+8) with
    # 1e5 walkers per energy, checked by properties that hold at any size: every walker is
    # tallied once, every exit is in the histogram, exits differ from their injection energy
    # by multiples of the line spacing only, the energy-resolved current sums to the current,
    # and emission (weight 0.563) outweighs absorption (0.063)
    wl = inputs.WIRE_W10_L100
    c = case(W=wl.W, L=wl.L, eta=wl.eta, disorder=0.0, nE=wl.n_energies, emin=wl.emin,
             emax=wl.emax)
    c["V"] = inputs.onsite(wl)
    k = gpu_build(c)
    off, lam = list(inputs.PHONON_LINES), [float(x) for x in inputs.PHONON_WEIGHTS]
    t = gpu_table(k, off, lam)
    nw = 100_000
    tal, hist = gpu_walk(k, off, t, nw)
    assert (tal[:, :3].sum(axis=1) == nw).all() and tal[:, 2].sum() == 0
    assert (hist.sum(axis=2) == tal[:, :2].T).all()
    de = np.subtract.outer(np.arange(wl.n_energies), np.arange(wl.n_energies)).T  # e - e0
    assert hist[:, de % inputs.PHONON_STEPS != 0].sum() == 0
    assert hist[:, de < 0].sum() > 5 * hist[:, de > 0].sum() > 0
    assert M.mc_negf_status(k) & (M.FLAG_TRUNC | M.FLAG_RANGE | M.FLAG_NONFINITE) == 0
    w = torch.tensor(c["w"], device=DEV)
    T = torch.empty(k.nE, dtype=torch.float64, device=DEV)
    sg = torch.empty_like(T)
    _, I, sI = M.mc_negf_current(k, 0, 0, torch.from_numpy(tal).to(DEV), w, T, sg)
    S = torch.empty((2, k.nE), dtype=torch.float64, device=DEV)
    M.mc_negf_spectrum(k, 0, torch.from_numpy(tal).to(DEV), torch.from_numpy(hist).to(DEV), w, S)
    torch.cuda.synchronize()
    assert float(S[1].sum()) == pytest.approx(I, rel=1e-12)
    assert sI < 0.01 * I


def test_the_largest_energy_grid_equals_the_oracle_walker():
    # nE = 4096, the most energies the walker's exit-energy histogram holds in LDS (2 nE
    # counters), on a two-site chain: tallies and the full histogram equal the oracle walker's
    nE = 4096
    c = case(W=1, L=2, eta=0.5, disorder=0.2, nE=nE, emin=-1.9, emax=1.9)
    k = gpu_build(c)
    sols = oracle_solve(c)
    thr, al = oracle_alias_tables(sols, k.alias_pitch)
    k.set_alias_tables(thr, al)
    A = np.array([s.Adiag for s in sols])
    offsets, lambdas = [-8, 0, 8], [0.5, 1.0, 0.5]
    et = IN.energy_table(A, offsets, lambdas)
    nw = 300
    tal, hist = gpu_walk(k, offsets, to_device_table(et), nw, 1, 9, 4)
    rt, rh, bad = IN.walk_alias(thr, al, et, offsets, SEED, 4, 1, 9, nw)
    assert not bad
    assert np.array_equal(tal, rt)
    assert np.array_equal(hist, rh)
    assert (tal[:, :3].sum(axis=1) == nw).all()
    assert hist[:, :, :8].sum() > 0 and hist[:, :, -8:].sum() > 0   # walks reach both ends


def test_graph_replays_match_eager():
    # Capture: the step-7' table, zeroed tallies and histogram (fill kernels, no memset node),
    # the inelastic walks and the energy-resolved current.  Replay three times with eager
    # work and synchronisations between replays; every replay must equal the eager run.
    c = case(W=3, L=4, eta=0.3, disorder=0.3, nE=10, emin=-1.8, emax=1.6)
    k = gpu_build(c)
    off, lam = [-1, 0, 1], [0.5, 1.0, 0.5]
    table = torch.empty(M.mc_negf_energy_table_bytes(k, 3) // 8, dtype=torch.int64, device=DEV)
    tal = torch.zeros((k.nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    hist = torch.zeros((2, k.nE, k.nE), dtype=torch.int64, device=DEV)
    S = torch.empty((2, k.nE), dtype=torch.float64, device=DEV)
    wts = torch.tensor(c["w"], device=DEV)

    def step(stream):
        tal.zero_()
        hist.zero_()
        M.mc_negf_energy_table(k, off, lam, table, stream)
        M.mc_negf_walk_inelastic(k, off, table, SEED, 1, 0, 0, 20_000, 1_000_000, tal, hist,
                                 stream)
        M.mc_negf_spectrum(k, 0, tal, hist, wts, S, stream)

    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        step(s)
    s.synchronize()
    eager = [x.cpu().numpy().copy() for x in (table, tal, hist, S)]
    assert eager[2].sum() == 20_000 * k.nE - eager[1][:, 2].sum()
    with torch.cuda.stream(s):
        M.mc_negf_graph_begin(s)
        step(s)
        g = M.mc_negf_graph_end(s)
    try:
        for rep in range(3):
            for x in (table, tal, hist):
                x.fill_(-1)
            S.fill_(float("nan"))
            y = torch.randn(1 << 16, device=DEV, dtype=torch.float64)
            (y * y).sum().item()
            g.launch(s)
            s.synchronize()
            for x, e in zip((table, tal, hist, S), eager):
                assert (x.cpu().numpy() == e).all(), rep
    finally:
        g.destroy()
