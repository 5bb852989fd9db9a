"""Rows of more than 4096 outcomes: W = 32 wires (the paper's 32 x 32 blocks) from N = 4160
to the full N = 16000 workload, against the sparse-column oracle (oracle/columns.py).

At N = 4160 and 8320 (the two large-row shapes of the alias build) every energy's DIRECT
T_eff is compared with the oracle's probe solve over all N columns (1e-10 relative), the
walker replays the GPU's own tables bit for bit in the oracle's C walker (N = 4160), and
sampled columns of |G|^2 and sampled alias rows are compared one by one; rows of the maximum
length (N + 2 = 16320 outcomes, a W = 2 wire of 8159 slices) get the same sampled checks, the
bit-for-bit walker replay and the Monte Carlo/DIRECT agreement.  At N = 16000, with
the batch of energies the benchmark builds at once, the oracle computes sampled columns and
kernel rows one by one and the T_eff of one energy from all 16000 columns (1e-10 relative,
about a minute on the host); the other energies' T_eff are checked by the property that
holds at any size: the Monte Carlo current agrees with the DIRECT one within its standard
error.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import columns as C  # noqa: E402
from oracle import walker as OW  # noqa: E402
from paper_1805_10164_amd import inputs  # noqa: E402
from paper_1805_10164_amd import mcnegf as M  # noqa: E402

DEV = "cuda"
SEED = inputs.RNG_SEED


def table_distribution(thr, al):
    """Distribution sampled by an alias row with uint32 thresholds (test-side helper)."""
    n = len(thr)
    keep = thr.astype(np.float64) / 4294967296.0
    p = np.bincount(np.arange(n), weights=keep / n, minlength=n)
    p += np.bincount(al.astype(np.int64), weights=(1.0 - keep) / n, minlength=n)
    return p


def build(wl, energies):
    sysm = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead)
    ws = M.allocate_workspace(sysm, len(energies))
    V = torch.tensor(inputs.onsite(wl), device=DEV)
    g = torch.tensor(inputs.dephasing(wl), device=DEV)
    E = torch.tensor(energies, dtype=torch.float64, device=DEV)
    k = M.mc_negf_build_kernel(sysm, V, g, E, ws)
    k._keep = (V, g, E)
    return k


def oracle_energy(wl, E):
    return C.SparseEnergy(E, wl.W, wl.L, wl.t, inputs.onsite(wl), inputs.dephasing(wl),
                          wl.lead_model, wl.delta_lead, wl.gamma_l)


def check_columns_and_rows(k, e, ora, cols, rows):
    """|G|^2 columns and alias rows of energy e against the sparse oracle."""
    N, n = k.N, k.n_out
    P = k.P()
    ref = np.abs(ora.columns(cols)) ** 2
    for c, j in enumerate(cols):
        got = P[e, :, j].cpu().numpy()
        assert np.abs(got - ref[:, c]).max() <= 1e-10 * ref[:, c].max(), (e, j)
    thr, al = k.alias_rows(e, rows)
    for r_i, r in enumerate(rows):
        assert (al[r_i] >= 0).all() and (al[r_i] < n).all()
        p = table_distribution(thr[r_i], al[r_i])
        K = ora.kernel_row(r)
        assert np.abs(p - K / K.sum()).max() < 4.0 * 2.0 ** -32 + 1e-12, (e, r)


def flags_ok(k):
    bad = M.FLAG_NONFINITE | M.FLAG_SINGULAR | M.FLAG_NOTSPD | M.FLAG_ROWSUM
    return (M.mc_negf_status(k) & bad) == 0


@pytest.mark.parametrize("L,nE", [(130, 2), (260, 1)])
def test_w32_long_rows_match_sparse_oracle(L, nE):
    wl = inputs.SCALE_W32_L500.replace(L=L, n_energies=nE)
    E, w = inputs.energy_grid(-3.1, 2.9, nE)
    k = build(wl, E)
    N = k.N
    assert k.n_out > 4096 * (L // 130)
    wt = torch.tensor(w, device=DEV)
    T = torch.empty(nE, dtype=torch.float64, device=DEV)
    sg = torch.empty_like(T)
    st, I, _ = M.mc_negf_current(k, 1, 0, None, wt, T, sg)
    assert st == M.OK and flags_ok(k)
    rng = np.random.default_rng(L)
    for e in range(nE):
        ora = oracle_energy(wl, E[e])
        Tref = ora.effective_transmission()
        assert abs(T[e].item() - Tref) <= 1e-10 * abs(Tref), (e, T[e].item(), Tref)
        cols = [0, int(rng.integers(1, N - 1)), N - 1]
        rows = sorted({0, int(rng.integers(1, N - 1)), N - 1, N, N + 1})
        check_columns_and_rows(k, e, ora, cols, rows)


def test_w32_l130_walker_replays_long_tables_bit_for_bit():
    # outcome indices above 4095 in the packed entries: the oracle's C walker, given the
    # GPU's tables, must reproduce the GPU walker's tallies exactly
    wl = inputs.SCALE_W32_L500.replace(L=130, n_energies=2, eta=0.05)
    E, _ = inputs.energy_grid(-1.3, 0.7, 2)
    k = build(wl, E)
    thr, al = k.alias_tables()
    nw = 20_000
    for inject in (0, 1):
        tal = torch.zeros((2, M.TALLY_N), dtype=torch.int64, device=DEV)
        M.mc_negf_walk(k, SEED, 3, inject, 500, nw, 1_000_000, tal)
        ref = OW.walk_alias(thr, al, SEED, 3, inject, 500, nw)
        assert (tal.cpu().numpy() == ref).all()
        assert ref[:, 3].sum() > 3 * nw  # walks of several steps visit many rows


def test_rows_of_the_maximum_length():
    # N + 2 = 16320 outcomes, the longest row the alias build holds in one workgroup's LDS
    # (10 bytes per outcome), on a thin wire: W = 2, L = 8159 (N = 16318), two energies in
    # both transverse bands
    wl = inputs.WIRE_W10_L100.replace(W=2, L=8159, n_energies=2, eta=0.1)
    E, w = inputs.energy_grid(-1.5, 0.5, 2)
    k = build(wl, E)
    N, n = k.N, k.n_out
    assert n == 16320
    wt = torch.tensor(w, device=DEV)
    Td = torch.empty(2, dtype=torch.float64, device=DEV)
    sd = torch.empty_like(Td)
    st, I_d, _ = M.mc_negf_current(k, 1, 0, None, wt, Td, sd)
    assert st == M.OK and flags_ok(k)
    rng = np.random.default_rng(16320)
    for e in range(2):
        ora = oracle_energy(wl, E[e])
        cols = [0, int(rng.integers(1, N - 1)), N - 1]
        rows = sorted({0, int(rng.integers(1, N - 1)), N - 1, N, N + 1})
        check_columns_and_rows(k, e, ora, cols, rows)
    # the oracle's C walker replays the GPU walker on the GPU's own tables (alias indices up
    # to 16319 in the packed entries)
    thr, al = k.alias_tables()
    nw = 20_000
    tal = torch.zeros((2, M.TALLY_N), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, SEED, 0, 0, 0, nw, 1_000_000, tal)
    ref = OW.walk_alias(thr, al, SEED, 0, 0, 0, nw)
    assert (tal.cpu().numpy() == ref).all()
    del thr, al
    # Monte Carlo against DIRECT (a property at any size)
    nw = 400_000
    tal.zero_()
    M.mc_negf_walk(k, SEED, 1, 0, 0, nw, 1_000_000, tal)
    T = torch.empty(2, dtype=torch.float64, device=DEV)
    sg = torch.empty_like(T)
    st, I_mc, s_mc = M.mc_negf_current(k, 0, 0, tal, wt, T, sg)
    assert st == M.OK
    assert abs(I_mc - I_d) <= 4.0 * s_mc, (I_mc, I_d, s_mc)
    del k, tal
    torch.cuda.empty_cache()


def test_full_size_w32_l500_batch():
    # N = 16000 (n = 16002 outcomes per row) with the benchmark's batch of energies
    wl = inputs.SCALE_W32_L500
    Eall, wall = inputs.energy_grid(wl.emin, wl.emax, wl.n_energies)
    pick = np.arange(0, wl.n_energies, wl.n_energies // inputs.SCALE_BATCH)
    E, w = Eall[pick], wall[pick]
    nE = len(E)
    assert nE == inputs.SCALE_BATCH
    k = build(wl, E)
    N = k.N
    assert N == 16000
    wt = torch.tensor(w, device=DEV)
    Td = torch.empty(nE, dtype=torch.float64, device=DEV)
    sd = torch.empty_like(Td)
    st, I_d, _ = M.mc_negf_current(k, 1, 0, None, wt, Td, sd)
    assert st == M.OK and flags_ok(k)
    # T_eff of one energy against the oracle's probe solve over all 16000 columns
    ora = oracle_energy(wl, E[1])
    Tref = ora.effective_transmission()
    del ora
    assert abs(Td[1].item() - Tref) <= 1e-10 * abs(Tref), (Td[1].item(), Tref)
    rng = np.random.default_rng(16000)
    for e in (0, nE // 2 + 1):
        ora = oracle_energy(wl, E[e])
        cols = [0, int(rng.integers(1, N - 1)), N - 1]
        rows = sorted({int(rng.integers(0, N)), N - 1, N, N + 1})
        check_columns_and_rows(k, e, ora, cols, rows)
    nw = 1_000_000
    tal = torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, SEED, 0, 0, 0, nw, 1_000_000, tal)
    T = torch.empty(nE, dtype=torch.float64, device=DEV)
    sg = torch.empty_like(T)
    st, I_mc, s_mc = M.mc_negf_current(k, 0, 0, tal, wt, T, sg)
    assert st == M.OK
    assert abs(I_mc - I_d) <= 4.0 * s_mc, (I_mc, I_d, s_mc)
    z = (T - Td).abs() / sg.clamp_min(1e-300)
    assert int((z > 4.0).sum()) <= 1  # per-energy 4-sigma exceedances (32 energies)
    del k, tal
    torch.cuda.empty_cache()  # return the 180 GB workspace before the next test
