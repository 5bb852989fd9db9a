"""Importance-sampled walks (Sec. V A, "Improved estimator") on the GPU, through the C ABI,
against the oracle (oracle/weighted.py).

- The modified tables sample p'_ij = p_ij b_j / rho_i within the alias format's resolution of
  the oracle's rows, and rho matches the oracle's at 1e-12; with b = 1 they are the kernel's
  own tables bit for bit and rho is exactly 1.
- On tables and rho the oracle built, the GPU's weighted walks give the oracle walker's
  integer counts bit for bit and its score sums to 1e-12 (summation order only).
- With b = the oracle's exact absorption probabilities every walk scores T_eff: the GPU's
  estimate is the oracle's DIRECT T_eff at 1e-9 with a standard error below 1e-7 of it.
- With a ramp bias the estimate is unbiased (within 4 sigma of DIRECT) and its sigma is well
  below the plain walk's at the same walker count.
- Graph capture: modified tables and weighted walks captured once; every replay equals the
  eager run.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import dense as D  # noqa: E402
from oracle import weighted as WT  # noqa: E402
from paper_1805_10164_amd import mcnegf as M  # noqa: E402
from test_gpu_parity import DEV, SEED, case, gpu_build, oracle_solve, rel  # noqa: E402
from test_gpu_parity import table_distribution  # noqa: E402


def tables_for(k, bias):
    buf = torch.empty(M.mc_negf_weighted_tables_bytes(k), dtype=torch.uint8, device=DEV)
    b = torch.tensor(np.asarray(bias, dtype=np.float64), device=DEV)
    M.mc_negf_weighted_tables(k, b, buf)
    torch.cuda.synchronize()
    return buf, b


def walk(k, buf, b, nw, inject=0, begin=0, realization=0, max_steps=1_000_000):
    tal = torch.zeros((k.nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    ws = torch.zeros((k.nE, 2), dtype=torch.float64, device=DEV)
    scratch = torch.empty(max(M.mc_negf_walk_weighted_bytes(k, nw), 256), dtype=torch.uint8,
                          device=DEV)
    M.mc_negf_walk_weighted(k, buf, b, SEED, realization, inject, begin, nw, max_steps, tal, ws,
                            scratch)
    torch.cuda.synchronize()
    return tal, ws


def unpack(packed, low):
    packed = packed.cpu().numpy().view(np.uint32)
    low = low.cpu().numpy().view(np.uint16).astype(np.uint32)
    return (packed & np.uint32(0xFFFF0000)) | low, (packed & np.uint32(0xFFFF)).astype(np.int32)


def pack_into(buf, k, thr, al, rho):
    packed, low, r = M.weighted_tables_views(k, buf)
    thr = np.asarray(thr, dtype=np.uint32)
    al = np.asarray(al, dtype=np.uint32)
    packed.copy_(torch.from_numpy(((thr & np.uint32(0xFFFF0000)) |
                                   (al & np.uint32(0xFFFF))).view(np.int32)).to(DEV))
    low.copy_(torch.from_numpy((thr & np.uint32(0xFFFF)).astype(np.uint16).view(np.int16)).to(DEV))
    r.copy_(torch.from_numpy(np.ascontiguousarray(rho, dtype=np.float64)).to(DEV))


@pytest.mark.parametrize("W,L,nE", [(3, 4, 3), (16, 100, 2)])
def test_modified_tables_and_rho_against_the_oracle(W, L, nE):
    c = case(W=W, L=L, eta=0.1, disorder=0.3, nE=nE, emin=-2.0, emax=1.5)
    k = gpu_build(c)
    sols = oracle_solve(c)
    n = k.n_out
    bias = np.stack([WT.ramp_bias(W, L, 0, a=3.0, floor_p=0.01) * (1.0 + 0.1 * e)
                     for e in range(nE)])
    buf, b = tables_for(k, bias)
    assert M.mc_negf_status(k) == 0
    packed, low, rho = M.weighted_tables_views(k, buf)
    thr_all, al_all = unpack(packed, low)
    rng = np.random.default_rng(3)
    for e, s in enumerate(sols):
        K = s.transition_kernel()
        rho_ref = WT.rho(K, bias[e])
        assert rel(rho[e].cpu().numpy(), rho_ref) < 1e-12
        Kb = WT.modified_rows(K, bias[e])
        rows = sorted(set([0, n - 1, n - 2, n - 3] + list(rng.integers(0, n, 6))))
        for r in rows:
            thr, al = thr_all[e, r, :n], al_all[e, r, :n]
            assert (al < n).all()
            p = table_distribution(thr, al)
            ref = Kb[r] / Kb[r].sum()
            assert np.abs(p - ref).max() < 4.0 * 2.0 ** -32 + 1e-12, (e, r)


def test_unit_bias_gives_the_kernels_own_tables_and_the_plain_walk():
    c = case(W=4, L=7, eta=0.2, disorder=0.3, nE=3, emin=-1.7, emax=1.1)
    k = gpu_build(c)
    n = k.n_out
    buf, b = tables_for(k, np.ones((3, n)))
    packed, low, rho = M.weighted_tables_views(k, buf)
    assert torch.equal(packed[:, :, :n], k.alias_packed()[:, :, :n])
    assert torch.equal(low[:, :, :n], k.alias_low()[:, :, :n])
    assert bool((rho == 1.0).all())
    for inject in (0, 1):
        tal, ws = walk(k, buf, b, 30_000, inject=inject, begin=77)
        plain = torch.zeros_like(tal)
        M.mc_negf_walk(k, SEED, 0, inject, 77, 30_000, 1_000_000, plain)
        assert torch.equal(tal, plain)
        hits = plain[:, 1 - inject].double()
        assert torch.equal(ws[:, 0], hits) and torch.equal(ws[:, 1], hits)


@pytest.mark.parametrize("inject,max_steps", [(0, 1_000_000), (1, 1_000_000), (0, 3)])
def test_weighted_walk_replays_the_oracle_walker(inject, max_steps):
    # tables and rho from the oracle, handed to the GPU walker: identical paths and counts,
    # score sums equal up to summation order
    c = case(W=3, L=5, eta=0.25, disorder=0.3, nE=3, emin=-1.5, emax=1.5)
    k = gpu_build(c)
    sols = oracle_solve(c)
    n = k.n_out
    pitch = k.alias_pitch
    bias = np.stack([WT.ramp_bias(3, 5, inject, a=2.0, floor_p=0.05) for _ in range(3)])
    thr = np.zeros((3, n, pitch), np.uint32)
    al = np.zeros((3, n, pitch), np.int32)
    rho = np.zeros((3, n))
    for e, s in enumerate(sols):
        K = s.transition_kernel()
        Kb = WT.modified_rows(K, bias[e])
        rho[e] = WT.rho(K, bias[e])
        for r in range(n):
            thr[e, r, :n], al[e, r, :n] = D.alias_vose(Kb[r])
    buf = torch.empty(M.mc_negf_weighted_tables_bytes(k), dtype=torch.uint8, device=DEV)
    pack_into(buf, k, thr, al, rho)
    b = torch.tensor(bias, device=DEV)
    nw = 40_000
    tal, ws = walk(k, buf, b, nw, inject=inject, begin=1234, realization=5, max_steps=max_steps)
    ref_t, ref_w = WT.walk_weighted_alias(thr, al, rho, bias, SEED, 5, inject, 1234, nw,
                                          max_steps=max_steps)
    assert (tal.cpu().numpy() == ref_t).all()
    assert rel(ws.cpu().numpy(), ref_w) < 1e-12
    if max_steps == 3:
        assert ref_t[:, 2].sum() > 0


def test_exact_absorption_bias_has_zero_variance():
    c = case(W=4, L=10, eta=0.15, disorder=0.3, nE=3, emin=-2.2, emax=1.8)
    k = gpu_build(c)
    sols = oracle_solve(c)
    n = k.n_out
    N = n - 2
    bias = np.zeros((3, n))
    for e, s in enumerate(sols):
        h = D.absorption_probabilities(s.transition_kernel())
        bias[e] = h
        bias[e, N] = 0.0
        bias[e, N + 1] = 1.0
    buf, b = tables_for(k, bias)
    tal, ws = walk(k, buf, b, 20_000)
    t = tal.cpu().numpy()
    assert (t[:, 0] == 0).all() and (t[:, 2] == 0).all()
    w = torch.tensor(c["w"], device=DEV)
    T = torch.empty(3, dtype=torch.float64, device=DEV)
    sg = torch.empty_like(T)
    st, I, sI = M.mc_negf_current_weighted(k, 0, tal, ws, w, T, sg)
    assert st == M.OK
    Tref = np.array([s.T_eff for s in sols])
    assert rel(T.cpu().numpy(), Tref) < 1e-9
    assert (sg.cpu().numpy() < 1e-7 * Tref).all()
    assert abs(I - D.current(sols, c["w"])) < 1e-9 * abs(I)


def test_ramp_bias_is_unbiased_and_reduces_the_variance():
    c = case(W=6, L=40, eta=0.1, disorder=0.3, nE=4, emin=-2.0, emax=1.0)
    k = gpu_build(c)
    n = k.n_out
    bias = np.tile(WT.ramp_bias(6, 40, 0, a=5.0, floor_p=1e-3), (4, 1))
    buf, b = tables_for(k, bias)
    nw = 200_000
    tal, ws = walk(k, buf, b, nw)
    w = torch.tensor(c["w"], device=DEV)
    T = torch.empty(4, dtype=torch.float64, device=DEV)
    sg = torch.empty_like(T)
    st, I_w, s_w = M.mc_negf_current_weighted(k, 0, tal, ws, w, T, sg)
    assert st == M.OK
    # the same estimator in the oracle, from the GPU's sums
    lead = k.lead().cpu().numpy()
    T_o, sg_o, I_o, sI_o = WT.weighted_current(tal.cpu().numpy(), ws.cpu().numpy(),
                                              lead[:, M.LEAD_CL], c["w"])
    assert rel(T.cpu().numpy(), T_o) < 1e-12 and rel(sg.cpu().numpy(), sg_o) < 1e-12
    assert I_w == pytest.approx(I_o, rel=1e-12) and s_w == pytest.approx(sI_o, rel=1e-12)
    Td = torch.empty_like(T)
    _, I_d, _ = M.mc_negf_current(k, 1, 0, None, w, Td, sg)
    assert abs(I_w - I_d) < 4 * s_w
    plain = torch.zeros_like(tal)
    M.mc_negf_walk(k, SEED, 0, 0, 0, nw, 1_000_000, plain)
    _, I_p, s_p = M.mc_negf_current(k, 0, 0, plain, w, T, sg)
    assert s_w < 0.5 * s_p


def test_weighted_sums_are_deterministic_and_argument_checks():
    c = case(W=3, L=6, eta=0.2, disorder=0.3, nE=2, emin=-1.0, emax=1.0)
    k = gpu_build(c)
    n = k.n_out
    bias = np.tile(WT.ramp_bias(3, 6, 0, a=2.0, floor_p=0.1), (2, 1))
    buf, b = tables_for(k, bias)
    t1, w1 = walk(k, buf, b, 70_001)
    t2, w2 = walk(k, buf, b, 70_001)
    assert torch.equal(t1, t2) and torch.equal(w1, w2)
    # a short table buffer, a misaligned scratch and a range ending at 2^32 are refused
    tal = torch.zeros((2, M.TALLY_N), dtype=torch.int64, device=DEV)
    ws = torch.zeros((2, 2), dtype=torch.float64, device=DEV)
    scratch = torch.empty(M.mc_negf_walk_weighted_bytes(k, 1000) + 512, dtype=torch.uint8,
                          device=DEV)
    with pytest.raises(M.McnegfError) as ei:
        M.mc_negf_walk_weighted(k, buf[:1024], b, SEED, 0, 0, 0, 1000, 100, tal, ws, scratch)
    assert ei.value.code == M.EWS
    with pytest.raises(M.McnegfError) as ei:
        M.mc_negf_walk_weighted(k, buf, b, SEED, 0, 0, 0, 1000, 100, tal, ws, scratch[8:])
    assert ei.value.code == M.EWS
    with pytest.raises(M.McnegfError) as ei:
        M.mc_negf_walk_weighted(k, buf, b, SEED, 0, 0, 2 ** 32 - 10, 10, 100, tal, ws, scratch)
    assert ei.value.code == M.EINVAL
    # a negative bias entry is flagged
    bad = bias.copy()
    bad[1, 3] = -1.0
    tables_for(k, bad)
    assert M.mc_negf_status(k) & M.FLAG_NONFINITE


def test_modified_tables_from_a_kernel_without_its_own_tables():
    # a MCNEGF_BUILD_NO_ALIAS kernel has the rows' ingredients: its modified tables, rho and
    # c_p equal those of the full build bit for bit
    c = case(W=5, L=6, eta=0.15, disorder=0.3, nE=3, emin=-2.0, emax=2.0)
    k = gpu_build(c)
    s0 = M.make_system(5, 6, 1.0, 0, 0.0, 1e-10, M.BUILD_NO_ALIAS)
    ws0 = M.allocate_workspace(s0, 3)
    V = torch.tensor(c["V"], dtype=torch.float64, device=DEV)
    g = torch.tensor(c["g"], dtype=torch.float64, device=DEV)
    E = torch.tensor(c["E"], dtype=torch.float64, device=DEV)
    k0 = M.mc_negf_build_kernel(s0, V, g, E, ws0)
    bias = np.tile(WT.ramp_bias(5, 6, 1, a=2.0, floor_p=0.0), (3, 1))
    buf, b = tables_for(k, bias)
    buf0, _ = tables_for(k0, bias)
    assert torch.equal(buf, buf0)
    assert torch.equal(k.lead()[:, M.LEAD_CL:M.LEAD_CR + 1], k0.lead()[:, M.LEAD_CL:M.LEAD_CR + 1])
    tal, ws = walk(k0, buf0, b, 20_000, inject=1)
    t2, w2 = walk(k, buf, b, 20_000, inject=1)
    assert torch.equal(tal, t2) and torch.equal(ws, w2)


def test_graph_replays_match_eager():
    # Capture: the modified tables, zeroed counts and score sums (fill kernels, no memset node)
    # and the importance-sampled walks.  Replay three times with eager work and
    # synchronisations between replays; every replay must equal the eager run.
    W, L, nE = 3, 4, 4
    c = case(W=W, L=L, eta=0.3, disorder=0.3, nE=nE, emin=-1.5, emax=1.5)
    k = gpu_build(c)
    bias = np.stack([WT.ramp_bias(W, L, 0, a=3.0, floor_p=0.01) for _ in range(nE)])
    b = torch.tensor(bias, device=DEV)
    buf = torch.empty(M.mc_negf_weighted_tables_bytes(k), dtype=torch.uint8, device=DEV)
    nw = 20_000
    tal = torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    wsum = torch.zeros((nE, 2), dtype=torch.float64, device=DEV)
    scratch = torch.empty(max(M.mc_negf_walk_weighted_bytes(k, nw), 256), dtype=torch.uint8,
                          device=DEV)

    def step(stream):
        tal.zero_()
        wsum.zero_()
        M.mc_negf_weighted_tables(k, b, buf, stream)
        M.mc_negf_walk_weighted(k, buf, b, SEED, 0, 0, 0, nw, 1_000_000, tal, wsum, scratch,
                                stream)

    def written():
        # what the build writes: the entries of the n outcomes of every row, and rho (the
        # pitch padding and alignment gaps of the buffer are never written)
        packed, low, rho = M.weighted_tables_views(k, buf)
        n = k.n_out
        return [packed[..., :n].cpu().numpy().copy(), low[..., :n].cpu().numpy().copy(),
                rho.cpu().numpy().copy(), tal.cpu().numpy().copy(), wsum.cpu().numpy().copy()]

    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        step(s)
    s.synchronize()
    eager = written()
    assert eager[3][:, :3].sum() == nw * nE
    with torch.cuda.stream(s):
        M.mc_negf_graph_begin(s)
        step(s)
        g = M.mc_negf_graph_end(s)
    try:
        for rep in range(3):
            buf.fill_(0xAB)
            tal.fill_(-1)
            wsum.fill_(float("nan"))
            y = torch.randn(1 << 16, device=DEV, dtype=torch.float64)
            (y * y).sum().item()
            g.launch(s)
            s.synchronize()
            for i, (x, e) in enumerate(zip(written(), eager)):
                assert (x == e).all(), (rep, i)
    finally:
        g.destroy()
