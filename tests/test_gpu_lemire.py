"""The redraw branch of the bucket sampler on the GPU, bit for bit against the oracle walker.

A bucket word is rejected with probability (2^32 mod n) / 2^32 < 4e-6 per step, so ordinary
replays never reach the redraw branch.  tests/golden/lemire_redraws.txt lists walkers whose
injection draw is rejected once, or at least twice, found by brute force with the oracle's
Philox (tests/golden/make_lemire_redraws.py).  Each is walked alone on tables built so that
its step count reveals the injection bucket: the injection rows keep every bucket, and probe
j moves to j - 1 with certainty (probe 0 to lead R), so a walk injected into probe c takes
c + 2 steps.  The per-kernel, batched, energy-sampled, counting and inelastic (single elastic
line) walkers must give the oracle's tallies, which must show the listed bucket.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import walker as OW  # noqa: E402
from paper_1805_10164_amd import mcnegf as M  # noqa: E402

DEV = "cuda"
HERE = os.path.dirname(os.path.abspath(__file__))
SHAPES = {16138: (8, 2017), 1002: (10, 100)}  # n_out -> (W, L)


def golden():
    rows = []
    with open(os.path.join(HERE, "golden", "lemire_redraws.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append(tuple(int(x) for x in line.split()))
    return rows


def chain_down_tables(n, pitch):
    """thr/alias [1][n][pitch]: injection rows N, N + 1 keep every bucket; probe j goes to
    j - 1 (probe 0 to lead R = N + 1) whatever the bucket."""
    N = n - 2
    thr = np.zeros((1, n, pitch), np.uint32)
    al = np.zeros((1, n, pitch), np.int32)
    al[0, 1:N, :] = np.arange(0, N - 1, dtype=np.int32)[:, None]
    al[0, 0, :] = N + 1
    thr[0, N:, :n] = 0xFFFFFFFF
    al[0, N:, :n] = np.arange(n, dtype=np.int32)[None, :]
    return thr, al


@pytest.fixture(scope="module")
def built():
    out = {}
    for n, (W, L) in SHAPES.items():
        sysm = M.make_system(W, L, flags=M.BUILD_NO_DIRECT)
        ws = M.allocate_workspace(sysm, 1)
        V = torch.zeros(W * L, dtype=torch.float64, device=DEV)
        g = torch.full((W * L,), 0.05, dtype=torch.float64, device=DEV)
        E = torch.tensor([0.3], dtype=torch.float64, device=DEV)
        k = M.mc_negf_build_kernel(sysm, V, g, E, ws)
        k._keep = (V,)
        thr, al = chain_down_tables(n, k.alias_pitch)
        k.set_alias_tables(thr, al)
        torch.cuda.synchronize()
        out[n] = (k, thr, al)
    return out


def expected_tally(n, bucket):
    N = n - 2
    if bucket == N:
        return [1, 0, 0, 1, 1]
    if bucket == N + 1:
        return [0, 1, 0, 1, 1]
    s = bucket + 2
    return [0, 1, 0, s, s * s]


def test_golden_file_has_single_and_double_redraws():
    rows = golden()
    assert any(r[5] == 1 for r in rows if r[0] == 1002)
    assert any(r[5] == 1 for r in rows if r[0] == 16138)
    assert any(r[5] >= 2 for r in rows)
    assert {r[3] for r in rows} == {0, 1}


@pytest.mark.parametrize("row", golden(), ids=lambda r: f"n{r[0]}_w{r[4]}_r{r[5]}")
def test_redraw_walker_bit_exact(built, row):
    n, seed, real, lead, w, redraws, bucket = row
    k, thr, al = built[n]
    ref = OW.walk_alias(thr, al, seed, real, lead, w, 1)
    assert ref[0].tolist() == expected_tally(n, bucket)
    # per-kernel walker
    tal = torch.zeros((1, M.TALLY_N), dtype=torch.int64, device=DEV)
    M.mc_negf_walk(k, seed, real, lead, w, 1, 1_000_000, tal)
    torch.cuda.synchronize()
    assert (tal.cpu().numpy() == ref).all()
    # batched walker, two launch shapes
    for cfg in (None, M.walk_config(slots=1, wg_size=64, groups=1, chunk=1)):
        tb = torch.zeros((1, M.TALLY_N), dtype=torch.int64, device=DEV)
        b = M.mc_negf_batch_prepare([k], [real], lead, [tb])
        M.mc_negf_walk_batch(b, seed, w, 1, 1_000_000, cfg)
        torch.cuda.synchronize()
        assert (tb.cpu().numpy() == ref).all()
    # energy-sampled walker (one energy: every walker draws it)
    ts = torch.zeros((1, M.TALLY_N), dtype=torch.int64, device=DEV)
    wts = torch.ones(1, dtype=torch.float64, device=DEV)
    scratch = torch.empty(M.mc_negf_walk_sampled_bytes(k, 1), dtype=torch.uint8, device=DEV)
    M.mc_negf_walk_sampled(k, seed, real, lead, w, 1, 1_000_000, wts, ts, scratch)
    torch.cuda.synchronize()
    assert (ts.cpu().numpy() == ref).all()
    # inelastic walker with the single elastic line (its table is never read); at n = 1002 the
    # injection row is staged in LDS, at n = 16138 it is read from the global table
    ti = torch.zeros((1, M.TALLY_N), dtype=torch.int64, device=DEV)
    hist = torch.zeros((2, 1, 1), dtype=torch.int64, device=DEV)
    et = torch.full((n - 2,), 2 ** 32, dtype=torch.int64, device=DEV)
    M.mc_negf_walk_inelastic(k, [0], et, seed, real, lead, w, 1, 1_000_000, ti, hist)
    torch.cuda.synchronize()
    assert (ti.cpu().numpy() == ref).all()
    assert hist.cpu().numpy()[:, 0, 0].tolist() == ref[0, :2].tolist()
    # counting walker (score-function gradient): same tallies; the walk to q is counted
    if n == 1002:
        tc = torch.zeros((1, M.TALLY_N), dtype=torch.int64, device=DEV)
        cnt = torch.zeros(n * n, dtype=torch.int32, device=DEV)
        M.mc_negf_walk_counts(k, seed, real, lead, w, 1, 1_000_000, cnt, tc)
        torch.cuda.synchronize()
        assert (tc.cpu().numpy() == ref).all()
        q_hits = ref[0, 1 - lead]
        assert int(cnt.sum()) == (ref[0, 3] if q_hits else 0)


def test_redraw_walkers_among_neighbours(built):
    # the listed walkers of the wire-sized table inside a range of 4096 walkers each, so the
    # redraw runs in a wavefront whose other lanes take the ordinary path
    n = 1002
    k, thr, al = built[n]
    for n_, seed, real, lead, w, _, _ in golden():
        if n_ != n:
            continue
        lo = max(0, w - 2048)
        ref = OW.walk_alias(thr, al, seed, real, lead, lo, 4096)
        tal = torch.zeros((1, M.TALLY_N), dtype=torch.int64, device=DEV)
        M.mc_negf_walk(k, seed, real, lead, lo, 4096, 1_000_000, tal)
        torch.cuda.synchronize()
        assert (tal.cpu().numpy() == ref).all()
