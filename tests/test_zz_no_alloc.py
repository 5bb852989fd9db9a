"""The allocation-free energy-sampled walk (mc_negf_walk_sampled_noalloc) against the entry
point with a caller-owned scratch buffer (mc_negf_walk_sampled): the same tallies bit for bit,
on two calls in a row (the second with fewer energies and walkers, so the fixed scratch holds
the first call's leftovers), and a size beyond the fixed scratch is refused."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_1805_10164_amd import inputs  # noqa: E402
from paper_1805_10164_amd import mcnegf as M  # noqa: E402

DEV = "cuda"


def build(W, L, nE, eta, seed):
    sysm = M.make_system(W, L)
    E, w = inputs.energy_grid(-2.6, 2.6, nE)
    V = torch.tensor(inputs.random_sites(W * L, seed, -0.3, 0.3), device=DEV)
    g = torch.full((W * L,), eta, dtype=torch.float64, device=DEV)
    ws = M.allocate_workspace(sysm, nE)
    k = M.mc_negf_build_kernel(sysm, V, g, torch.tensor(E, device=DEV), ws)
    k._keep = (V,)
    # uneven weights, one of them zero
    wts = np.linspace(0.5, 1.5, nE) * w
    wts[nE // 3] = 0.0
    return k, torch.tensor(wts, device=DEV)


def both(k, wts, seed, real, lead, wbegin, n):
    nE = k.nE
    ref = torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    scratch = torch.empty(M.mc_negf_walk_sampled_bytes(k, n), dtype=torch.uint8, device=DEV)
    M.mc_negf_walk_sampled(k, seed, real, lead, wbegin, n, 1_000_000, wts, ref, scratch)
    got = torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=DEV)
    M.mc_negf_walk_sampled_noalloc(k, seed, real, lead, wbegin, n, 1_000_000, wts, got)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def test_noalloc_sampled_walk_equals_the_scratch_entry_point_twice():
    k1, w1 = build(4, 9, 40, 0.1, 21)
    ref, got = both(k1, w1, 0xABCDEF, 2, 0, 1000, 300_000)
    assert ref[:, :3].sum() == 300_000 and ref[40 // 3].sum() == 0
    assert (got == ref).all()
    # second call: fewer energies, fewer walkers, the other lead
    k2, w2 = build(3, 5, 7, 0.2, 22)
    ref, got = both(k2, w2, 77, 0, 1, 5, 20_001)
    assert ref[:, :3].sum() == 20_001
    assert (got == ref).all()


def test_noalloc_refuses_sizes_beyond_the_fixed_scratch():
    k, w = build(2, 3, 4, 0.1, 23)
    n = 1 << 24  # 8 bytes per walker alone exceed the 64 MiB scratch
    assert M.mc_negf_walk_sampled_bytes(k, n) > M.STATIC_SCRATCH_BYTES
    t = torch.zeros((4, M.TALLY_N), dtype=torch.int64, device=DEV)
    with pytest.raises(M.McnegfError) as ei:
        M.mc_negf_walk_sampled_noalloc(k, 1, 0, 0, 0, n, 1_000_000, w, t)
    assert ei.value.code == M.EWS
    torch.cuda.synchronize()
    assert (t == 0).all()
