"""Pins of the sparse-column oracle (oracle/columns.py), CPU only.

It must give the dense oracle's G^r columns and kernel rows on small systems (a different
LAPACK-free route: SuperLU on the sparse E - H - Sigma), and on its own it must satisfy the
spectral row-sum identity A = G Gamma G^+ (Sec. II A) and the clean wire's integer
transmission, so a wrong sign, index or lead block in the sparse assembly fails here.
"""
import numpy as np
import pytest

from oracle import columns as C
from oracle import dense as D
from paper_1805_10164_amd import inputs


def both(W, L, E, g, V, **kw):
    return (D.EnergySolution(E, W, L, 1.0, V, g, **kw),
            C.SparseEnergy(E, W, L, 1.0, V, g, **kw))


CASES = [
    dict(W=1, L=9, E=0.3, eta=0.05, dis=0.0),
    dict(W=3, L=5, E=-1.1, eta=0.1, dis=0.4),
    dict(W=4, L=6, E=2.2, eta="mixed", dis=0.3),
    dict(W=3, L=4, E=0.7, eta=0.2, dis=0.2, lead_model=1, gamma_l=0.8),
]


@pytest.mark.parametrize("c", CASES)
def test_columns_and_rows_equal_dense_oracle(c):
    W, L = c["W"], c["L"]
    N = W * L
    V = inputs.random_sites(N, 7, -c["dis"], c["dis"]) if c["dis"] else np.zeros(N)
    if c["eta"] == "mixed":  # zeros and unequal rates
        g = np.abs(inputs.random_sites(N, 8, -0.2, 0.2))
        g[::5] = 0.0
    else:
        g = np.full(N, c["eta"])
    kw = {k: c[k] for k in ("lead_model", "gamma_l") if k in c}
    d, s = both(W, L, c["E"], g, V, **kw)
    cols = [0, N // 2, N - 1]
    assert np.abs(s.columns(cols) - d.G[:, cols]).max() < 1e-12 * np.abs(d.G).max()
    K = d.transition_kernel()
    for r in range(N + 2):
        row = s.kernel_row(r)
        assert np.abs(row - K[r]).max() < 1e-12 * K[r].sum(), r


def test_probe_rows_sum_to_spectral_function():
    # sum_i gamma_i |G_ij|^2 + <psi|Gamma_L|psi> + <psi|Gamma_R|psi> = A_jj = -2 Im G_jj
    W, L = 5, 7
    N = W * L
    V = inputs.random_sites(N, 9, -0.5, 0.5)
    s = C.SparseEnergy(0.4, W, L, 1.0, V, np.full(N, 0.07))
    for j in (0, 3, N // 2, N - 1):
        Gjj = s.columns([j])[j, 0]
        assert abs(s.kernel_row(j).sum() - (-2.0 * Gjj.imag)) < 1e-12 * abs(Gjj)


@pytest.mark.parametrize("W", [1, 3, 6])
def test_clean_wire_transmission_counts_open_channels(W):
    # No dephasing, no disorder: T_RL = Tr Gamma_R G_{L-1,0} Gamma_L G_{L-1,0}^+ equals the
    # number of transverse modes with |E - eps_m| < 2t.
    L, E = 8, 0.35
    N = W * L
    s = C.SparseEnergy(E, W, L, 1.0, np.zeros(N), np.zeros(N))
    Gc = s.columns(list(range(W)))[D.slice_sites(L - 1, W), :]  # G_{L-1,0}
    T = np.real(np.trace(s.GamR @ Gc @ s.GamL @ Gc.conj().T))
    _, eps = D.transverse_modes(W, 1.0)
    assert abs(T - np.sum(np.abs(E - eps) < 2.0)) < 1e-8


@pytest.mark.parametrize("c", [CASES[0], CASES[1], CASES[3],
                               dict(W=4, L=6, E=-2.6, eta=0.02, dis=0.5)])
def test_effective_transmission_equals_dense_lead_current(c):
    # transmission-form probe solve (this module) against the dense oracle's current into
    # lead R from the lesser Green's function (Eqs. (8), (15))
    W, L = c["W"], c["L"]
    N = W * L
    V = inputs.random_sites(N, 11, -c["dis"], c["dis"]) if c["dis"] else np.zeros(N)
    kw = {k: c[k] for k in ("lead_model", "gamma_l") if k in c}
    d, s = both(W, L, c["E"], np.full(N, c["eta"]), V, **kw)
    assert abs(s.effective_transmission() - d.T_eff) < 1e-11 * abs(d.T_eff)


def test_effective_transmission_rejects_zero_rates():
    s = C.SparseEnergy(0.1, 2, 3, 1.0, np.zeros(6), np.array([0.1, 0, 0.1, 0.1, 0.1, 0.1]))
    with pytest.raises(ValueError):
        s.effective_transmission()
