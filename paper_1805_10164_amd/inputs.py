"""Seeded synthetic workloads shared by the HIP path's callers and the oracle's tests.

This module holds only workload definitions and seeded random inputs (onsite disorder,
per-site dephasing rates) and the energy points and weights of a workload's window, which
the library takes as inputs.  It contains none of the method's arithmetic: no Green's
functions, no transmissions, no walks, no sums over energies.

The workloads stand in for the paper's CdTe nanowires (Sec. IV: two-by-two unit-cell
cross-section, 32x32 Hamiltonian blocks, lengths of tens of unit cells, dephasing rates of a
few percent of the band scale).  The CdTe tight-binding parameters are not available, so a
square-lattice tight-binding wire of width W and length L with hopping t stands in, with
uniform Anderson disorder and a site-diagonal dephasing rate eta (Sec. III A: constant
lifetime, sigma_i = -(i/2) gamma_i).
"""
from __future__ import annotations

import dataclasses

import numpy as np

RNG_SEED = 180510164          # key of the walkers' counter-based generator
DISORDER_SEED_BASE = 1805     # disorder realization r uses seed DISORDER_SEED_BASE + r


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic transport problem: a W x L wire between two clean leads."""
    name: str
    W: int                    # sites per slice
    L: int                    # slices
    t: float = 1.0            # hopping (H_ij = -t between nearest neighbours)
    eta: float = 0.05         # dephasing rate gamma_i on every site
    disorder: float = 0.0     # onsite V_i ~ U[-disorder, disorder] (times t)
    emin: float = -1.9
    emax: float = 1.9
    n_energies: int = 64
    walkers_per_energy: int = 100_000
    lead_model: int = 0       # 0 clean semi-infinite leads, 1 wide-band leads
    gamma_l: float = 0.0      # wide-band coupling (lead_model 1)
    delta_lead: float = 1e-10 # regulator inside the leads, z = E + i delta_lead (times t)
    realization: int = 0

    @property
    def N(self) -> int:
        return self.W * self.L

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# 1D chain, N = 50 sites, eta = 0.05 t, 64 energies in [-1.9 t, 1.9 t], 1e5 walkers / energy.
CHAIN50 = Workload(name="chain_N50_eta0.05", W=1, L=50, eta=0.05, emin=-1.9, emax=1.9,
                   n_energies=64, walkers_per_energy=100_000)

# 2D wire W = 10, L = 100 (N = 1000), disorder U[-0.25 t, 0.25 t], 256 energies in
# [-3.5 t, 3.5 t], 1e6 walkers / energy; eta in {0.01, 0.05, 0.1} t.
WIRE_W10_L100 = Workload(name="wire_W10_L100", W=10, L=100, eta=0.05, disorder=0.25,
                         emin=-3.5, emax=3.5, n_energies=256, walkers_per_energy=1_000_000)
WIRE_ETAS = (0.01, 0.05, 0.1)

# Inelastic walks (step 7') on the wire's grid (spacing 7 t / 256 = 0.0273 t): an elastic line
# and optical-phonon lines at hbar omega = 8 grid steps (0.219 t), emission (offset -8) weighted
# by n_B + 1 and absorption (+8) by n_B, n_B = 1 / (exp(hbar omega / kT) - 1) at kT = 0.1 t,
# both with coupling 0.5 against 1 for the elastic line.
PHONON_STEPS = 8
_N_BOSE = 1.0 / (np.exp(PHONON_STEPS * 7.0 / 256 / 0.1) - 1.0)
PHONON_LINES = (-PHONON_STEPS, 0, PHONON_STEPS)
PHONON_WEIGHTS = (0.5 * (_N_BOSE + 1.0), 1.0, 0.5 * _N_BOSE)

# Differentiation workload: W = 16, L = 200 (N = 3200), eta = 0.02 t, disorder U[-0.5 t, 0.5 t],
# 128 energies in [-3.5 t, 3.5 t]; dI/dV_i for every site and dI/deta = sum_i dI/dgamma_i.
DIFF_W16_L200 = Workload(name="diff_W16_L200", W=16, L=200, eta=0.02, disorder=0.5,
                         emin=-3.5, emax=3.5, n_energies=128, walkers_per_energy=0)


# Batched workload: 64 disorder realizations x 256 energies, W = 8, L drawn uniformly from
# {50, 100, 200, 400} per realization (seeded), eta = 0.05 t, disorder U[-0.5 t, 0.5 t],
# energies in [-3.5 t, 3.5 t] (inside the W = 8 lead band |E| < 3.879 t), 1e5 walkers/energy.
BATCH_W8 = Workload(name="batch_W8", W=8, L=50, eta=0.05, disorder=0.5, emin=-3.5, emax=3.5,
                    n_energies=256, walkers_per_energy=100_000)
BATCH_LENGTHS = (50, 100, 200, 400)
BATCH_REALIZATIONS = 64
BATCH_LENGTH_SEED = 1806


def batch_workloads(n: int = BATCH_REALIZATIONS):
    """The batched workload's realizations: realization r has length L_r drawn uniformly
    from BATCH_LENGTHS with numpy's default generator seeded by BATCH_LENGTH_SEED, and the
    disorder of realization r (see onsite)."""
    rng = np.random.default_rng(BATCH_LENGTH_SEED)
    Ls = rng.choice(np.array(BATCH_LENGTHS), size=n)
    return [BATCH_W8.replace(L=int(L), realization=r, name=f"batch_W8_L{int(L)}_r{r}")
            for r, L in enumerate(Ls)]


# Precision at scale: W = 32, L = 500 (N = 16000; the paper's 32 x 32 blocks, Sec. IV),
# eta = 0.01 t, disorder U[-0.3 t, 0.3 t], 512 energies in [-3.5 t, 3.5 t] (inside the W = 32
# lead band |E| < 3.991 t), 1e7 walkers/energy.  One energy's |G|^2, alias tables and probe
# matrix take 5.6 GB, so the energies are processed in batches (SCALE_BATCH per build).
SCALE_W32_L500 = Workload(name="scale_W32_L500", W=32, L=500, eta=0.01, disorder=0.3,
                          emin=-3.5, emax=3.5, n_energies=512, walkers_per_energy=10_000_000)
SCALE_BATCH = 32


def onsite(w: Workload) -> np.ndarray:
    """Onsite energies V_i (float64, length N, slice-major i = x*W + y).

    Uniform iid disorder drawn with numpy's default generator seeded by
    DISORDER_SEED_BASE + realization; all zeros when the disorder amplitude is zero.
    """
    if w.disorder == 0.0:
        return np.zeros(w.N, dtype=np.float64)
    rng = np.random.default_rng(DISORDER_SEED_BASE + w.realization)
    return rng.uniform(-w.disorder * w.t, w.disorder * w.t, size=w.N).astype(np.float64)


def dephasing(w: Workload) -> np.ndarray:
    """Per-site dephasing rates gamma_i = eta (float64, length N)."""
    return np.full(w.N, w.eta * w.t, dtype=np.float64)


def random_sites(n: int, seed: int, lo: float, hi: float) -> np.ndarray:
    """Seeded uniform values, used by tests for random onsite or dephasing arrays."""
    return np.random.default_rng(seed).uniform(lo, hi, size=n).astype(np.float64)


def energy_grid(emin: float, emax: float, n: int):
    """Energy points and weights of a window [emin, emax] (caller inputs of the library): the
    centres of n equal cells and the cell width as every point's weight, i.e. the midpoint
    rule of Sec. III C.  The library forms the weighted sum over energies itself."""
    dE = (emax - emin) / n
    return emin + (np.arange(n) + 0.5) * dE, np.full(n, dE)


def ramp_bias(W: int, L: int, a: float, inject_lead: int = 0, floor_p: float = 1e-3):
    """A bias over the N + 2 outcomes for importance-sampled walks (a caller input of the
    library): probes on slice x weigh (x + 1/2 + a) / (L + 2 a), x counted from the injecting
    lead p; the collecting lead weighs 1 and lead p weighs floor_p.  It is the exit
    probability of one-dimensional diffusion along the wire with contact length a (slices)."""
    x = np.repeat(np.arange(L, dtype=np.float64), W)
    if inject_lead == 1:
        x = (L - 1) - x
    b = np.empty(W * L + 2, dtype=np.float64)
    b[:W * L] = (x + 0.5 + a) / (L + 2.0 * a)
    b[W * L + 1 - inject_lead] = 1.0
    b[W * L + inject_lead] = floor_p
    return b
