"""Inelastic Buttiker walks: the energy draw of step 7' (Sec. II F) and the exact Markov chain
it defines.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Never called by the HIP library.

Model.  Buttiker's approximation with an energy-changing coupling lambda~_i(E, E') (Sec. II F):
after step 6' has drawn a probe i at energy E_n, step 7' draws the next energy with
    p(E) = lambda~_i(E, E_n) A_ii(E) / integral dE lambda~_i(E, E_n) A_ii(E)      (Eq. (74))
and the walk continues from probe i's row at that energy (step 11: psi = G(E)|i>).  Here the
coupling is a sum of lines on the energy grid, lambda~_i(E, E_n) = sum_k lambda_k
delta(E - E_n - Delta_k) with Delta_k = offsets[k] grid steps (an elastic line at 0, phonon
emission and absorption at -/+ hbar omega, ...), the same for every site; a line that falls
outside the grid has weight 0 (the energy window is closed).  So from (E_n, i) the walk moves
to E_n + Delta_k with probability x_k / sum x, x_k = lambda_k A_ii(E_n + Delta_k).

Condition (iv) of Sec. II F (Eq. (69)) ties the dephasing rates to the coupling, gamma_i(E) =
integral dE' lambda~_i(E', E) A_ii(E'); the walk is a proper Markov chain whether or not the
caller's gamma satisfies it (step 7' is normalised by its own sum).

Walk (the C walker, oracle/walker.c): states (energy index e, row s).  Inject at lead p at
energy e0, step 6' on the rows of energy e; a probe outcome i is followed by step 7'.  A walk
is scored by its injection energy: X = c_p(e0) [exit at q] as in Eq. (66), so the current
estimator of the elastic walk applies unchanged; the exit energy is counted as well.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import walker as OW

TWO32 = 4294967296.0


def line_weights(Adiag, offsets, lambdas):
    """x[e][i][k] = lambda_k A_ii(E_{e + offsets[k]}) (0 when e + offsets[k] is off the grid)."""
    A = np.asarray(Adiag, dtype=np.float64)
    nE, N = A.shape
    off = np.asarray(offsets, dtype=np.int64)
    lam = np.asarray(lambdas, dtype=np.float64)
    x = np.zeros((nE, N, off.size))
    for e in range(nE):
        for k, (d, l) in enumerate(zip(off, lam)):
            if 0 <= e + d < nE:
                x[e, :, k] = l * A[e + d]
    return x


def energy_probabilities(Adiag, offsets, lambdas):
    """p[e][i][k]: probability that step 7' from probe i at energy e moves to e + offsets[k]."""
    x = line_weights(Adiag, offsets, lambdas)
    return x / x.sum(axis=2, keepdims=True)


def energy_table(Adiag, offsets, lambdas):
    """uint64 thresholds [nE][N][K] of the draw: t_k = floor(2^32 cum_k / total) with cum_k the
    running sum of x_0..x_k (in order, FP64) and total = cum_{K-1}; the first k with
    r < t_k is drawn for a uniform 32-bit word r.  Offsets after the last line with weight
    keep t = 2^32, lines of zero weight repeat the previous threshold (never drawn)."""
    x = line_weights(Adiag, offsets, lambdas)
    cum = np.cumsum(x, axis=2)
    total = cum[:, :, -1:]
    if not (total > 0).all():
        raise ValueError("a probe has no energy to move to (all lines weightless)")
    return np.floor(cum / total * TWO32).astype(np.uint64)


def table_probabilities(table):
    """The exact probabilities the thresholds give: (t_k - t_{k-1}) / 2^32 with t_{-1} = 0
    and the last entry read as 2^32."""
    t = np.asarray(table, dtype=np.float64).copy()
    t[:, :, -1] = TWO32
    prev = np.concatenate([np.zeros_like(t[:, :, :1]), t[:, :, :-1]], axis=2)
    return np.maximum(t - prev, 0.0) / TWO32


def exit_distribution(Ks, Adiag, offsets, lambdas, inject_lead=0, p_energy=None):
    """B[e0][r][e]: probability that a walk injected at lead p at energy index e0 is absorbed
    at lead r with energy index e, from the first-step equations of the chain on the probe
    states (e, i): X = Q X + R with Q[(e, j), (e', i)] = P_e[j, i] p(e' | e, i) and
    R[(e, j), (r, e)] = P_e[j, N + r] (dense LAPACK solve over nE N states).  Ks [nE][n][n]
    are the step-6' weight rows (rows normalised here).  p_energy [nE][N][K] overrides the
    step-7' probabilities (e.g. table_probabilities of a threshold table)."""
    Ks = np.asarray(Ks, dtype=np.float64)
    nE, n, _ = Ks.shape
    N = n - 2
    off = np.asarray(offsets, dtype=np.int64)
    pe = energy_probabilities(Adiag, offsets, lambdas) if p_energy is None else \
        np.asarray(p_energy, dtype=np.float64)
    P = Ks / Ks.sum(axis=2, keepdims=True)
    M = nE * N
    Q = np.zeros((M, M))
    R = np.zeros((M, 2 * nE))
    for e in range(nE):
        for j in range(N):
            row = e * N + j
            for k, d in enumerate(off):
                if not 0 <= e + d < nE:
                    continue
                Q[row, (e + d) * N:(e + d + 1) * N] += P[e, j, :N] * pe[e, :, k]
            R[row, e] = P[e, j, N]
            R[row, nE + e] = P[e, j, N + 1]
    X = np.linalg.solve(np.eye(M) - Q, R)
    B = np.zeros((nE, 2, nE))
    row = N + inject_lead
    for e0 in range(nE):
        b = np.zeros(2 * nE)
        b[e0] += P[e0, row, N]
        b[nE + e0] += P[e0, row, N + 1]
        for k, d in enumerate(off):
            if not 0 <= e0 + d < nE:
                continue
            first = P[e0, row, :N] * pe[e0, :, k]    # probe i, then energy e0 + d
            b += first @ X[(e0 + d) * N:(e0 + d + 1) * N]
        B[e0] = b.reshape(2, nE)
    return B


def spectrum(tallies, hist, c, weights, inject_lead=0):
    """Energy-resolved current out of lead q (the lead opposite p) and into lead p:
    S[r][e] = sum_{e0} w_{e0} c_p(e0) hist[r][e0][e] / N_{e0} (N_{e0} = walkers at e0,
    truncated ones included), so sum_e S[q][e] is the Monte Carlo current I of the tallies."""
    t = np.asarray(tallies, dtype=np.int64)
    h = np.asarray(hist, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    nw = (t[:, 0] + t[:, 1] + t[:, 2]).astype(np.float64)
    scale = np.where(nw > 0, w * c / np.where(nw > 0, nw, 1.0), 0.0)
    return np.einsum("e,ref->rf", scale, h)


def _walk(mode, tables, etab, offsets, seed, realization, inject_lead, walker_begin,
          n_walkers, max_steps):
    etab = np.ascontiguousarray(etab, dtype=np.uint64)
    off = np.ascontiguousarray(offsets, dtype=np.int32)
    nE = etab.shape[0]
    tal = np.zeros((nE, 5), dtype=np.int64)
    hist = np.zeros((2, nE, nE), dtype=np.int64)
    bad = ctypes.c_int32(0)
    vp, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    L = OW.lib()
    if mode == 0:
        K = np.ascontiguousarray(tables, dtype=np.float64)
        n = K.shape[1]
        f = L.oracle_walk_inelastic_cdf
        f.argtypes = [vp, i32, i32, vp, vp, i32, u64, u32, u32, u64, u64, u32, vp, vp, vp]
        args = [K.ctypes.data, nE, n]
    else:
        thr = np.ascontiguousarray(tables[0], dtype=np.uint32)
        al = np.ascontiguousarray(tables[1], dtype=np.int32)
        n, pitch = thr.shape[1], thr.shape[2]
        f = L.oracle_walk_inelastic_alias
        f.argtypes = [vp, vp, ctypes.c_int64, i32, i32, vp, vp, i32, u64, u32, u32, u64, u64,
                      u32, vp, vp, vp]
        args = [thr.ctypes.data, al.ctypes.data, pitch, nE, n]
    f.restype = ctypes.c_int
    if f(*args, etab.ctypes.data, off.ctypes.data, off.size, seed, realization, inject_lead,
         walker_begin, n_walkers, max_steps, tal.ctypes.data, hist.ctypes.data,
         ctypes.byref(bad)) != 0:
        raise ValueError("the inelastic walker rejected its arguments")
    return tal, hist, bool(bad.value)


def walk_cdf(K, etab, offsets, seed, realization, inject_lead, walker_begin, n_walkers,
             max_steps=1_000_000):
    """(tallies [nE][5], hist [2][nE][nE], bad) of the C walker with the paper's step-6'
    sampler on weight rows K [nE][n][n] and the step-7' table etab [nE][N][K]."""
    return _walk(0, K, etab, offsets, seed, realization, inject_lead, walker_begin, n_walkers,
                 max_steps)


def walk_alias(thr, alias, etab, offsets, seed, realization, inject_lead, walker_begin,
               n_walkers, max_steps=1_000_000):
    """The same on alias tables thr/alias [nE][n][pitch]."""
    return _walk(1, (thr, alias), etab, offsets, seed, realization, inject_lead, walker_begin,
                 n_walkers, max_steps)
