"""Importance-sampled (weighted) walks: the variance reduction of Sec. V A, "Improved estimator".

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper proposes replacing the step-6' probabilities p (Sec. II F, Eqs. (75), (76)) by other
probabilities p' and weighting the estimator of Eq. (66) by the ratio p/p' along the path.
The oracle takes p' in the form that keeps every row's support and makes the ratio a product
of per-state factors: for a non-negative bias b over the N + 2 outcomes (probes, lead L, lead
R),
    p'_ij = p_ij b_j / rho_i,     rho_i = sum_j p_ij b_j,
so a step i -> j multiplies the path's likelihood ratio by p_ij / p'_ij = rho_i / b_j.  A walk
injected at lead p that exits at the collecting lead q scores X' = c_p times the product of
its ratios; any other walk scores 0.  E'[X'] = c_p P(exit at q) = T_qp for every b that is
positive on the probes and on q (paths through a zero-bias probe would be lost).

With b = h, the absorption probabilities at q (dense.absorption_probabilities), rho = h on
every row (h is harmonic for the walk), the product telescopes to h(injection row) / h(q) =
h(injection row) and every walk scores exactly T_qp: zero variance.  Approximations of h
(e.g. a ramp along the wire for transport from L to R) lower the variance; poor ones can make
the second moment infinite, which second_moment() detects.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import walker as OW


def normalised(K):
    """Rows of K (any non-negative weights) normalised to probabilities (zero rows kept)."""
    K = np.asarray(K, dtype=np.float64)
    s = K.sum(axis=-1, keepdims=True)
    return np.divide(K, s, out=np.zeros_like(K), where=s > 0)


def modified_rows(K, b):
    """Weights of p' (unnormalised): K_ij b_j."""
    return np.asarray(K, dtype=np.float64) * np.asarray(b, dtype=np.float64)[..., None, :]


def rho(K, b):
    """rho_i = sum_j p_ij b_j (the mean bias of row i's outcomes under p)."""
    return np.einsum("...ij,...j->...i", normalised(K), np.asarray(b, dtype=np.float64))


def ramp_bias(W, L, inject_lead=0, a=5.0, floor_p=0.0):
    """A bias for transport from lead p to q along a W x L wire: probes on slice x get
    (x + 1/2 + a) / (L + 2 a) measured from lead p (the harmonic function of 1D diffusion with
    contact length a), q gets 1 and p gets floor_p."""
    x = np.repeat(np.arange(L, dtype=np.float64), W)
    if inject_lead == 1:
        x = (L - 1) - x
    b = np.empty(W * L + 2)
    b[:W * L] = (x + 0.5 + a) / (L + 2.0 * a)
    q = W * L + 1 - inject_lead
    b[q] = 1.0
    b[W * L + inject_lead] = floor_p
    return b


def _walk(mode, tables, rho_, bias, seed, realization, inject_lead, walker_begin, n_walkers,
          max_steps, tallies, wsum):
    rho_ = np.ascontiguousarray(rho_, dtype=np.float64)
    bias = np.ascontiguousarray(bias, dtype=np.float64)
    if rho_.ndim == 1:
        rho_, bias = rho_[None], bias[None]
    nE, n = rho_.shape
    if bias.shape != (nE, n):
        raise ValueError("bias must match rho: [nE][n]")
    if tallies is None:
        tallies = np.zeros((nE, 5), dtype=np.int64)
    if wsum is None:
        wsum = np.zeros((nE, 2), dtype=np.float64)
    L = OW.lib()
    i32, u32, u64, vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    if mode == 0:
        Kb = np.ascontiguousarray(tables, dtype=np.float64)
        if Kb.ndim == 2:
            Kb = Kb[None]
        f = L.oracle_walk_weighted_cdf
        f.argtypes = [vp, i32, i32, vp, vp, u64, u32, u32, u64, u64, u32, vp, vp]
        f.restype = ctypes.c_int
        rc = f(Kb.ctypes.data, nE, n, rho_.ctypes.data, bias.ctypes.data, seed, realization,
               inject_lead, walker_begin, n_walkers, max_steps, tallies.ctypes.data,
               wsum.ctypes.data)
    else:
        thr = np.ascontiguousarray(tables[0], dtype=np.uint32)
        al = np.ascontiguousarray(tables[1], dtype=np.int32)
        if thr.ndim == 2:
            thr, al = thr[None], al[None]
        pitch = thr.shape[2]
        f = L.oracle_walk_weighted_alias
        f.argtypes = [vp, vp, ctypes.c_int64, i32, i32, vp, vp, u64, u32, u32, u64, u64, u32,
                      vp, vp]
        f.restype = ctypes.c_int
        rc = f(thr.ctypes.data, al.ctypes.data, pitch, nE, n, rho_.ctypes.data,
               bias.ctypes.data, seed, realization, inject_lead, walker_begin, n_walkers,
               max_steps, tallies.ctypes.data, wsum.ctypes.data)
    if rc != 0:
        raise ValueError("oracle weighted walk rejected its arguments")
    return tallies, wsum


def walk_weighted_cdf(K, b, seed, realization, inject_lead, walker_begin, n_walkers,
                      max_steps=1_000_000, tallies=None, wsum=None):
    """Weighted walks with the paper's cumulative-sum sampler on the modified rows of the
    dense kernel K[nE][n][n] for the bias b[nE][n]; returns (tallies[nE][5], wsum[nE][2])."""
    K = np.asarray(K, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if K.ndim == 2:
        K, b = K[None], b[None]
    return _walk(0, modified_rows(K, b), rho(K, b), b, seed, realization, inject_lead,
                 walker_begin, n_walkers, max_steps, tallies, wsum)


def walk_weighted_alias(thr, alias, rho_, b, seed, realization, inject_lead, walker_begin,
                        n_walkers, max_steps=1_000_000, tallies=None, wsum=None):
    """Weighted walks on alias tables of the modified rows (thr/alias[nE][n][pitch]) with the
    given rho and bias [nE][n]; returns (tallies, wsum)."""
    return _walk(1, (thr, alias), rho_, b, seed, realization, inject_lead, walker_begin,
                 n_walkers, max_steps, tallies, wsum)


def weighted_current(tallies, wsum, c, weights):
    """Per-energy estimates from weighted walks: with N_k walkers (every walk, truncated ones
    included) and the score sums S1 = wsum[k, 0], S2 = wsum[k, 1] (scores without c_k),
        T_k = c_k S1 / N_k,
        sigma_k = c_k sqrt(s^2 / N_k), s^2 = (S2 - S1^2 / N_k) / (N_k - 1), the sample
                  variance of the N_k scores,
        I = sum_k w_k T_k,  sigma_I = sqrt(sum_k w_k^2 sigma_k^2).
    Returns (T[nE], sigma[nE], I, sigma_I)."""
    t = np.asarray(tallies, dtype=np.int64)
    ws = np.asarray(wsum, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    nE = t.shape[0]
    T = np.zeros(nE)
    sig = np.zeros(nE)
    for k in range(nE):
        n = int(t[k, 0] + t[k, 1] + t[k, 2])
        if n <= 0:
            continue
        T[k] = c[k] * ws[k, 0] / n
        if n > 1:
            var = max(ws[k, 1] - ws[k, 0] * ws[k, 0] / n, 0.0) / (n - 1)
            sig[k] = c[k] * np.sqrt(var / n)
    I = float(np.sum(w * T))
    sI = float(np.sqrt(np.sum(w * w * sig * sig)))
    return T, sig, I, sI


def second_moment(K, b, inject_lead=0):
    """Exact E'[(X'/c_p)^2] of the weighted score for one energy's kernel K[n][n], or inf when
    it diverges.  With m_i the second moment of the remaining ratio product from state i,
        m_i = sum_j p'_ij (rho_i / b_j)^2 m_j = rho_i sum_j p_ij m_j / b_j
    over probes j, with m_q = 1 and m = 0 at the other lead; the series converges when the
    spectral radius of rho_i p_ij / b_j over the probes is below 1."""
    P = normalised(K)
    b = np.asarray(b, dtype=np.float64)
    n = P.shape[0]
    N = n - 2
    q = N + 1 - inject_lead
    r = rho(K, b)
    with np.errstate(divide="ignore", invalid="ignore"):
        M = np.where(P[:N, :N] > 0, r[:N, None] * P[:N, :N] / b[None, :N], 0.0)
    if np.max(np.abs(np.linalg.eigvals(M))) >= 1.0:
        return float("inf")
    rhs = r[:N] * P[:N, q] / b[q]
    m = np.linalg.solve(np.eye(N) - M, rhs)
    row = N + inject_lead
    with np.errstate(divide="ignore", invalid="ignore"):
        tail = np.where(P[row, :N] > 0, P[row, :N] * m / b[:N], 0.0)
    return float(r[row] * (tail.sum() + P[row, q] / b[q]))
