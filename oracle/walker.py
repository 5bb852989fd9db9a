"""ctypes wrapper and build step for the oracle's C walker (oracle/walker.c).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "walker.c")
_LIB = os.path.join(_HERE, "liboraclewalker.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile walker.c with gcc (OpenMP) into oracle/liboraclewalker.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_walk_cdf.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_void_p]
        L.oracle_walk_cdf.restype = ctypes.c_int
        L.oracle_walk_alias.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                        ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p]
        L.oracle_walk_alias.restype = ctypes.c_int
        L.oracle_walk_sampled_cdf.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                              ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                              ctypes.c_uint32, ctypes.c_void_p]
        L.oracle_walk_sampled_cdf.restype = ctypes.c_int
        L.oracle_walk_sampled_alias.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                                ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                                ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                                ctypes.c_void_p]
        L.oracle_walk_sampled_alias.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def philox4x32_10(counter, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xffffffff for x in counter])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def walk_cdf(K, seed, realization, inject_lead, walker_begin, n_walkers, max_steps=1_000_000,
             tallies=None):
    """Walk n_walkers per energy on dense weight rows K[nE][n][n] with the paper's sampler."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    if K.ndim == 2:
        K = K[None]
    nE, n, _ = K.shape
    if tallies is None:
        tallies = np.zeros((nE, 5), dtype=np.int64)
    rc = lib().oracle_walk_cdf(K.ctypes.data, nE, n, seed, realization, inject_lead,
                               walker_begin, n_walkers, max_steps, tallies.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_walk_cdf rejected its arguments")
    return tallies


def walk_alias(thr, alias, seed, realization, inject_lead, walker_begin, n_walkers,
               max_steps=1_000_000, tallies=None):
    """Walk on alias tables thr/alias[nE][n][pitch] (uint32 / int32)."""
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    alias = np.ascontiguousarray(alias, dtype=np.int32)
    if thr.ndim == 2:
        thr, alias = thr[None], alias[None]
    nE, n, pitch = thr.shape
    if tallies is None:
        tallies = np.zeros((nE, 5), dtype=np.int64)
    rc = lib().oracle_walk_alias(thr.ctypes.data, alias.ctypes.data, pitch, nE, n, seed,
                                 realization, inject_lead, walker_begin, n_walkers, max_steps,
                                 tallies.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_walk_alias rejected its arguments")
    return tallies


def walk_sampled_cdf(K, weights, seed, realization, inject_lead, walker_begin, n_walkers,
                     max_steps=1_000_000, tallies=None):
    """Energy-sampled walks: walker w draws its energy with probability weights[k] / sum,
    then walks on the dense rows K[k] with the paper's sampler; tallies[k] collects the
    walkers that drew energy k."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    wts = np.ascontiguousarray(weights, dtype=np.float64)
    nE, n, _ = K.shape
    if tallies is None:
        tallies = np.zeros((nE, 5), dtype=np.int64)
    rc = lib().oracle_walk_sampled_cdf(K.ctypes.data, nE, n, wts.ctypes.data, seed, realization,
                                       inject_lead, walker_begin, n_walkers, max_steps,
                                       tallies.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_walk_sampled_cdf rejected its arguments")
    return tallies


def walk_sampled_alias(thr, alias, weights, seed, realization, inject_lead, walker_begin,
                       n_walkers, max_steps=1_000_000, tallies=None):
    """Energy-sampled walks on given alias tables thr/alias[nE][n][pitch]."""
    thr = np.ascontiguousarray(thr, dtype=np.uint32)
    alias = np.ascontiguousarray(alias, dtype=np.int32)
    wts = np.ascontiguousarray(weights, dtype=np.float64)
    nE, n, pitch = thr.shape
    if tallies is None:
        tallies = np.zeros((nE, 5), dtype=np.int64)
    rc = lib().oracle_walk_sampled_alias(thr.ctypes.data, alias.ctypes.data, pitch, nE, n,
                                         wts.ctypes.data, seed, realization, inject_lead,
                                         walker_begin, n_walkers, max_steps, tallies.ctypes.data)
    if rc != 0:
        raise ValueError("oracle_walk_sampled_alias rejected its arguments")
    return tallies


def mc_current(tallies, c, weights, inject_lead=0):
    """Per-energy transmission estimates, their standard errors and the current from exit
    counts of walks injected at lead p (p = inject_lead; the collecting lead q is the other
    one).  Every walker scores X = c_p [exit at q] (Eq. (66), c_p = Tr Gamma_p A, the total
    of the injection row); a truncated walk scores 0 and still counts as a walker.  Per
    energy k with N_k walkers of which R_k exit at q:
        T_k = c_k R_k / N_k,
        sigma_k = sqrt(s^2 / N_k), s^2 = the sample variance (divisor N_k - 1) of the N_k
                  scores, i.e. c_k sqrt(p (1 - p) / (N_k - 1)) with p = R_k / N_k,
        I = sum_k w_k T_k,  sigma_I = sqrt(sum_k w_k^2 sigma_k^2)  (midpoint rule, Sec. III C;
                  energies walked independently).
    Returns (T[nE], sigma[nE], I, sigma_I)."""
    t = np.asarray(tallies, dtype=np.int64)
    c = np.asarray(c, dtype=np.float64)
    w = np.asarray(weights, dtype=np.float64)
    nE = t.shape[0]
    T = np.zeros(nE)
    sig = np.zeros(nE)
    for k in range(nE):
        walkers = int(t[k, 0] + t[k, 1] + t[k, 2])
        hits = int(t[k, 1] if inject_lead == 0 else t[k, 0])
        if walkers <= 0:
            continue
        p = hits / walkers
        T[k] = c[k] * p
        if walkers > 1:
            sig[k] = c[k] * np.sqrt(p * (1.0 - p) / (walkers - 1))
    I = float(np.sum(w * T))
    sI = float(np.sqrt(np.sum(w * w * sig * sig)))
    return T, sig, I, sI


def sampled_current(tallies, c, weights, inject_lead=0):
    """(I, sigma_I) of energy-sampled walks: the variable X = W c_p(E_k) when the walker exits
    at the collecting lead, 0 otherwise (Eq. (66) with the energy density h proportional to
    the weights, W = sum of the weights), averaged over all N walkers; sigma_I from the sample
    variance of X."""
    t = np.asarray(tallies, dtype=np.int64)
    c = np.asarray(c, dtype=np.float64)
    W = float(np.sum(weights))
    hits = t[:, 1] if inject_lead == 0 else t[:, 0]
    N = float(t[:, :3].sum())
    X = W * c  # the value of X for an exit at q at each energy
    mean = float(np.dot(X, hits)) / N
    mean_sq = float(np.dot(X * X, hits)) / N
    var = (mean_sq - mean * mean) * N / (N - 1.0) if N > 1 else 0.0
    return mean, float(np.sqrt(max(var, 0.0) / N))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def find_redraws(seed, realization, inject_lead, k, n_step, nout, w_begin, count, min_redraws,
                 max_out=64):
    """Walkers of [w_begin, w_begin + count) at energy index k whose step-n_step bucket over
    nout outcomes needs at least min_redraws redraws of Lemire's rejection: (number found,
    [(walker, redraws, accepted bucket), ...] for the first max_out of them)."""
    L = lib()
    f = L.oracle_find_redraws
    f.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                  ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                  ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_int64]
    f.restype = ctypes.c_int64
    ow = np.zeros(max_out, np.uint32)
    orr = np.zeros(max_out, np.uint32)
    oc = np.zeros(max_out, np.uint32)
    n = f(seed, realization, inject_lead, k, n_step, nout, w_begin, count, min_redraws,
          ow.ctypes.data, orr.ctypes.data, oc.ctypes.data, max_out)
    if n < 0:
        raise ValueError("oracle_find_redraws rejected its arguments")
    m = min(int(n), max_out)
    return int(n), [(int(ow[i]), int(orr[i]), int(oc[i])) for i in range(m)]


def _interp(mode, tables, lo, alpha32, seed, realization, inject_lead, walker_begin, n_walkers,
            max_steps, tallies):
    lo = np.ascontiguousarray(lo, dtype=np.int32)
    a32 = np.ascontiguousarray(alpha32, dtype=np.uint32)
    nF = len(lo)
    if tallies is None:
        tallies = np.zeros((nF, 5), dtype=np.int64)
    L = lib()
    i32, u32, u64, vp = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
    if mode == 0:
        K = np.ascontiguousarray(tables, dtype=np.float64)
        nN, n, _ = K.shape
        f = L.oracle_walk_interp_cdf
        f.argtypes = [vp, i32, i32, vp, vp, i32, u64, u32, u32, u64, u64, u32, vp]
        f.restype = ctypes.c_int
        rc = f(K.ctypes.data, nN, n, lo.ctypes.data, a32.ctypes.data, nF, seed, realization,
               inject_lead, walker_begin, n_walkers, max_steps, tallies.ctypes.data)
    else:
        thr = np.ascontiguousarray(tables[0], dtype=np.uint32)
        al = np.ascontiguousarray(tables[1], dtype=np.int32)
        nN, n, pitch = thr.shape
        f = L.oracle_walk_interp_alias
        f.argtypes = [vp, vp, ctypes.c_int64, i32, i32, vp, vp, i32, u64, u32, u32, u64, u64,
                      u32, vp]
        f.restype = ctypes.c_int
        rc = f(thr.ctypes.data, al.ctypes.data, pitch, nN, n, lo.ctypes.data, a32.ctypes.data,
               nF, seed, realization, inject_lead, walker_begin, n_walkers, max_steps,
               tallies.ctypes.data)
    if rc != 0:
        raise ValueError("oracle interpolated walk rejected its arguments")
    return tallies


def walk_interp_cdf(K, lo, alpha32, seed, realization, inject_lead, walker_begin, n_walkers,
                    max_steps=1_000_000, tallies=None):
    """Interpolated walks (oracle/walker.c) on the nodes' dense rows K[nN][n][n]: fine energy
    f mixes node lo[f] and lo[f] + 1 with weight alpha32[f] / 2^32; tallies per fine energy."""
    return _interp(0, K, lo, alpha32, seed, realization, inject_lead, walker_begin, n_walkers,
                   max_steps, tallies)


def walk_interp_alias(thr, alias, lo, alpha32, seed, realization, inject_lead, walker_begin,
                      n_walkers, max_steps=1_000_000, tallies=None):
    """Interpolated walks on the nodes' alias tables thr/alias[nN][n][pitch]."""
    return _interp(1, (thr, alias), lo, alpha32, seed, realization, inject_lead, walker_begin,
                   n_walkers, max_steps, tallies)
