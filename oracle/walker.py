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
