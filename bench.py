"""Benchmark of the Monte Carlo NEGF hot path on one MI355X.

One step = the whole path for the W=10 x L=100 disordered wire (N = 1000 sites, 256
midpoint energies in [-3.5 t, 3.5 t], disorder U[-0.25 t, 0.25 t]) at each dephasing rate
eta in {0.01, 0.05, 0.1} t: build G / kernel rows / alias tables for all 256 energies,
walk 1e6 walkers per energy, MC current, DIRECT current.  Inputs are resident in HBM before
the timed region starts.  The timed steps run as they would in use; the same steps are then
run again with every kernel launch timed by HIP events on its own stream (the library's
opt-in launch timer), which gives the per-kernel times and the roofline of the dominant
kernel.

Printed (one JSON line): walk steps per second of the whole step, per-stage and per-kernel
times, the roofline of the dominant kernel, time to a 1% relative deviation of the lead
current for MC and for the DIRECT GPU solve (with the error realized at the stop), and the
oracle timed on the host's cores for a bounded sample of the same workload.  Further
objects: "chain" (the N = 50 chain, with the oracle's DIRECT and MC-to-1% times on all its
energies), "grad" (dI/dV_i for all sites and dI/dgamma_i on the W=16 x L=200
differentiation workload), "batched" (64 realizations x 256 energies of W=8 wires of four
lengths, walked in memory-bounded waves, each wave one replayed HIP graph with one batched
walker launch) and "scale" (all 512 energies of the W=32 x L=500 wire in 16 timed batches).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_1805_10164_amd import inputs  # noqa: E402
from paper_1805_10164_amd import mcnegf as M  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TFLOPS = 78.6
# Algorithmic bytes of one walk step: one alias entry of an FP64 threshold and an int32 alias
# index.  The walker stores entries packed into 4 bytes (16 threshold bits and a 16-bit alias
# index; the low 16 threshold bits are read only on a 2^-16 tie), and that figure is reported
# beside the algorithmic one.
STEP_BYTES = 12
ALIAS_ENTRY_BYTES = 4
PROFILES = os.path.join(ROOT, "profiles")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--walkers", type=int, default=None, help="walkers per energy (default 1e6)")
    ap.add_argument("--etas", type=str, default=None, help="comma-separated dephasing rates")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttp", action="store_true", help="skip the time-to-1%% measurement")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the gradient measurement on the differentiation workload")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched uneven workload (64 realizations x 256 energies)")
    ap.add_argument("--no-scale", action="store_true",
                    help="skip the W=32 x L=500 (N = 16000) workload")
    ap.add_argument("--no-chain", action="store_true", help="skip the N = 50 chain")
    ap.add_argument("--no-inelastic", action="store_true",
                    help="skip the inelastic walks (step 7') on the wire")
    ap.add_argument("--no-resistance", action="store_true",
                    help="skip the resistance-versus-length sweep")
    ap.add_argument("--only", choices=["grad", "batched", "scale", "chain", "inelastic",
                                       "resistance"],
                    default=None,
                    help="run only this leg and print its object (profiling; no top-level metric)")
    ap.add_argument("--serial-builds", action="store_true",
                    help="issue the three dephasing rates' builds one after another on one stream")
    ap.add_argument("--scale-batches", type=int, default=None,
                    help="time only this many energy batches of the N = 16000 leg and skip its "
                         "FP32 variants (profiling runs)")
    ap.add_argument("--batch-budget-gb", type=float, default=160.0,
                    help="device memory for one wave of build workspaces in the batched leg")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="before the timed steps, run one plain device copy of this many MiB "
                         "(reference dispatch for HBM byte counters)")
    return ap.parse_args()


class Problem:
    """Device-resident inputs and workspace for one dephasing rate."""

    def __init__(self, wl: inputs.Workload, torch, dev):
        self.wl = wl
        self.sys = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead)
        # the DIRECT current alone needs no alias tables
        self.sys_direct = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l,
                                        wl.delta_lead, M.BUILD_NO_ALIAS)
        E, w = inputs.energy_grid(wl.emin, wl.emax, wl.n_energies)
        self.V = torch.tensor(inputs.onsite(wl), device=dev)
        self.g = torch.tensor(inputs.dephasing(wl), device=dev)
        self.E = torch.tensor(E, device=dev)
        self.w = torch.tensor(w, device=dev)
        self.ws = M.allocate_workspace(self.sys, wl.n_energies, dev)
        self.tal = torch.zeros((wl.n_energies, M.TALLY_N), dtype=torch.int64, device=dev)
        self.sampled_scratch = None  # energy-sampled walks (time-to-1%), allocated on first use
        self.weighted = None  # importance-sampled walks (time-to-1%), allocated on first use
        self.T = torch.empty(wl.n_energies, dtype=torch.float64, device=dev)
        self.sig = torch.empty_like(self.T)
        self.Td = torch.empty_like(self.T)
        self.sigd = torch.empty_like(self.T)
        self.out = torch.zeros((2, 2), dtype=torch.float64, device=dev)  # (MC, DIRECT) x (I, sigma)
        self.k = None


def run_step(p: Problem, walkers, seed, walk_on):
    """Whole hot path for one problem, asynchronous on the current stream: build, walks, MC
    current and DIRECT current into p.out (read after the stream is synchronised)."""
    p.k = M.mc_negf_build_kernel(p.sys, p.V, p.g, p.E, p.ws)
    if walk_on:
        p.tal.zero_()
        M.mc_negf_walk(p.k, seed, p.wl.realization, 0, 0, walkers, 1_000_000, p.tal)
        M.mc_negf_current_async(p.k, 0, 0, p.tal, p.w, p.T, p.sig, p.out[0])
    M.mc_negf_current_async(p.k, 1, 0, None, p.w, p.Td, p.sigd, p.out[1])


def run_step_overlapped(probs, streams, walkers, seed, walk_on):
    """The step of run_step for several problems, with their builds (RGF sweeps, full inverse,
    lead terms, alias tables: independent workspaces) issued on their own streams so that they
    overlap, and the walks and both currents issued afterwards in order on the current stream
    (a walk runs alone: its tables stay in the XCDs' L2)."""
    import torch
    main = torch.cuda.current_stream()
    start = torch.cuda.Event()
    start.record(main)
    done = []
    for p, st in zip(probs, streams):
        st.wait_event(start)
        p.k = M.mc_negf_build_kernel(p.sys, p.V, p.g, p.E, p.ws, stream=st)
        ev = torch.cuda.Event()
        ev.record(st)
        done.append(ev)
    for p, ev in zip(probs, done):
        main.wait_event(ev)
        if walk_on:
            p.tal.zero_()
            M.mc_negf_walk(p.k, seed, p.wl.realization, 0, 0, walkers, 1_000_000, p.tal)
            M.mc_negf_current_async(p.k, 0, 0, p.tal, p.w, p.T, p.sig, p.out[0])
        M.mc_negf_current_async(p.k, 1, 0, None, p.w, p.Td, p.sigd, p.out[1])


def step_results(p: Problem, walk_on):
    """(status_mc, I_mc, sigma_mc, status_d, I_d) after the stream is synchronised."""
    out = p.out.cpu().numpy()
    flags = M.mc_negf_status(p.k)
    bad = flags & (M.FLAG_NONFINITE | M.FLAG_SINGULAR | M.FLAG_NOTSPD)
    st_d = M.ENUMERIC if bad else (M.WNUMERIC if flags & M.FLAG_ROWSUM else M.OK)
    st_mc = None
    if walk_on:
        st_mc = M.ENUMERIC if bad else (M.WTRUNC if flags & M.FLAG_TRUNC else st_d)
    return (st_mc, float(out[0, 0]) if walk_on else None, float(out[0, 1]) if walk_on else None,
            st_d, float(out[1, 0]))


def kernel_work(name, wl, walk_steps):
    """Algorithmic work of one launch of `name` for workload wl: (bound, amount, unit)."""
    N, W, nE = wl.N, wl.W, wl.n_energies
    n = N + 2
    if name == "walk_kernel":
        return "hbm", walk_steps * STEP_BYTES / 1e9, "GB"
    if name == "cholesky_kernel":
        # factorization N^3/3 plus the two forward substitutions of the bordered rows, 2 N^2
        return "mfma", nE * (N ** 3 / 3.0 + 2.0 * N * N) / 1e12, "TFLOP"
    if name == "fullinv_kernel":
        # two sweeps per column slice: L*(L-1) complex W x W block products per energy
        return "alu", nE * 8.0 * W ** 3 * wl.L * (wl.L - 1) / 1e12, "TFLOP"
    if name == "alias_build_kernel":
        # read gamma_i |G_ji|^2 rows and write one 4-byte entry plus 2 low threshold bytes per outcome
        return "hbm", nE * (8.0 * N * N + 6.0 * n * n) / 1e9, "GB"
    return None


def roofline(name, wl, ms_per_launch, walk_steps):
    w = kernel_work(name, wl, walk_steps)
    if w is None:
        return None
    bound, amount, unit = w
    if unit == "GB":
        achieved = amount / (ms_per_launch * 1e-3)
        r = {"kernel": name, "bound": bound, "achieved": achieved, "peak": HBM_PEAK_GBS,
             "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
             "algorithmic_per_launch": amount * 1e9, "avg_launch_ms": ms_per_launch}
        if name == "walk_kernel":
            r.update(walker_entry_figures(walk_steps, ms_per_launch))
        return r
    achieved = amount / (ms_per_launch * 1e-3)
    # gfx950's FP64 matrix-core peak equals its FP64 vector FMA peak
    return {"kernel": name, "bound": bound, "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_VALU_PEAK_TFLOPS,
            "algorithmic_per_launch": amount * 1e12, "avg_launch_ms": ms_per_launch}


def walker_entry_figures(steps_per_launch, ms_per_launch):
    """The walker's rate in walk steps and in the bytes of the packed entries it reads (4 per
    step), beside the algorithmic 12 bytes per step of the roofline."""
    sps = steps_per_launch / (ms_per_launch * 1e-3)
    return {"bytes_per_step": STEP_BYTES, "steps_per_launch": steps_per_launch,
            "steps_per_s": sps, "entry_bytes_per_step": ALIAS_ENTRY_BYTES,
            "entry_gbs": sps * ALIAS_ENTRY_BYTES / 1e9,
            "entry_frac": sps * ALIAS_ENTRY_BYTES / 1e9 / HBM_PEAK_GBS}


def window_plan(n_steps, launches_per_step, cap):
    """Steps per launch-timer window: whole steps, at most `cap` launches in a window (the
    timer records at most that many), n_steps in all."""
    per = max(1, cap // max(1, launches_per_step))
    if launches_per_step > cap:
        raise RuntimeError(f"one step issues {launches_per_step} launches; the launch timer "
                           f"holds {cap}")
    plan = []
    left = n_steps
    while left > 0:
        plan.append(min(per, left))
        left -= plan[-1]
    return plan


def require_complete(lt):
    """Raise if a launch-timer window dropped records (its per-launch figures would cover
    only part of the work that the wall time and the tallies cover)."""
    if getattr(lt, "dropped", 0):
        raise RuntimeError(f"launch timer dropped {lt.dropped} records")
    return lt


def timed_records(n_steps, launches_per_step, issue, cap=None):
    """Issue n_steps steps (issue() issues one) under launch-timer windows of whole steps;
    returns every launch's (name, ms).  Every window is checked for dropped records."""
    cap = M.PROFILE_MAX if cap is None else cap
    records = []
    for n in window_plan(n_steps, launches_per_step, cap):
        with M.LaunchTimes() as lt:
            for _ in range(n):
                issue()
        records += require_complete(lt).records
    return records


def per_kernel_table(records, steps):
    """Per kernel: launches, mean ms per launch and ms per step over `steps` steps."""
    names = sorted(set(n for n, _ in records))
    out = {}
    for n in names:
        ms = [m for k, m in records if k == n]
        out[n] = {"launches": len(ms), "ms_per_launch": sum(ms) / len(ms),
                  "ms_per_step": sum(ms) / steps}
    return out


def measured_traffic(name, workload="wire_W10_L100"):
    """HBM bytes per launch from the committed rocprofv3 counter summary for `name` on
    `workload`, or None when the kernel's source changed since the counters were taken."""
    path = os.path.join(PROFILES, f"{name}_{workload}_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
            return None
        return float(rec["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def add_traffic_rate(roof):
    """The measured HBM bytes per launch (`traffic`, rocprofv3) as a rate over the launch's
    measured duration, and its fraction of the HBM peak: what the kernel moves, beside what it
    needs (`achieved`)."""
    t, ms = roof.get("traffic"), roof.get("avg_launch_ms")
    if t is not None and ms:
        roof["traffic_gbs"] = t / 1e9 / (ms * 1e-3)
        roof["traffic_frac_of_hbm_peak"] = roof["traffic_gbs"] / HBM_PEAK_GBS
        # the useful fraction of what moves: algorithmic bytes over measured bytes
        if roof.get("unit") == "GB/s" and roof.get("algorithmic_per_launch"):
            roof["useful_fraction_of_traffic"] = roof["algorithmic_per_launch"] / t
    return roof


def grad_work(wl: inputs.Workload):
    """Algorithmic work of one adjoint_solve_kernel launch (all energies): HBM bytes (G read
    in both sweeps, the forward results written and read back) and FP64 flops (two complex
    W x W block products per slice for N + W right-hand sides)."""
    N, W, nE = wl.N, wl.W, wl.n_energies
    nbytes = nE * (2.0 * 16 * N * N + 2.0 * 16 * N * (N + W))
    flops = nE * (N + W) * 2.0 * wl.L * 8.0 * W * W
    return nbytes, flops


def grad_bench(torch, dev, steps, warmup, with_cpu):
    """dI/dV_i for every site and dI/deta on the differentiation workload (mc_negf_grad:
    DIRECT solve, back substitution, G columns, adjoint solves, assembly), HIP-event timed."""
    wl = inputs.DIFF_W16_L200
    sysm = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead,
                         M.BUILD_NO_ALIAS)
    E, w = inputs.energy_grid(wl.emin, wl.emax, wl.n_energies)
    V = torch.tensor(inputs.onsite(wl), device=dev)
    g = torch.tensor(inputs.dephasing(wl), device=dev)
    tE, tw = torch.tensor(E, device=dev), torch.tensor(w, device=dev)
    ws = M.allocate_workspace(sysm, wl.n_energies, dev)
    k = M.mc_negf_build_kernel(sysm, V, g, tE, ws)
    gws = torch.empty(M.mc_negf_grad_workspace_bytes(k), dtype=torch.uint8, device=dev)
    dV = torch.empty(wl.N, dtype=torch.float64, device=dev)
    dg = torch.empty_like(dV)
    for _ in range(max(1, warmup)):
        M.mc_negf_grad(k, 0, tw, gws, dV, dg)
    torch.cuda.synchronize()
    res = {}

    def one_grad():
        res["st"], res["I"] = M.mc_negf_grad(k, 0, tw, gws, dV, dg)

    with M.LaunchTimes() as lt0:
        one_grad()
    per_grad = len(require_complete(lt0).records)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    records = timed_records(steps, per_grad, one_grad)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    st, I = res["st"], res["I"]
    per_kernel = per_kernel_table(records, steps)
    adj_ms = per_kernel["adjoint_solve_kernel"]["ms_per_launch"]
    nbytes, flops = grad_work(wl)
    achieved = nbytes / 1e9 / (adj_ms * 1e-3)
    out = {
        "workload": f"W={wl.W} L={wl.L} N={wl.N}, eta={wl.eta}t, disorder U[-{wl.disorder},"
                    f"{wl.disorder}]t, {wl.n_energies} energies in [{wl.emin},{wl.emax}]t",
        "value": 1.0 / wall, "unit": "gradients/s (dI/dV_i for all N sites and dI/dgamma_i)",
        "ms_per_grad": 1e3 * wall, "I": I, "dI_deta": float(dg.sum().item()),
        "status": st, "per_kernel": per_kernel,
        "roofline": {"kernel": "adjoint_solve_kernel", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "algorithmic_per_launch": nbytes, "avg_launch_ms": adj_ms,
                     "fp64_tflops": flops / 1e12 / (adj_ms * 1e-3),
                     "traffic": measured_traffic("adjoint_solve_kernel", "diff_W16_L200")},
    }
    add_traffic_rate(out["roofline"])
    exact_V, exact_eta = dV.cpu().numpy(), float(dg.sum().item())
    del k, ws, gws
    torch.cuda.empty_cache()
    out["mc"] = grad_mc_bench(torch, dev, wl, V, g, tE, tw, exact_V, exact_eta)
    torch.cuda.empty_cache()
    out["w32"] = grad_w32_bench(torch, dev, steps)
    if with_cpu:
        # the oracle's reverse-mode dense adjoint on one of the energies, scaled to all of them
        from oracle import grad as OG
        import torch as _t
        j = wl.n_energies // 3
        t0 = time.perf_counter()
        OG.adjoint(wl.W, wl.L, wl.t, inputs.onsite(wl), inputs.dephasing(wl), E[j:j + 1],
                   w[j:j + 1])
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / (dt * wl.n_energies), "unit": "gradients/s",
                               "cores": _t.get_num_threads(), "kind": "oracle",
                               "sample": f"1 of {wl.n_energies} energies (dense torch adjoint, "
                                         f"{dt:.1f} s), scaled to all energies"}
    return out


def grad_mc_bench(torch, dev, wl, V, g, tE, tw, exact_V, exact_eta, walkers=100_000,
                  batches=4, seed=inputs.RNG_SEED):
    """The score-function gradient of the Monte Carlo current on the differentiation workload:
    per batch, walks with transition counts (mc_negf_walk_counts) and the gradient from them
    (mc_negf_grad_mc), against the exact adjoint gradient: dI/deta and the relative error of
    dI/dV over the sites, the spread over independent batches giving the standard error."""
    sysm = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead,
                         M.BUILD_NO_DIRECT)
    ws = M.allocate_workspace(sysm, wl.n_energies, dev)
    k = M.mc_negf_build_kernel(sysm, V, g, tE, ws)
    cnt = torch.zeros(M.mc_negf_walk_counts_bytes(k) // 4, dtype=torch.int32, device=dev)
    tal = torch.zeros((wl.n_energies, M.TALLY_N), dtype=torch.int64, device=dev)
    gws = torch.empty(M.mc_negf_grad_workspace_bytes(k), dtype=torch.uint8, device=dev)
    dV = torch.empty(wl.N, dtype=torch.float64, device=dev)
    dg = torch.empty_like(dV)
    etas, errs, walk_ms, grad_ms = [], [], [], []
    for b in range(batches):
        cnt.zero_()
        tal.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.mc_negf_walk_counts(k, seed, 0, 0, b * walkers, walkers, 1_000_000, cnt, tal)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        M.mc_negf_grad_mc(k, 0, cnt, tal, tw, gws, dV, dg)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        walk_ms.append(1e3 * (t1 - t0))
        grad_ms.append(1e3 * (t2 - t1))
        etas.append(float(dg.sum().item()))
        d = dV.cpu().numpy()
        errs.append(float(np.linalg.norm(d - exact_V) / np.linalg.norm(exact_V)))
    m, sd = float(np.mean(etas)), float(np.std(etas, ddof=1) / np.sqrt(batches))
    out = {"what": "score-function gradient of the Monte Carlo current: walks with transition "
                   "counts, then per-row block-tridiagonal solves of the count-weighted "
                   "adjoint (all sites), against the exact adjoint",
           "walkers_per_energy_per_batch": walkers, "batches": batches,
           "walk_counts_ms": float(np.median(walk_ms)), "grad_from_counts_ms":
               float(np.median(grad_ms)),
           "dI_deta_batches": etas, "dI_deta_mean": m, "dI_deta_stderr": sd,
           "dI_deta_exact": exact_eta, "dI_deta_err_in_sigma": (m - exact_eta) / sd if sd else None,
           "rel_l2_err_dI_dV_per_batch": errs}
    del k, ws, cnt, gws
    return out


def grad_w32_bench(torch, dev, steps, chunk=16):
    """The gradient at the paper's 32 x 32 blocks: W = 32, L = 130 (N = 4160), the
    differentiation workload's disorder, dephasing and 128 energies, differentiated in chunks
    of `chunk` energies (each chunk's G regenerated from the stored RGF blocks)."""
    wl = inputs.DIFF_W16_L200.replace(W=32, L=130)
    sysm = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead,
                         M.BUILD_NO_ALIAS)
    E, w = inputs.energy_grid(wl.emin, wl.emax, wl.n_energies)
    V = torch.tensor(inputs.onsite(wl), device=dev)
    g = torch.tensor(inputs.dephasing(wl), device=dev)
    tE, tw = torch.tensor(E, device=dev), torch.tensor(w, device=dev)
    ws = M.allocate_workspace(sysm, wl.n_energies, dev)
    k = M.mc_negf_build_kernel(sysm, V, g, tE, ws)
    nb = M.mc_negf_grad_workspace_bytes_chunk(k, chunk)
    gws = torch.empty(nb, dtype=torch.uint8, device=dev)
    dV = torch.empty(wl.N, dtype=torch.float64, device=dev)
    dg = torch.empty_like(dV)
    M.mc_negf_grad(k, 0, tw, gws, dV, dg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(max(1, min(steps, 3))):
        st, I = M.mc_negf_grad(k, 0, tw, gws, dV, dg)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / max(1, min(steps, 3))
    out = {"workload": f"W=32 L=130 N={wl.N}, eta={wl.eta}t, disorder U[-{wl.disorder},"
                       f"{wl.disorder}]t, {wl.n_energies} energies in [{wl.emin},{wl.emax}]t",
           "ms_per_grad": 1e3 * wall, "I": I, "status": st, "chunk_energies": chunk,
           "workspace_gb": nb / 1e9,
           "workspace_gb_all_energies_at_once": M.mc_negf_grad_workspace_bytes(k) / 1e9,
           "build_workspace_gb": ws.numel() / 1e9}
    del k, ws, gws
    torch.cuda.empty_cache()
    return out


def batched_bench(torch, dev, steps, warmup, budget_gb, seed):
    """The batched uneven workload: realizations planned into memory-bounded waves
    (mc_negf_plan_waves), each wave captured once as a HIP graph of its builds, one batched
    walk of all its (realization, energy) units with the autotuned launch shape, and the MC
    current of every realization; one step replays every wave's graph."""
    wls = inputs.batch_workloads()
    base = inputs.BATCH_W8
    flags = M.BUILD_NO_DIRECT  # Monte Carlo only
    systems = [M.make_system(w.W, w.L, w.t, w.lead_model, w.gamma_l, w.delta_lead, flags)
               for w in wls]
    nE, nw = base.n_energies, base.walkers_per_energy
    budget = int(budget_gb * (1 << 30))
    order, wave_of, n_waves = M.mc_negf_plan_waves(systems, nE, budget)
    sizes = [M.mc_negf_workspace_bytes(sm, nE) for sm in systems]
    waves = [[i for i in order if wave_of[i] == wv] for wv in range(n_waves)]
    pool_bytes = max(sum((sizes[i] + 255) // 256 * 256 for i in wv) for wv in waves)
    pool = torch.empty(pool_bytes, dtype=torch.uint8, device=dev)
    E, w = inputs.energy_grid(base.emin, base.emax, nE)
    tE, tw = torch.tensor(E, device=dev), torch.tensor(w, device=dev)
    V = [torch.tensor(inputs.onsite(wl), device=dev) for wl in wls]
    g = [torch.tensor(inputs.dephasing(wl), device=dev) for wl in wls]
    tal = [torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=dev) for _ in wls]
    T = [torch.empty(nE, dtype=torch.float64, device=dev) for _ in wls]
    sg = [torch.empty(nE, dtype=torch.float64, device=dev) for _ in wls]
    out = torch.zeros((len(wls), 2), dtype=torch.float64, device=dev)
    s = torch.cuda.Stream()
    plans = []
    cfg, tune_ms = None, None
    with torch.cuda.stream(s):
        for wv in waves:
            off, ks = 0, {}
            for i in wv:
                ws = pool[off:off + sizes[i]]
                off += (sizes[i] + 255) // 256 * 256
                ks[i] = (ws, M.mc_negf_build_kernel(systems[i], V[i], g[i], tE, ws, s))
            b = M.mc_negf_batch_prepare([ks[i][1] for i in wv], [wls[i].realization for i in wv],
                                        0, [tal[i] for i in wv], dev, s)
            if cfg is None:  # tune the launch shape once, on the first (largest) wave
                cfg, tune_ms = M.mc_negf_walk_batch_autotune(b, seed, max(1, nw // 10),
                                                             1_000_000, s)
            plans.append((wv, ks, b))
        graphs = []
        for wv, ks, b in plans:
            M.mc_negf_graph_begin(s)
            for i in wv:
                tal[i].zero_()
                M.mc_negf_build_kernel(systems[i], V[i], g[i], tE, ks[i][0], s)
            M.mc_negf_walk_batch(b, seed, 0, nw, 1_000_000, cfg, s)
            for i in wv:
                M.mc_negf_current_async(ks[i][1], 0, 0, tal[i], tw, T[i], sg[i], out[i], s)
            graphs.append(M.mc_negf_graph_end(s))
    try:
        for _ in range(max(1, warmup)):
            for gr in graphs:
                gr.launch(s)
        s.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in graphs]
        wave_ms = [0.0] * len(graphs)
        walk_steps = 0
        t0 = time.perf_counter()
        for _ in range(steps):
            for j, gr in enumerate(graphs):
                ev[j][0].record(s)
                gr.launch(s)
                ev[j][1].record(s)
            s.synchronize()
            for j in range(len(graphs)):
                wave_ms[j] += ev[j][0].elapsed_time(ev[j][1]) / steps
            walk_steps += int(sum(t[:, M.TALLY_STEPS].sum().item() for t in tal))
        wall = (time.perf_counter() - t0) / steps
    finally:
        for gr in graphs:
            gr.destroy()
    res = out.cpu().numpy()
    tally = np.stack([t.cpu().numpy() for t in tal])
    counts = dict(zip(*np.unique([wl.L for wl in wls], return_counts=True)))
    result = {
        "workload": f"{len(wls)} realizations x {nE} energies, W={base.W}, L drawn from "
                    f"{list(inputs.BATCH_LENGTHS)} (counts {dict((int(k), int(v)) for k, v in counts.items())}), "
                    f"eta={base.eta}t, disorder U[-{base.disorder},{base.disorder}]t, {nw} walkers/energy",
        "value": walk_steps / steps / wall, "unit": "walk steps/s",
        "ms_per_batch": 1e3 * wall, "waves": n_waves, "wave_ms": wave_ms,
        "wave_sizes": [len(wv) for wv in waves], "pool_gb": pool_bytes / 2 ** 30,
        "walk_config": cfg.as_dict(), "autotune_best_ms_at_tenth_walkers": tune_ms,
        "walkers": int(len(wls) * nE * nw), "steps_per_batch": walk_steps // steps,
        "truncated": int(tally[:, :, M.TALLY_TRUNC].sum()),
        "I_mc": [float(x) for x in res[:, 0]], "sigma_I_mc": [float(x) for x in res[:, 1]],
        "graph": "one captured graph per wave (builds, batched walk, MC currents), replayed",
    }
    del pool, plans
    torch.cuda.empty_cache()
    return result


def next_batch(done, I, s, first, cap):
    """Walkers for the next batch: the count that would bring sigma_I to 1% of I (sigma falls
    as 1 / sqrt(walkers)), with a 20% margin, at least `first`, at most cap - done."""
    if s > 0.0 and I != 0.0:
        want = int(1.2 * done * (s / (0.01 * abs(I))) ** 2) - done
    else:
        want = done
    return max(first, min(want, cap - done))


def time_to_1pct(p: Problem, torch, seed, walk_on):
    """Wall time to a 1% relative deviation of I, median of 5 warm repetitions.
    MC: build + a first batch of 1024 walkers per energy, then batches sized from the
    measured sigma_I until sigma_I <= 1% of I.
    MC, energy-sampled (the paper's estimator: energies drawn from the weights, constant
    estimator): build + a first batch of 4096 walkers over all energies, then likewise.
    MC, importance-sampled (Sec. V A, improved estimator): build without the plain tables +
    the modified tables of a ramp bias + a first batch of 256 walkers per energy, then
    likewise (the weights cut the variance per walker).
    DIRECT: build without alias tables + probe-system solve (deterministic; its error is the
    quadrature's).
    The stop is sigma_I / I <= 1%, a one-sigma rule: the realized deviation from the DIRECT
    current of the same system (|I_MC - I_DIRECT| / I_DIRECT, reported for every repetition)
    lies within 1% with probability about 0.68 and within 3% with probability about 0.997."""
    mc_t, dir_t, mc_walkers, smp_t, smp_walkers = [], [], [], [], []
    mc_I, smp_I = [], []
    wt_t, wt_walkers, wt_I, wt_sig = [], [], [], []
    itp_t, itp_walkers, itp_I, itp_nodes, itp_bias = [], [], [], None, None
    I_dir = None
    max_sampled = 1 << 24
    if walk_on and p.sampled_scratch is None:
        k0 = M.mc_negf_build_kernel(p.sys, p.V, p.g, p.E, p.ws)
        p.sampled_scratch = torch.empty(M.mc_negf_walk_sampled_bytes(k0, max_sampled),
                                        dtype=torch.uint8, device=p.E.device)
    if walk_on and p.weighted is None:
        p.weighted = weighted_setup(p, torch, max_sampled)
    for rep in range(5):
        if walk_on:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = M.mc_negf_build_kernel(p.sys, p.V, p.g, p.E, p.ws)
            p.tal.zero_()
            done, batch = 0, 1024
            while True:
                M.mc_negf_walk(k, seed + 1 + rep, 0, 0, done, batch, 1_000_000, p.tal)
                done += batch
                st, I, s = M.mc_negf_current(k, 0, 0, p.tal, p.w, p.T, p.sig)
                if s <= 0.01 * abs(I) or done >= 1 << 24:
                    break
                batch = next_batch(done, I, s, 1024, 1 << 24)
            mc_t.append(time.perf_counter() - t0)
            mc_walkers.append(done)
            mc_I.append(I)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = M.mc_negf_build_kernel(p.sys, p.V, p.g, p.E, p.ws)
            p.tal.zero_()
            done, batch = 0, 4096
            while True:
                M.mc_negf_walk_sampled(k, seed + 101 + rep, 0, 0, done, batch, 1_000_000, p.w,
                                       p.tal, p.sampled_scratch)
                done += batch
                st, I, s = M.mc_negf_current(k, 2, 0, p.tal, p.w, p.T, p.sig)
                if s <= 0.01 * abs(I) or done >= max_sampled:
                    break
                batch = next_batch(done, I, s, 4096, max_sampled)
            smp_t.append(time.perf_counter() - t0)
            smp_walkers.append(done)
            smp_I.append(I)
            # importance-sampled walks: build without the kernel's own tables, the modified
            # tables of the ramp bias, then batches until sigma_I <= 1% of I
            tables, bias, wscratch, wsum = p.weighted
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = M.mc_negf_build_kernel(p.sys_direct, p.V, p.g, p.E, p.ws)
            M.mc_negf_weighted_tables(k, bias, tables)
            p.tal.zero_()
            wsum.zero_()
            done, batch = 0, 256
            while True:
                M.mc_negf_walk_weighted(k, tables, bias, seed + 301 + rep, 0, 0, done, batch,
                                        1_000_000, p.tal, wsum, wscratch)
                done += batch
                st, I, s = M.mc_negf_current_weighted(k, 0, p.tal, wsum, p.w, p.T, p.sig)
                if s <= 0.01 * abs(I) or done >= max_sampled:
                    break
                batch = next_batch(done, I, s, 256, max_sampled)
            wt_t.append(time.perf_counter() - t0)
            wt_walkers.append(done)
            wt_I.append(I)
            wt_sig.append(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = M.mc_negf_build_kernel(p.sys_direct, p.V, p.g, p.E, p.ws)
        _, I_dir, _ = M.mc_negf_current(k, 1, 0, None, p.w, p.T, p.sig)
        dir_t.append(time.perf_counter() - t0)
        if walk_on:
            r = interp_mc(p, torch, seed + 201 + rep, 4, 1024, 1 << 24,
                          bias_walkers=(1_000_000 if rep == 0 else 0))
            itp_t.append(r[0])
            itp_walkers.append(r[1])
            itp_I.append(r[2])
            itp_nodes = r[4]
            if rep == 0:
                itp_bias = r[5:7]
    out = {"eta": p.wl.eta,
           "mc_ms": 1e3 * float(np.median(mc_t)) if mc_t else None,
           "mc_walkers_per_energy": int(np.median(mc_walkers)) if mc_walkers else None,
           "mc_energy_sampled_ms": 1e3 * float(np.median(smp_t)) if smp_t else None,
           "mc_energy_sampled_walkers": int(np.median(smp_walkers)) if smp_walkers else None,
           "direct_ms": 1e3 * float(np.median(dir_t)), "I_direct": I_dir}
    out.update(realized_errors(mc_I, smp_I, I_dir))
    if wt_t:
        out["mc_weighted"] = {
            "what": "importance-sampled walks (Sec. V A, improved estimator): step-6' rows "
                    f"reweighted by a ramp bias along the wire (contact length "
                    f"{WEIGHTED_RAMP_A:g} slices), scores = path likelihood ratios; build "
                    "without the plain tables",
            "ms": 1e3 * float(np.median(wt_t)),
            "walkers_per_energy": int(np.median(wt_walkers)),
            "rel_err_at_stop": [abs(v - I_dir) / abs(I_dir) for v in wt_I],
            "err_at_stop_in_sigma": [(v - I_dir) / sg for v, sg in zip(wt_I, wt_sig)]}
    if itp_t:
        out["mc_interpolated"] = {
            "what": "every 4th energy built (and the last), intervals whose rows differ by "
                    "more than 5% built exactly, all energies walked on interpolated rows",
            "ms": 1e3 * float(np.median(itp_t)),
            "walkers_per_energy": int(np.median(itp_walkers)),
            "built_energies": itp_nodes, "energies": int(p.E.numel()),
            "rel_err_at_stop": [abs(v - I_dir) / abs(I_dir) for v in itp_I],
            "I_at_1e6_walkers": itp_bias[0], "sigma_at_1e6_walkers": itp_bias[1],
            "bias_vs_direct_in_sigma": (itp_bias[0] - I_dir) / itp_bias[1],
            "rel_bias_vs_direct": (itp_bias[0] - I_dir) / I_dir}
    return out


def interp_mc(p: Problem, torch, seed, stride, walkers_first, cap, bias_walkers=0):
    """The interpolating Monte Carlo (Sec. V A, "Interpolation") on the wire's energy grid:
    build every stride-th energy (and the last) without alias tables, measure how far the
    normalised rows of neighbouring built energies differ, build exactly every energy inside
    an interval that differs by more than 5%, then walk all energies on the mixed rows of
    their neighbouring built energies in batches sized from sigma_I until sigma_I <= 1% of I.
    Returns (wall s, walkers per energy, I, sigma_I, built energies, tallies tensor)."""
    E = p.E.cpu().numpy()
    nE = len(E)
    coarse_idx = list(range(0, nE, stride)) + ([nE - 1] if (nE - 1) % stride else [])
    sys0 = M.make_system(p.wl.W, p.wl.L, p.wl.t, p.wl.lead_model, p.wl.gamma_l, p.wl.delta_lead,
                         M.BUILD_NO_ALIAS | M.BUILD_NO_DIRECT)
    sys1 = M.make_system(p.wl.W, p.wl.L, p.wl.t, p.wl.lead_model, p.wl.gamma_l, p.wl.delta_lead,
                         M.BUILD_NO_DIRECT)
    tc = p.E[coarse_idx].contiguous()
    dist = torch.empty(len(coarse_idx) - 1, dtype=torch.float64, device=p.E.device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    k0 = M.mc_negf_build_kernel(sys0, p.V, p.g, tc, p.ws)
    M.mc_negf_interp_distances(k0, dist)
    exact = M.mc_negf_interp_plan(E[coarse_idx], dist.cpu().numpy(), E, 0.05)
    nodes_idx = sorted(set(coarse_idx) | set(exact))
    tn = p.E[nodes_idx].contiguous()
    k1 = M.mc_negf_build_kernel(sys1, p.V, p.g, tn, p.ws)
    p.tal.zero_()
    done, batch = 0, walkers_first
    while True:
        M.mc_negf_walk_interp(k1, p.E, seed, 0, 0, done, batch, 1_000_000, p.tal)
        done += batch
        st, I, sI = M.mc_negf_current_interp(k1, p.E, 0, p.tal, p.w, p.T, p.sig)
        if sI <= 0.01 * abs(I) or done >= cap:
            break
        batch = next_batch(done, I, sI, walkers_first, cap)
    wall = time.perf_counter() - t0
    out = (wall, done, I, sI, len(nodes_idx))
    if bias_walkers:
        p.tal.zero_()
        M.mc_negf_walk_interp(k1, p.E, seed + 7, 0, 0, 0, bias_walkers, 1_000_000, p.tal)
        _, Ib, sIb = M.mc_negf_current_interp(k1, p.E, 0, p.tal, p.w, p.T, p.sig)
        out = out + (Ib, sIb)
    return out


WEIGHTED_RAMP_A = 10.0  # contact length (slices) of the ramp bias of the weighted walks


def weighted_setup(p: Problem, torch, max_walkers):
    """Buffers of the importance-sampled walks on p's wire: the modified tables, the ramp bias
    (the harmonic function of 1D diffusion from L to R, the same for every energy), walker
    scratch and the score sums."""
    dev = p.E.device
    k0 = M.mc_negf_build_kernel(p.sys_direct, p.V, p.g, p.E, p.ws)
    tables = torch.empty(M.mc_negf_weighted_tables_bytes(k0), dtype=torch.uint8, device=dev)
    b = torch.tensor(inputs.ramp_bias(p.wl.W, p.wl.L, WEIGHTED_RAMP_A), device=dev)
    bias = b.unsqueeze(0).repeat(p.wl.n_energies, 1).contiguous()
    scratch = torch.empty(M.mc_negf_walk_weighted_bytes(k0, max_walkers), dtype=torch.uint8,
                          device=dev)
    wsum = torch.zeros((p.wl.n_energies, 2), dtype=torch.float64, device=dev)
    return tables, bias, scratch, wsum


def realized_errors(mc_I, smp_I, I_dir):
    """|I_MC - I_DIRECT| / I_DIRECT at the 1% stop of every repetition, for both estimators."""
    out = {"stop_rule": "sigma_I / I <= 0.01 (one sigma: |error| <= 1% with p ~ 0.68, "
                        "<= 3% with p ~ 0.997)"}
    for key, vals in (("mc", mc_I), ("mc_energy_sampled", smp_I)):
        if vals and I_dir:
            errs = [abs(v - I_dir) / abs(I_dir) for v in vals]
            out[f"{key}_rel_err_at_stop"] = errs
            out[f"{key}_rel_err_at_stop_max"] = max(errs)
    return out


def scale_bench(torch, dev, warmup, with_cpu, seed, timed_batches=None, fp32=True):
    """The W=32 x L=500 wire (N = 16000, the paper's 32 x 32 blocks), all 512 energies in 16
    batches of SCALE_BATCH (batch b takes every 16th energy from b), one build per batch:
    build, 1e7 walks per energy, MC and DIRECT currents, all FP64.  Every batch is timed; the
    current of the whole grid is the sum of the batches' currents.  One energy's tables are
    1 GB, so here every walk step reads memory (no table stays in L2)."""
    wl = inputs.SCALE_W32_L500
    Eall, wall_w = inputs.energy_grid(wl.emin, wl.emax, wl.n_energies)
    n_batches = wl.n_energies // inputs.SCALE_BATCH
    picks = [np.arange(b, wl.n_energies, n_batches) for b in range(n_batches)]
    nE, nw = inputs.SCALE_BATCH, wl.walkers_per_energy
    sysm = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead)
    V = torch.tensor(inputs.onsite(wl), device=dev)
    g = torch.tensor(inputs.dephasing(wl), device=dev)
    tE = [torch.tensor(Eall[pk], device=dev) for pk in picks]
    tw = [torch.tensor(wall_w[pk], device=dev) for pk in picks]
    ws = M.allocate_workspace(sysm, nE, dev)
    tal = torch.zeros((n_batches, nE, M.TALLY_N), dtype=torch.int64, device=dev)
    T = torch.empty((n_batches, nE), dtype=torch.float64, device=dev)
    sg = torch.empty_like(T)
    Td = torch.empty_like(T)
    sgd = torch.empty_like(T)
    out = torch.zeros((n_batches, 2, 2), dtype=torch.float64, device=dev)
    holder = {}

    def one_batch(b, sysx=sysm):
        k = M.mc_negf_build_kernel(sysx, V, g, tE[b], ws)
        tal[b].zero_()
        M.mc_negf_walk(k, seed, 0, 0, 0, nw, 1_000_000, tal[b])
        M.mc_negf_current_async(k, 0, 0, tal[b], tw[b], T[b], sg[b], out[b, 0])
        M.mc_negf_current_async(k, 1, 0, None, tw[b], Td[b], sgd[b], out[b, 1])
        holder["k"] = k

    for _ in range(max(1, warmup)):
        one_batch(0)
    torch.cuda.synchronize()
    # one timing window per batch: a batch launches about 270 kernels (the factorization of
    # a 16000-row system is one launch per 64-column block) and a window records 512
    records = []
    flags = 0
    t0 = time.perf_counter()
    # (profiling runs may time fewer batches; the reported totals then cover those only)
    n_timed = n_batches if timed_batches is None else max(1, min(timed_batches, n_batches))
    for b in range(n_timed):
        with M.LaunchTimes() as lt:
            one_batch(b)
        records += require_complete(lt).records
        flags |= M.mc_negf_status(holder["k"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    o = out.cpu().numpy()[:n_timed]
    ta = tal.cpu().numpy()[:n_timed]
    walk_steps = int(ta[:, :, M.TALLY_STEPS].sum())
    per_kernel = per_kernel_table(records, n_timed)
    for v in per_kernel.values():
        v["ms_per_batch"] = v.pop("ms_per_step")
    walk_ms = per_kernel["walk_kernel"]["ms_per_batch"] * n_timed
    n_walk = per_kernel["walk_kernel"]["launches"]
    chol_ms = per_kernel["cholesky_kernel"]["ms_per_batch"]
    chol_flop = nE * (wl.N ** 3 / 3.0 + 2.0 * wl.N * wl.N)
    fi_ms = per_kernel["fullinv_kernel"]["ms_per_launch"]
    fi_flop = nE * 8.0 * wl.W ** 3 * wl.L * (wl.L - 1)
    I_mc, s_mc = float(o[:, 0, 0].sum()), float(np.sqrt(np.sum(o[:, 0, 1] ** 2)))
    I_d = float(o[:, 1, 0].sum())

    def per_batch_traffic(name, pk):
        t = measured_traffic(name, "scale_W32_L500")
        return None if t is None else t * pk[name]["launches"] / n_timed

    walk_roof = {"bound": "hbm", "achieved": walk_steps * STEP_BYTES / 1e9 / (walk_ms * 1e-3),
                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "algorithmic_per_launch": walk_steps * STEP_BYTES / n_walk,
                 "avg_launch_ms": walk_ms / n_walk,
                 "traffic": measured_traffic("walk_kernel", "scale_W32_L500")}
    walk_roof["frac"] = walk_roof["achieved"] / HBM_PEAK_GBS
    walk_roof.update(walker_entry_figures(walk_steps / n_walk, walk_ms / n_walk))
    res = {
        "workload": f"W={wl.W} L={wl.L} N={wl.N}, eta={wl.eta}t, disorder U[-{wl.disorder},"
                    f"{wl.disorder}]t, {wl.n_energies} energies in [{wl.emin},{wl.emax}]t in "
                    f"{n_batches} batches of {nE} ("
                    + ("all" if n_timed == n_batches else f"{n_timed}") + f" timed), {nw} "
                    "walkers/energy",
        "s_all_energies": wall if n_timed == n_batches else None,
        "batches_timed": n_timed,
        "ms_per_batch": 1e3 * wall / n_timed,
        "walk_steps": walk_steps,
        "walker_kernel_steps_per_s": walk_steps / (walk_ms * 1e-3),
        "mean_steps_per_walker": float(ta[:, :, M.TALLY_STEPS].sum() / ta[:, :, :3].sum()),
        "truncated": int(ta[:, :, M.TALLY_TRUNC].sum()),
        "I_direct": I_d, "I_mc": I_mc, "sigma_I_mc": s_mc,
        "mc_minus_direct_in_sigma": (I_mc - I_d) / s_mc if s_mc else None,
        "per_batch_mc_minus_direct_in_sigma": [float((o[b, 0, 0] - o[b, 1, 0]) / o[b, 0, 1])
                                               for b in range(n_timed)],
        "status_flags": int(flags),
        "per_kernel": per_kernel,
        "rooflines": {
            "walk_kernel": walk_roof,
            # the factorization is one launch per 64-column block: figures per batch
            "cholesky_kernel": {"bound": "mfma", "achieved": chol_flop / 1e12 / (chol_ms * 1e-3),
                                "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": chol_flop / 1e12 / (chol_ms * 1e-3) /
                                FP64_VALU_PEAK_TFLOPS, "algorithmic_per_batch": chol_flop,
                                "ms_per_batch": chol_ms,
                                "traffic_per_batch": per_batch_traffic("cholesky_kernel",
                                                                       per_kernel)},
            # the RGF block products of the full inverse (v_mfma_f64_16x16x4f64)
            "fullinv_kernel": {"bound": "mfma", "achieved": fi_flop / 1e12 / (fi_ms * 1e-3),
                               "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": fi_flop / 1e12 / (fi_ms * 1e-3) / FP64_VALU_PEAK_TFLOPS,
                               "algorithmic_per_launch": fi_flop, "avg_launch_ms": fi_ms,
                               "traffic": measured_traffic("fullinv_mfma_kernel",
                                                           "scale_W32_L500")},
        },
    }
    add_traffic_rate(res["rooflines"]["walk_kernel"])
    add_traffic_rate(res["rooflines"]["fullinv_kernel"])
    j = 1  # an energy of batch 0 away from the window's edge
    E0, w0 = Eall[picks[0]], wall_w[picks[0]]
    T64 = Td[0].cpu().numpy()
    I64 = float(o[0, 1, 0])
    T_gpu = float(T64[j])

    sweep64_ms = per_kernel.get("rgf_sweep_kernel", {}).get("ms_per_batch")

    def fp32_variant(flags, what):
        # batch 0 again, built with FP32 options (workspace as the flags need); errors against
        # the FP64 batch 0 above
        nonlocal ws
        need = M.mc_negf_workspace_bytes(M.make_system(wl.W, wl.L, wl.t, wl.lead_model,
                                                       wl.gamma_l, wl.delta_lead, flags), nE)
        if ws.numel() < need:
            del ws
            holder.clear()
            torch.cuda.empty_cache()
            ws = M.allocate_workspace(M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l,
                                                    wl.delta_lead, flags), nE, dev)
        sysx = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead, flags)
        one_batch(0, sysx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with M.LaunchTimes() as ltx:
            one_batch(0, sysx)
        torch.cuda.synchronize()
        wallx = time.perf_counter() - t0
        require_complete(ltx)
        ox = out.cpu().numpy()
        Tx = Td[0].cpu().numpy()
        r = {"what": what, "ms_per_batch": 1e3 * wallx,
             "fullinv_ms": ltx.total_ms("fullinv_kernel") +
             ltx.total_ms("fullinv_store_g_kernel"),
             "fullinv_ms_fp64": fi_ms,
             "rgf_sweep_ms": ltx.total_ms("rgf_sweep_kernel"), "rgf_sweep_ms_fp64": sweep64_ms,
             "refine_ms": ltx.total_ms("refine_kernel"),
             "max_rel_err_T_direct_vs_fp64": float(np.max(np.abs(Tx - T64) / np.abs(T64))),
             "rel_err_I_direct_vs_fp64": abs(float(ox[0, 1, 0]) - I64) / abs(I64),
             "mc_minus_fp64_direct_in_sigma": (float(ox[0, 0, 0]) - I64) / float(ox[0, 0, 1]),
             "status_flags": int(M.mc_negf_status(holder["k"])),
             "workspace_gb": ws.numel() / 1e9}
        return r, float(Tx[j])

    P, R, S = M.BUILD_FP32_PRODUCTS, M.BUILD_FP32_REFINE, M.BUILD_FP32_SWEEPS
    if not fp32:
        del holder, ws
        torch.cuda.empty_cache()
        return res
    res["fp32_products"], T_gpu32 = fp32_variant(
        P, "batch 0 with the full-inverse block products in FP32 on the matrix cores (FP64 RGF "
           "sweeps, |G|^2, alias tables, probe solve, tallies); no refinement")
    res["fp32_refined"], T_gpur = fp32_variant(
        P | R, "batch 0 with FP32 block products, then one FP64 refinement step on G (FP64 "
               "residual from the stencil, FP32 correction solve with the RGF blocks)")
    res["fp32_sweeps_refined"], T_gpus = fp32_variant(
        P | R | S, "batch 0 with FP32 RGF sweeps and FP32 block products, then one FP64 "
                   "refinement step on G")
    del holder, ws
    torch.cuda.empty_cache()
    if with_cpu:
        # the oracle's T_eff at one energy of batch 0: every column of G by a sparse LU,
        # then the dense probe system
        from oracle import columns as OC
        import threadpoolctl
        blas = max((i["num_threads"] for i in threadpoolctl.threadpool_info()), default=1)
        t0 = time.perf_counter()
        ora = OC.SparseEnergy(E0[j], wl.W, wl.L, wl.t, inputs.onsite(wl), inputs.dephasing(wl),
                              wl.lead_model, wl.delta_lead, wl.gamma_l)
        T_ref = ora.effective_transmission()
        dt = time.perf_counter() - t0
        del ora
        res["cpu_baseline"] = {
            "value": 1.0 / dt, "unit": "energies/s (DIRECT T_eff)", "cores": blas,
            "kind": "oracle",
            "sample": f"energy {E0[j]:.6f}t (1 of {wl.n_energies}): sparse LU columns (one "
                      f"thread) + dense probe solve ({blas} BLAS threads), {dt:.1f} s",
            "oracle_direct_s_projected_all_energies": dt * wl.n_energies,
            "T_oracle": T_ref, "T_gpu_direct": T_gpu,
            "rel_err_direct": abs(T_gpu - T_ref) / abs(T_ref),
            "rel_err_direct_fp32_products": abs(T_gpu32 - T_ref) / abs(T_ref),
            "rel_err_direct_fp32_refined": abs(T_gpur - T_ref) / abs(T_ref),
            "rel_err_direct_fp32_sweeps_refined": abs(T_gpus - T_ref) / abs(T_ref)}
    return res


def oracle_mc_to_1pct(K, c, w, seed, first=1024, cap=1 << 20):
    """The oracle's walker (the paper's cumulative-sum sampler) in batches sized from the
    measured sigma_I, as the GPU's time-to-1% runs, until sigma_I <= 1% of I: (walkers per
    energy, I, sigma_I, tallies)."""
    from oracle import walker as OW
    tal = np.zeros((K.shape[0], 5), np.int64)
    done, batch = 0, first
    while True:
        OW.walk_cdf(K, seed, 0, 0, done, batch, tallies=tal)
        done += batch
        _, _, I, sI = OW.mc_current(tal, c, w)
        if sI <= 0.01 * abs(I) or done >= cap:
            return done, I, sI, tal
        batch = next_batch(done, I, sI, first, cap)


def chain_bench(torch, dev, steps, warmup, seed, with_cpu):
    """The N = 50 chain (eta = 0.05 t, 64 midpoint energies in [-1.9 t, 1.9 t], 1e5 walkers
    per energy): one step = build, walks, MC and DIRECT currents, timed like the wire; time to
    1% for MC and DIRECT; the oracle's DIRECT solve and its MC to 1% on all 64 energies."""
    wl = inputs.CHAIN50
    p = Problem(wl, torch, dev)
    walkers = wl.walkers_per_energy
    for _ in range(max(1, warmup)):
        run_step(p, walkers, seed, True)
    torch.cuda.synchronize()
    with M.LaunchTimes() as lt0:
        run_step(p, walkers, seed, True)
    per_step = len(require_complete(lt0).records)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    records = timed_records(steps, per_step, lambda: run_step(p, walkers, seed, True))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st_mc, I_mc, s_mc, st_d, I_d = step_results(p, True)
    tal = p.tal.cpu().numpy()
    steps_total = steps * int(tal[:, M.TALLY_STEPS].sum())
    per_kernel = per_kernel_table(records, steps)
    walk_ms = per_kernel["walk_kernel"]["ms_per_step"] * steps
    out = {
        "workload": f"chain W=1 L={wl.L} N={wl.N}, eta={wl.eta}t, {wl.n_energies} energies in "
                    f"[{wl.emin},{wl.emax}]t, {walkers} walkers/energy",
        "value": steps_total / wall, "unit": "walk steps/s", "ms_per_step": 1e3 * wall / steps,
        "walker_kernel_steps_per_s": steps_total / (walk_ms * 1e-3),
        "I_mc": I_mc, "sigma_I_mc": s_mc, "status_mc": st_mc, "I_direct": I_d,
        "status_direct": st_d, "mc_minus_direct_in_sigma": (I_mc - I_d) / s_mc if s_mc else None,
        "mean_steps_per_walker": float(tal[:, 3].sum() / tal[:, :3].sum()),
        "per_kernel": per_kernel,
        "time_to_1pct": time_to_1pct(p, torch, seed, True),
    }
    # the same step captured once as a HIP graph and replayed: at N = 50 its dozen small
    # kernels take less time than their launches
    gs = torch.cuda.Stream(device=dev)  # default priority
    torch.cuda.synchronize()
    with torch.cuda.stream(gs):
        M.mc_negf_graph_begin(gs)
        run_step(p, walkers, seed, True)
        graph = M.mc_negf_graph_end(gs)
    try:
        for _ in range(max(1, warmup)):
            graph.launch(gs)
        gs.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.launch(gs)
        gs.synchronize()
        gwall = time.perf_counter() - t0
    finally:
        graph.destroy()
    g_mc, g_I, g_s, g_d, g_Id = step_results(p, True)
    out["graph"] = {"ms_per_step": 1e3 * gwall / steps, "value": steps_total / gwall,
                    "same_results": bool(g_I == I_mc and g_s == s_mc and g_Id == I_d),
                    "what": "one step captured as a HIP graph (build, walks, MC and DIRECT "
                            "currents) and replayed"}
    if with_cpu:
        from oracle import dense as D
        E, w = inputs.energy_grid(wl.emin, wl.emax, wl.n_energies)
        V, g = inputs.onsite(wl), inputs.dephasing(wl)
        t0 = time.perf_counter()
        sols = D.solve_workload(wl.W, wl.L, wl.t, V, g, E)
        I_ref = D.current(sols, w)
        t_dir = time.perf_counter() - t0
        t0 = time.perf_counter()
        sols = D.solve_workload(wl.W, wl.L, wl.t, V, g, E)
        K = np.stack([s_.transition_kernel() for s_ in sols])
        c = K[:, wl.N, :].sum(axis=1)
        n_mc, I_o, sI_o, otal = oracle_mc_to_1pct(K, c, w, seed)
        t_mc = time.perf_counter() - t0
        from oracle import walker as OW
        out["oracle"] = {
            "cores": OW.num_threads(), "I": I_ref,
            "rel_err_gpu_direct": abs(I_d - I_ref) / abs(I_ref),
            "direct_s": t_dir, "mc_to_1pct_s": t_mc, "mc_walkers_per_energy": n_mc,
            "mc_rel_err_at_stop": abs(I_o - I_ref) / abs(I_ref),
            "what": "dense LAPACK G per energy, transmissions and probe solve (DIRECT); the same "
                    "plus kernel rows and the C walker with the paper's cumulative-sum "
                    "sampler in batches until sigma_I <= 1% of I (MC); all 64 energies"}
    del p
    torch.cuda.empty_cache()
    return out


def inelastic_bench(torch, dev, steps, warmup, seed, with_cpu, walkers=None, ttp=True):
    """Inelastic walks (step 7') on the wire (W = 10, L = 100, eta = 0.05 t, 256 energies,
    1e6 walkers per energy) with an elastic line and optical-phonon emission / absorption lines
    8 grid steps away (inputs.PHONON_LINES / PHONON_WEIGHTS).  One step = build (no DIRECT
    workspace), step-7' table, walks, MC current and energy-resolved current; the walker's
    roofline counts 12 bytes per step plus the 8-byte thresholds a probe step compares."""
    wl = inputs.WIRE_W10_L100
    walkers = walkers or wl.walkers_per_energy
    nE, N = wl.n_energies, wl.N
    off, lam = list(inputs.PHONON_LINES), [float(x) for x in inputs.PHONON_WEIGHTS]
    sysm = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead,
                         M.BUILD_NO_DIRECT)
    E, w = inputs.energy_grid(wl.emin, wl.emax, nE)
    V = torch.tensor(inputs.onsite(wl), device=dev)
    g = torch.tensor(inputs.dephasing(wl), device=dev)
    tE = torch.tensor(E, device=dev)
    tw = torch.tensor(w, device=dev)
    ws = M.allocate_workspace(sysm, nE, dev)
    tal = torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=dev)
    hist = torch.zeros((2, nE, nE), dtype=torch.int64, device=dev)
    T = torch.empty(nE, dtype=torch.float64, device=dev)
    sg = torch.empty_like(T)
    out_I = torch.zeros(2, dtype=torch.float64, device=dev)
    S = torch.empty((2, nE), dtype=torch.float64, device=dev)
    state = {}

    def one_step():
        k = M.mc_negf_build_kernel(sysm, V, g, tE, ws)
        table = state.get("table")
        if table is None:
            table = state["table"] = torch.empty(M.mc_negf_energy_table_bytes(k, len(off)) // 8,
                                                 dtype=torch.int64, device=dev)
        M.mc_negf_energy_table(k, off, lam, table)
        tal.zero_()
        hist.zero_()
        M.mc_negf_walk_inelastic(k, off, table, seed, 0, 0, 0, walkers, 1_000_000, tal, hist)
        M.mc_negf_current_async(k, 0, 0, tal, tw, T, sg, out_I)
        M.mc_negf_spectrum(k, 0, tal, hist, tw, S)
        state["k"] = k

    for _ in range(max(1, warmup)):
        one_step()
    torch.cuda.synchronize()
    with M.LaunchTimes() as lt0:
        one_step()
    per_step = len(require_complete(lt0).records)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    records = timed_records(steps, per_step, one_step)
    torch.cuda.synchronize()
    k = state["k"]
    flags = M.mc_negf_status(k)
    t = tal.cpu().numpy()
    h = hist.cpu().numpy().astype(np.float64)
    I, sI = (float(x) for x in out_I.cpu().numpy())
    Sg = S.cpu().numpy()
    walk_steps = int(t[:, M.TALLY_STEPS].sum())
    exits = int(t[:, :2].sum())
    probe_steps = walk_steps - exits
    per_kernel = per_kernel_table(records, steps)
    walk_ms = per_kernel["walk_inelastic_kernel"]["ms_per_launch"]
    algo = STEP_BYTES * walk_steps + 8 * (len(off) - 1) * probe_steps
    roof = {"kernel": "walk_inelastic_kernel", "bound": "hbm",
            "achieved": algo / 1e9 / (walk_ms * 1e-3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "algorithmic_per_launch": algo, "avg_launch_ms": walk_ms,
            "bytes": f"{STEP_BYTES} per step + {8 * (len(off) - 1)} per probe step (thresholds)",
            "traffic": measured_traffic("walk_inelastic_kernel")}
    roof["frac"] = roof["achieved"] / HBM_PEAK_GBS
    add_traffic_rate(roof)
    # energy transfer: exit energy minus injection energy over the walks absorbed at R
    de = np.subtract.outer(np.arange(nE), np.arange(nE)).T * (E[1] - E[0])  # [e0][e]
    hR = h[1]
    elastic_R = float(np.trace(hR))
    out = {
        "workload": f"wire W={wl.W} L={wl.L} N={N}, eta={wl.eta}t, {nE} energies in "
                    f"[{wl.emin},{wl.emax}]t, {walkers} walkers/energy; step 7' with lines "
                    f"{off} grid steps (spacing {E[1] - E[0]:.4f}t), weights "
                    f"{[round(x, 4) for x in lam]}",
        "value": walk_steps / (wall / steps), "unit": "walk steps/s",
        "ms_per_step": 1e3 * wall / steps,
        "walker_kernel_steps_per_s": walk_steps / (walk_ms * 1e-3),
        "I_mc": I, "sigma_I_mc": sI,
        "I_spectrum_sum": float(Sg[1].sum()),
        "mean_steps_per_walker": walk_steps / float(t[:, :3].sum()),
        "mean_energy_change_at_R_t": float((hR * de).sum() / hR.sum()),
        "fraction_exits_at_R_with_changed_energy": 1.0 - elastic_R / float(hR.sum()),
        "status_flags": int(flags),
        "per_kernel": per_kernel,
        "roofline": roof,
    }
    # time to sigma_I <= 1% of I (median of 5 warm repetitions): build, step-7' table, then
    # batches of inelastic walks (1024 per energy first, then sized from sigma_I); the
    # realized deviation is measured against the 1e6-walker current above
    times, counts, devs = [], [], []
    table = state["table"]
    for rep in range(5 if ttp else 0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = M.mc_negf_build_kernel(sysm, V, g, tE, ws)
        M.mc_negf_energy_table(k, off, lam, table)
        tal.zero_()
        hist.zero_()
        done, batch = 0, 1024
        while True:
            M.mc_negf_walk_inelastic(k, off, table, seed + 1 + rep, 0, 0, done, batch, 1_000_000,
                                     tal, hist)
            done += batch
            _, Ib, sb = M.mc_negf_current(k, 0, 0, tal, tw, T, sg)
            if sb <= 0.01 * abs(Ib) or done >= 1 << 24:
                break
            batch = next_batch(done, Ib, sb, 1024, 1 << 24)
        times.append(time.perf_counter() - t0)
        counts.append(done)
        devs.append(abs(Ib - I) / abs(I))
    if ttp:
        out["time_to_1pct"] = {"mc_ms": 1e3 * float(np.median(times)),
                               "mc_walkers_per_energy": int(np.median(counts)),
                               "rel_dev_from_1e6_walker_current": devs,
                               "stop_rule": "sigma_I / I <= 0.01"}
    if with_cpu:
        out["cpu_baseline"] = inelastic_cpu_baseline(wl, off, lam, seed)
    del ws, state
    torch.cuda.empty_cache()
    return out


def resistance_bench(torch, dev, seed, walkers=100_000):
    """Linear-in-length resistance (Sec. IV A): clean W = 10 wires of L = 50, 100, 200, 400
    slices at eta = 0.1 t, 64 energies in [-3.5 t, 3.5 t]; per length the DIRECT current (build
    without alias tables plus the probe solve) and the Monte Carlo current (build plus walks),
    timed after one warm-up, then the straight line 1/I = a + b L through the DIRECT currents."""
    W, eta, nE = 10, 0.1, 64
    E, w = inputs.energy_grid(-3.5, 3.5, nE)
    tE = torch.tensor(E, device=dev)
    tw = torch.tensor(w, device=dev)
    rows = []
    for L in (50, 100, 200, 400):
        V = torch.zeros(W * L, dtype=torch.float64, device=dev)
        g = torch.full((W * L,), eta, dtype=torch.float64, device=dev)
        T = torch.empty(nE, dtype=torch.float64, device=dev)
        sg = torch.empty_like(T)
        rec = {"L": L}
        sys_d = M.make_system(W, L, flags=M.BUILD_NO_ALIAS)
        ws = M.allocate_workspace(sys_d, nE, dev)
        for timed in (False, True):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = M.mc_negf_build_kernel(sys_d, V, g, tE, ws)
            st, I, _ = M.mc_negf_current(k, 1, 0, None, tw, T, sg)
            if timed:
                rec.update(I_direct=I, status_direct=st,
                           direct_ms=1e3 * (time.perf_counter() - t0))
        del ws
        sys_m = M.make_system(W, L, flags=M.BUILD_NO_DIRECT)
        ws = M.allocate_workspace(sys_m, nE, dev)
        tal = torch.zeros((nE, M.TALLY_N), dtype=torch.int64, device=dev)
        for timed in (False, True):
            tal.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            k = M.mc_negf_build_kernel(sys_m, V, g, tE, ws)
            M.mc_negf_walk(k, seed, 0, 0, 0, walkers, 1_000_000, tal)
            st, I, sI = M.mc_negf_current(k, 0, 0, tal, tw, T, sg)
            if timed:
                t = tal.cpu().numpy()
                rec.update(I_mc=I, sigma_I_mc=sI, status_mc=st,
                           mc_ms=1e3 * (time.perf_counter() - t0),
                           mean_steps_per_walker=float(t[:, 3].sum() / t[:, :3].sum()))
        rec["mc_minus_direct_in_sigma"] = (rec["I_mc"] - rec["I_direct"]) / rec["sigma_I_mc"]
        rows.append(rec)
        del ws
        torch.cuda.empty_cache()
    Ls = np.array([r["L"] for r in rows], dtype=np.float64)
    R = np.array([1.0 / r["I_direct"] for r in rows])
    b, a = np.polyfit(Ls, R, 1)
    return {"workload": f"clean wires W={W}, L in {[r['L'] for r in rows]}, eta={eta}t, {nE} "
                        f"energies in [-3.5,3.5]t, {walkers} walkers/energy",
            "lengths": rows, "slope_per_slice": float(b), "contact_resistance": float(a),
            "max_rel_residual": float(np.abs(a + b * Ls - R).max() / R.min())}


def inelastic_cpu_baseline(wl, off, lam, seed, n_sample=16, nw=20_000):
    """The oracle's inelastic walker (C, the paper's cumulative-sum sampler) on n_sample
    consecutive energies of the wire's grid from the middle of the band, taken as a closed
    window (dense LAPACK rows and A_jj per energy): its rate in walk steps/s."""
    from oracle import dense as D
    from oracle import inelastic as IN
    from oracle import walker as OW
    E, _ = inputs.energy_grid(wl.emin, wl.emax, wl.n_energies)
    lo = wl.n_energies // 2 - n_sample // 2
    V, g = inputs.onsite(wl), inputs.dephasing(wl)
    t0 = time.perf_counter()
    sols = D.solve_workload(wl.W, wl.L, wl.t, V, g, E[lo:lo + n_sample])
    K = np.stack([s_.transition_kernel() for s_ in sols])
    A = np.stack([s_.Adiag for s_ in sols])
    table = IN.energy_table(A, off, lam)
    t_build = time.perf_counter() - t0
    t1 = time.perf_counter()
    tal, _, _ = IN.walk_cdf(K, table, off, seed, 0, 0, 0, nw)
    t_walk = time.perf_counter() - t1
    steps = int(tal[:, 3].sum())
    return {"value": steps / t_walk, "unit": "walk steps/s", "cores": OW.num_threads(),
            "kind": "oracle",
            "sample": f"energies {lo}..{lo + n_sample - 1} of {wl.n_energies} as a closed window "
                      f"x {nw} walkers: C walker, {steps} steps in {t_walk:.1f} s (dense rows "
                      f"and A_jj {t_build:.1f} s)",
            "build_s_per_energy": t_build / n_sample}


def cpu_baseline(wl: inputs.Workload, seed: int):
    """The oracle on the host cores for a bounded sample of the workload (about 10 s): dense
    LAPACK solves plus the C walker (the paper's cumulative-sum sampler), 24 of the 256
    energies with 25 000 walkers each, at the middle dephasing rate."""
    from oracle import dense as D
    from oracle import walker as OW
    E, _ = inputs.energy_grid(wl.emin, wl.emax, wl.n_energies)
    idx = np.linspace(0, wl.n_energies - 1, 24).round().astype(int)
    V, g = inputs.onsite(wl), inputs.dephasing(wl)
    nw = 25_000
    t0 = time.perf_counter()
    sols = D.solve_workload(wl.W, wl.L, wl.t, V, g, E[idx])
    t_solve = time.perf_counter() - t0
    K = np.stack([s.transition_kernel() for s in sols])
    t_kernel = time.perf_counter() - t0 - t_solve
    t1 = time.perf_counter()
    tal = OW.walk_cdf(K, seed, 0, 0, 0, nw)
    t_walk = time.perf_counter() - t1
    dt = time.perf_counter() - t0
    steps = int(tal[:, 3].sum())
    scale = wl.n_energies / len(idx)
    steps_per_walker = steps / (len(idx) * nw)
    return {"value": steps / dt, "unit": "walk steps/s", "cores": OW.num_threads(),
            "kind": "oracle",
            "sample": f"{len(idx)} of {wl.n_energies} energies x {nw} walkers at eta={wl.eta}: "
                      f"dense LAPACK G per energy + C walker (cumulative-sum sampler), "
                      f"{steps} steps in {dt:.1f} s",
            "walker_steps_per_s": steps / t_walk,
            "solve_s_per_energy": t_solve / len(idx),
            "kernel_rows_s_per_energy": t_kernel / len(idx),
            # projections of the sample to all energies (the whole oracle run takes minutes)
            "direct_s_projected": t_solve * scale,
            "mc_to_1pct_s_projected_1024_walkers": (t_solve + t_kernel) * scale +
            1024 * wl.n_energies * steps_per_walker / (steps / t_walk),
            "projection": f"sample times x {scale:.2f} energies; MC adds 1024 walkers per energy "
                          f"(the GPU's first batch, which reaches 1%) at the sample's walker rate"}


def calibration_copy(torch, dev, mib):
    """One plain device copy of `mib` MiB (read and written): the reference dispatch that
    scales the HBM byte counters of a profiled run."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.neg(src, out=dst)  # reads and writes n * 8 bytes
    torch.cuda.synchronize()
    del src, dst


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only (one GPU's share of the workload); use --gpus 1"}))
        sys.exit(2)
    import torch
    dev = "cuda:0"
    torch.cuda.set_device(0)
    if args.only:
        if args.calib_copy_mb > 0:
            calibration_copy(torch, dev, args.calib_copy_mb)
        with_cpu = not args.no_cpu_baseline
        if args.only == "grad":
            leg = grad_bench(torch, dev, args.steps, args.warmup, with_cpu)
        elif args.only == "chain":
            leg = chain_bench(torch, dev, args.steps, args.warmup, inputs.RNG_SEED, with_cpu)
        elif args.only == "resistance":
            leg = resistance_bench(torch, dev, inputs.RNG_SEED)
        elif args.only == "inelastic":
            leg = inelastic_bench(torch, dev, args.steps, args.warmup, inputs.RNG_SEED, with_cpu,
                                  ttp=not args.no_ttp)
        elif args.only == "batched":
            leg = batched_bench(torch, dev, args.steps, args.warmup, args.batch_budget_gb,
                                inputs.RNG_SEED)
        else:
            leg = scale_bench(torch, dev, args.warmup, with_cpu, inputs.RNG_SEED,
                              args.scale_batches, args.scale_batches is None)
        print(json.dumps({args.only: leg}), flush=True)
        return
    base = inputs.WIRE_W10_L100
    walkers = args.walkers or base.walkers_per_energy
    etas = [float(x) for x in args.etas.split(",")] if args.etas else list(inputs.WIRE_ETAS)
    probs = [Problem(base.replace(eta=eta), torch, dev) for eta in etas]
    seed = inputs.RNG_SEED
    walk_on = True

    for _ in range(args.warmup):
        for p in probs:
            run_step(p, walkers, seed, walk_on)
    torch.cuda.synchronize()
    if args.calib_copy_mb > 0:
        calibration_copy(torch, dev, args.calib_copy_mb)

    build_streams = [torch.cuda.Stream(device=dev) for _ in probs]  # default priority

    def one_step_serial():
        for p in probs:
            run_step(p, walkers, seed, walk_on)

    def one_step():
        if args.serial_builds:
            one_step_serial()
        else:
            run_step_overlapped(probs, build_streams, walkers, seed, walk_on)

    # launches per step, from one more untimed step
    with M.LaunchTimes() as lt0:
        one_step_serial()
    per_step = len(require_complete(lt0).records)
    # the timed steps run without the launch timer (its two events per launch slow a step by
    # about 9%); the same steps are then run again under the timer for the per-kernel figures,
    # with the builds issued one after another so that every launch's duration is its own
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t0 = time.perf_counter()
    records = timed_records(args.steps, per_step, one_step_serial)
    torch.cuda.synchronize()
    wall_instrumented = time.perf_counter() - t0
    # every step walks the same seeded walkers, so each step's counts are the last step's
    results = [(p, step_results(p, walk_on)) for p in probs]
    steps_total = args.steps * sum(int(p.tal[:, M.TALLY_STEPS].sum()) for p in probs) if walk_on else 0

    per_kernel = per_kernel_table(records, args.steps)
    names = sorted(per_kernel)
    dominant = max(names, key=lambda n: per_kernel[n]["ms_per_step"])
    n_walk = per_kernel.get("walk_kernel", {}).get("launches", 0)
    walk_steps_per_launch = steps_total / n_walk if (walk_on and n_walk) else 0
    roof = roofline(dominant, base, per_kernel[dominant]["ms_per_launch"], walk_steps_per_launch)
    if roof is not None:
        roof["traffic"] = measured_traffic(dominant)
        add_traffic_rate(roof)
    rooflines = {n: roofline(n, base, per_kernel[n]["ms_per_launch"], walk_steps_per_launch)
                 for n in names}
    per_eta = []
    for p, (st_mc, I_mc, s_mc, st_d, I_d) in results:
        rec = {"eta": p.wl.eta, "I_direct": I_d, "status_direct": st_d}
        if walk_on:
            tal = p.tal.cpu().numpy()
            rec.update({"I_mc": I_mc, "sigma_I_mc": s_mc, "status_mc": st_mc,
                        "mc_minus_direct_in_sigma": (I_mc - I_d) / s_mc if s_mc else None,
                        "mean_steps_per_walker": float(tal[:, 3].sum() / tal[:, :3].sum())})
        per_eta.append(rec)
    line = {
        "metric": "walk steps/s; time-to-1% lead-current error vs direct NEGF, 1 MI355X",
        "value": steps_total / wall,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "ms_per_step_with_launch_timer": 1e3 * wall_instrumented / args.steps,
        "per_kernel_timing": "every launch timed with HIP events, builds issued serially",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"wire W={base.W} L={base.L} N={base.N}, disorder "
                               f"U[-{base.disorder},{base.disorder}]t, {base.n_energies} "
                               f"energies in [{base.emin},{base.emax}]t, {walkers} walkers/energy,"
                               f" eta in {etas}t",
                   "walkers_per_energy": walkers, "n_energies": base.n_energies, "etas": etas,
                   "parallelism": "single GPU"},
        "per_eta": per_eta,
        "per_kernel": per_kernel,
        "roofline": roof,
        "rooflines": {n: r for n, r in rooflines.items() if r is not None},
    }
    if walk_on:
        line["walker_kernel_steps_per_s"] = steps_total / (
            per_kernel["walk_kernel"]["ms_per_step"] * args.steps * 1e-3)
    if not args.no_ttp:
        line["time_to_1pct"] = [time_to_1pct(p, torch, seed, walk_on) for p in probs]
    if not args.no_cpu_baseline:
        mid = probs[len(probs) // 2].wl
        line["cpu_baseline"] = cpu_baseline(mid, seed)
    del probs, results
    torch.cuda.empty_cache()
    if not args.no_chain:
        line["chain"] = chain_bench(torch, dev, args.steps, args.warmup, seed,
                                    not args.no_cpu_baseline)
    if not args.no_resistance:
        line["resistance"] = resistance_bench(torch, dev, seed)
    if not args.no_inelastic:
        line["inelastic"] = inelastic_bench(torch, dev, args.steps, args.warmup, seed,
                                            with_cpu=not args.no_cpu_baseline,
                                            ttp=not args.no_ttp)
    if not args.no_grad:
        line["grad"] = grad_bench(torch, dev, args.steps, args.warmup, not args.no_cpu_baseline)
    if not args.no_batched:
        line["batched"] = batched_bench(torch, dev, args.steps, args.warmup, args.batch_budget_gb,
                                        seed)
        torch.cuda.empty_cache()
    if not args.no_scale:
        line["scale"] = scale_bench(torch, dev, min(args.warmup, 1), not args.no_cpu_baseline,
                                    seed, args.scale_batches, args.scale_batches is None)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
