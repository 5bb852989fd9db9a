"""Benchmark of the Monte Carlo NEGF hot path on one MI355X.

One step = the whole path for the W=10 x L=100 disordered wire (N = 1000 sites, 256
midpoint energies in [-3.5 t, 3.5 t], disorder U[-0.25 t, 0.25 t]) at each dephasing rate
eta in {0.01, 0.05, 0.1} t: build G / kernel rows / alias tables for all 256 energies,
walk 1e6 walkers per energy, MC current, DIRECT current.  Inputs are resident in HBM
before the timed region starts.

Printed (rank 0, one JSON line): walk steps per second of the whole step (total walk steps
/ wall time of the step), per-stage times, the walker kernel's own rate and roofline, the
time to a 1% relative deviation of the lead current for MC and for the DIRECT GPU solve,
and the oracle timed on the host's cores for a bounded sample.
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
ALIAS_ENTRY_BYTES = 8        # one {thr, alias} pair read per walk step
WALKER_SRC = os.path.join(ROOT, "paper_1805_10164_amd", "csrc", "walker.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_kernel_wire_W10_L100_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--walkers", type=int, default=None, help="walkers per energy (default 1e6)")
    ap.add_argument("--etas", type=str, default=None, help="comma-separated dephasing rates")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ttp", action="store_true", help="skip the time-to-1%% measurement")
    return ap.parse_args()


class Problem:
    """Device-resident inputs and workspace for one dephasing rate."""

    def __init__(self, wl: inputs.Workload, torch, dev):
        self.wl = wl
        self.sys = M.make_system(wl.W, wl.L, wl.t, wl.lead_model, wl.gamma_l, wl.delta_lead)
        E, w = M.energy_grid(wl.emin, wl.emax, wl.n_energies)
        self.V = torch.tensor(inputs.onsite(wl), device=dev)
        self.g = torch.tensor(inputs.dephasing(wl), device=dev)
        self.E = torch.tensor(E, device=dev)
        self.w = torch.tensor(w, device=dev)
        self.ws = M.allocate_workspace(self.sys, wl.n_energies, dev)
        self.tal = torch.zeros((wl.n_energies, M.TALLY_N), dtype=torch.int64, device=dev)
        self.T = torch.empty(wl.n_energies, dtype=torch.float64, device=dev)
        self.sig = torch.empty_like(self.T)
        self.k = None


def run_step(p: Problem, torch, walkers, seed, ev):
    """Whole hot path for one problem; returns per-stage event pairs and results."""
    e0, e1, e2, e3, e4 = ev
    e0.record()
    p.k = M.mc_negf_build_kernel(p.sys, p.V, p.g, p.E, p.ws)
    e1.record()
    p.tal.zero_()
    M.mc_negf_walk(p.k, seed, p.wl.realization, 0, 0, walkers, 1_000_000, p.tal)
    e2.record()
    st_mc, I_mc, s_mc = M.mc_negf_current(p.k, 0, 0, p.tal, p.w, p.T, p.sig)
    e3.record()
    st_d, I_d, _ = M.mc_negf_current(p.k, 1, 0, None, p.w, p.T, p.sig)
    e4.record()
    return (st_mc, I_mc, s_mc, st_d, I_d)


def time_to_1pct(p: Problem, torch, seed):
    """Wall time to a 1% relative deviation of I: MC (build + doubling walker batches)
    and DIRECT (build + probe-system solve), each on a warm GPU, median of 5."""
    mc_t, dir_t, mc_walkers = [], [], []
    for rep in range(5):
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
            batch = done
        mc_t.append(time.perf_counter() - t0)
        mc_walkers.append(done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = M.mc_negf_build_kernel(p.sys, p.V, p.g, p.E, p.ws)
        M.mc_negf_current(k, 1, 0, None, p.w, p.T, p.sig)
        dir_t.append(time.perf_counter() - t0)
    return dict(mc_ms=1e3 * float(np.median(mc_t)), direct_ms=1e3 * float(np.median(dir_t)),
                mc_walkers_per_energy=int(np.median(mc_walkers)), eta=p.wl.eta)


def cpu_baseline(wl: inputs.Workload, seed: int):
    """The oracle on the host cores: dense solves plus the C walker (the paper's cumulative
    sampler) for a bounded sample of the workload: 8 of the 256 energies, 20 000 walkers
    each, at the middle dephasing rate."""
    from oracle import dense as D
    from oracle import walker as OW
    E, _ = M.energy_grid(wl.emin, wl.emax, wl.n_energies)
    idx = np.linspace(0, wl.n_energies - 1, 8).round().astype(int)
    V, g = inputs.onsite(wl), inputs.dephasing(wl)
    nw = 20_000
    t0 = time.perf_counter()
    sols = D.solve_workload(wl.W, wl.L, wl.t, V, g, E[idx])
    K = np.stack([s.transition_kernel() for s in sols])
    tal = OW.walk_cdf(K, seed, 0, 0, 0, nw)
    dt = time.perf_counter() - t0
    steps = int(tal[:, 3].sum())
    return {"value": steps / dt, "unit": "walk steps/s", "cores": OW.num_threads(),
            "kind": "oracle",
            "sample": f"{len(idx)} of {wl.n_energies} energies x {nw} walkers at eta={wl.eta}: "
                      f"dense LAPACK G per energy + C walker (cumulative-sum sampler), "
                      f"{steps} steps in {dt:.1f} s"}


def walker_traffic(walk_steps_per_launch):
    """HBM bytes per walker launch from the committed rocprofv3 counter summary, or None
    when the walker source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        src = hashlib.sha256(open(WALKER_SRC, "rb").read()).hexdigest()
        if rec.get("walker_sha256") != src:
            return None
        return float(rec["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}))
        sys.exit(2)
    import torch
    dev = "cuda:0"
    torch.cuda.set_device(0)
    base = inputs.WIRE_W10_L100
    walkers = args.walkers or base.walkers_per_energy
    etas = [float(x) for x in args.etas.split(",")] if args.etas else list(inputs.WIRE_ETAS)
    probs = [Problem(base.replace(eta=eta), torch, dev) for eta in etas]
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in probs]
    seed = inputs.RNG_SEED

    for _ in range(args.warmup):
        for p, e in zip(probs, ev):
            run_step(p, torch, walkers, seed, e)
    torch.cuda.synchronize()

    stage = np.zeros((len(probs), 4))
    steps_total = 0
    walker_launches = 0
    results = []
    t0 = time.perf_counter()
    for it in range(args.steps):
        for j, (p, e) in enumerate(zip(probs, ev)):
            res = run_step(p, torch, walkers, seed, e)
            torch.cuda.synchronize()
            stage[j] += [e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]),
                         e[2].elapsed_time(e[3]), e[3].elapsed_time(e[4])]
            steps_total += int(p.tal[:, M.TALLY_STEPS].sum())
            walker_launches += 1
            if it == args.steps - 1:
                results.append((p, res))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    per_eta = []
    for (p, res), st in zip(results, stage / args.steps):
        st_mc, I_mc, s_mc, st_d, I_d = res
        tal = p.tal.cpu().numpy()
        per_eta.append({"eta": p.wl.eta, "I_mc": I_mc, "sigma_I_mc": s_mc, "I_direct": I_d,
                        "mc_minus_direct_in_sigma": (I_mc - I_d) / s_mc if s_mc > 0 else None,
                        "status_mc": st_mc, "status_direct": st_d,
                        "mean_steps_per_walker": float(tal[:, 3].sum() / tal[:, :3].sum()),
                        "ms_build": st[0], "ms_walk": st[1], "ms_mc_current": st[2],
                        "ms_direct_current": st[3]})
    walk_ms = float(stage[:, 1].sum() / args.steps)
    steps_per_step = steps_total / args.steps
    walk_rate = steps_per_step / (walk_ms * 1e-3)
    avg_launch_s = walk_ms * 1e-3 / len(probs)
    bytes_per_launch = steps_per_step / len(probs) * ALIAS_ENTRY_BYTES
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic = walker_traffic(steps_per_step / len(probs))
    line = {
        "metric": "walk steps/s; time-to-1% lead-current error vs direct NEGF, 1 MI355X",
        "value": steps_total / wall,
        "unit": "walk steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"wire W={base.W} L={base.L} N={base.N}, disorder "
                               f"U[-{base.disorder},{base.disorder}]t, {base.n_energies} "
                               f"energies in [{base.emin},{base.emax}]t, {walkers} walkers/energy,"
                               f" eta in {etas}t",
                   "walkers_per_energy": walkers, "n_energies": base.n_energies,
                   "etas": etas, "parallelism": "single GPU"},
        "walker_kernel_steps_per_s": walk_rate,
        "per_eta": per_eta,
        "roofline": {"kernel": "walk_kernel", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "algorithmic_bytes_per_step": ALIAS_ENTRY_BYTES,
                     "avg_launch_ms": avg_launch_s * 1e3},
    }
    if not args.no_ttp:
        line["time_to_1pct"] = [time_to_1pct(p, torch, seed) for p in probs]
    if not args.no_cpu_baseline:
        mid = probs[len(probs) // 2].wl
        line["cpu_baseline"] = cpu_baseline(mid, seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
