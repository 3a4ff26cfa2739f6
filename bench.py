"""Benchmark: soft-sphere MD throughput in atom-steps/s on one MI355X.

Workload (default): the largest single system, N = 4 000 000 atoms (fcc
100^3 x 4), density 0.8, T = 1, truncated-shifted LJ at r_c = 2^(1/6),
neighbour shell 0.4 rebuilt by the displacement rule, dt = 0.005, FP32
forces on FP64 positions/velocities.  A "step" is one leapfrog time step of
the whole system: (a) kick+drift, (b) wrap/bin/reorder/neighbour build when
due, (c) forces, (d) kick, (e) properties and the rebuild decision.  Inputs
are synthetic (seeded fcc start with random velocity directions, melted for
200 untimed steps so that the timed steps see the fluid's steady rebuild
rate) and resident in HBM before timing; every replay graph is captured at
creation.

Prints ONE JSON line.  Besides the throughput it reports
  roofline      the step kernel k_step (forces, list build at rebuilds,
                integration, binning: the dominant kernel) against HBM
                bandwidth: algorithmic bytes per launch over its average
                duration, measured with HIP events around every launch on the
                library's stream in a second region of the same length;
  cpu_baseline  the FP64 CPU oracle timed on this host on a bounded sample of
                the same workload (one core), with the host's CPU model;
  batched       the replica workload (256 systems, N = 4 k^3, k ~ U{6..20},
                5000 steps) in one batch, against the same systems stepped
                one after another through the single-system path;
  served        a Poisson trace of the served workload (k ~ U{6..50}, 1000 to
                20 000 steps, 50 arrivals/s) through the serving loop.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "atom-steps/s soft-sphere ρ=0.8 (single vs batched); p50/p99 request latency"
TRAFFIC_FILES = {n: os.path.join(ROOT, "profiles", f"k_step_{n}_traffic.json")
                 for n in ("sp256000", "sp4000000", "sp33461708")}
KERNEL_SRC = os.path.join(ROOT, "paper_0911_5631_amd", "csrc", "md_kernels.hip")


def step_bytes_per_atom(mean_m: float, rebuild_frac: float) -> float:
    """Algorithmic HBM bytes per atom of one k_step launch.  A list step reads
    r_i and v_i (48), the list length (4) and the list (4 m) and writes
    r_i(t+dt) and v_i (48); a rebuild writes the list instead of reading it,
    plus the length and reads the atom's cell (8 more).  Neighbour
    coordinates count as cache hits (each is read once per step by the tile
    windows)."""
    return 100.0 + 4.0 * mean_m + 8.0 * rebuild_frac


def model_bytes_per_atom_step(mean_m: float, rebuild_frac: float) -> float:
    """Whole-step model (fused step + amortised sort and build): the fused
    step above, plus per rebuild the binning (read r 24, cell 8, counts ~3),
    the sorted scatter (52 read + 52 written) and the build (24 + 4 m + 4)."""
    per_rebuild = 24 + 8 + 3 + 104 + 24 + 4.0 * mean_m + 4
    return 100.0 + 4.0 * mean_m + rebuild_frac * per_rebuild


def kernel_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_per_launch(n_atoms: int):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary of this workload size, if it was taken on the current kernel
    source."""
    path = TRAFFIC_FILES.get(f"sp{n_atoms}")
    if path is None:
        return None
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_sha():
        return None
    return t.get("hbm_bytes_per_launch")


TUNE_CACHE = os.path.join(ROOT, "paper_0911_5631_amd", "tune_cache.json")


def gpu_arch() -> str:
    import torch
    return getattr(torch.cuda.get_device_properties(0), "gcnArchName", "gfx950")


def batched(n_replicas: int, steps: int, n_solo: int, solo_steps: int,
            tune_cache: str) -> dict:
    """Replicas of uneven size (N = 4 k^3, k ~ U{6..20}, rho ~ U[0.7, 0.9],
    T ~ U[0.8, 1.5]) advanced together in one batch, against the same
    systems run one after another through the single-system path.  The
    batch's launch configuration comes from the tuning cache (arch, batch,
    atom-count bucket) or, without an entry, from the autotuner on the run
    itself (its trial steps are part of the timed work).  The sequential
    comparator creates and warms every solo system (upload, first sort,
    graph capture) before its clock starts and times only its steps."""
    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd import tune as TU
    from paper_0911_5631_amd.md import Batch, System
    systems = I.replica_batch(n_replicas=n_replicas, steps=steps)
    atoms = int(sum(s.n for s in systems))
    work = float(sum(s.n * s.steps for s in systems))
    key = TU.cache_key(gpu_arch(), "batch", atoms)
    b = Batch(64 << 30, n_replicas, 64)
    t_adm = time.perf_counter()
    for s in systems:
        b.admit(s.pos, s.vel, s.box, s.steps, shell=s.shell, dt=s.dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cfg = TU.apply_cached(b, tune_cache, key)
    tuned = None
    if cfg is None:
        tuned = TU.autotune(b, runs=3, warm_runs=2, trial_steps=192, cache_path=tune_cache, key=key)
        cfg = tuned["in_use"]
    done = 0
    while done < n_replicas:
        b.run()
        for slot in b.poll():
            b.release(slot)
            done += 1
    el = time.perf_counter() - t0
    b.close()
    # one after another, each system alone (a sample of the same replicas):
    # created and warmed first, then only md_step + the synchronising props
    solo = []
    for s in systems[:n_solo]:
        sy = System(s.pos, s.vel, s.box, shell=s.shell, dt=s.dt)
        sy.step(8)
        sy.props()
        solo.append((sy, s.n))
    el_solo = 0.0
    solo_work = 0.0
    for sy, n in solo:
        t1 = time.perf_counter()
        sy.step(solo_steps)
        sy.props()
        el_solo += time.perf_counter() - t1
        solo_work += n * solo_steps
        sy.close()
    rate = work / el
    seq = solo_work / el_solo
    out = {"replicas": n_replicas, "atoms": atoms, "steps": steps,
           "atom_steps_per_s": rate, "seconds": el,
           "admission_seconds": t0 - t_adm,
           "sequential_atom_steps_per_s": seq,
           "sequential_sample": f"first {n_solo} replicas x {solo_steps} steps, each alone, "
                                "created and warmed before timing (md_step + props only)",
           "speedup_vs_sequential": rate / seq,
           "launch_config": cfg, "tune_key": key,
           "tune_source": "cache" if tuned is None else "autotuned on this run"}
    if tuned is not None:
        out["tune_trials"] = tuned["trials"]
    return out


def served(n_requests: int, rate: float, k_hi: int, steps_lo: int, steps_hi: int,
           budget_gb: float) -> dict:
    """A Poisson trace of requests served through one continuously refilled
    batch under an HBM budget: latency percentiles and aggregate rate."""
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.server import serve
    reqs = I.served_stream(n_requests=n_requests, rate=rate, k_hi=k_hi, steps_lo=steps_lo,
                           steps_hi=steps_hi)
    res = serve(reqs, int(budget_gb * (1 << 30)), max_slots=min(256, n_requests))
    out = {k: v for k, v in res.items() if k != "served"}
    out.update({"rate_per_s": rate, "k_range": [6, k_hi], "steps_range": [steps_lo, steps_hi],
                "hbm_budget_gb": budget_gb, "requests": n_requests})
    return out


def equilibrated(shell: float) -> dict:
    """The paper's system S run as in Table 4: the Sec. 5.1 equilibration
    (velocities adjusted every 20 steps during the first 500), then a block
    average over steps 1001-2000, all on the device; then 1000 plain steps
    (no block) for the cost of summing the properties every step."""
    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.md import System
    wl = I.system_s(shell)
    n = wl.n
    s = System(wl.pos, wl.vel, wl.box, shell=wl.shell, dt=wl.dt, precision=wl.precision,
               even_cells=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.equilibrate_run(1000, wl.temperature)
    s.props()
    t1 = time.perf_counter()
    s.block_begin()
    s.step(1000)
    blk = s.block_end()
    t2 = time.perf_counter()
    pr = s.props()
    t3 = time.perf_counter()
    s.step(1000)
    s.props()
    t4 = time.perf_counter()
    s.close()
    return {"workload": wl.name, "n_atoms": n, "shell": shell, "steps": 2000,
            "atom_steps_per_s": 2000 * n / (t2 - t0),
            "equilibration_atom_steps_per_s": 1000 * n / (t1 - t0),
            "block_atom_steps_per_s": 1000 * n / (t2 - t1),
            "plain_atom_steps_per_s": 1000 * n / (t4 - t3),
            "block": blk, "n_rebuilds_2000": pr["n_rebuilds"],
            "steps_per_rebuild": 2000 / max(pr["n_rebuilds"], 1), "max_cell": pr["max_cell"],
            "cells": pr["cells_per_edge"] ** 3,
            # the paper's values for this system (Table 4, N_step = 2000; Table 5)
            "paper": {"etot_per_atom": 2.3260603, "ke_per_atom": 1.5000234,
                      "nebr_per_atom": {0.4: 11.57, 0.5: 13.33, 0.6: 15.44, 0.7: 18.12,
                                        0.8: 21.64}.get(shell)}}


def lennard_jones(rc: float, n_edge: int, steps: int) -> dict:
    """The paper's LJ system (Sec. 5.1: rho 0.38, T 1.2, shell 0.8, simple cubic
    start) with cutoff rc, no shift: 500 steps of equilibration untimed, then
    `steps` timed steps."""
    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.md import System
    pos, L = I.sc_lattice(n_edge, 0.38)
    vel = I.random_velocities(len(pos), 1.2, 8)
    n = len(pos)
    s = System(pos, vel, L, r_cut=rc, shell=0.8, even_cells=True)
    s.equilibrate_run(500, 1.2)
    p0 = s.props()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    pr = s.props()
    el = time.perf_counter() - t0
    s.close()
    return {"r_cut": rc, "n_atoms": n, "cells": pr["cells_per_edge"] ** 3, "steps": steps,
            "atom_steps_per_s": n * steps / el, "us_per_atom_step": el / (n * steps) * 1e6,
            "mean_neighbours": 2.0 * pr["n_pairs"] / n,
            "steps_per_rebuild": steps / max(pr["n_rebuilds"] - p0["n_rebuilds"], 1),
            "pe_per_atom": pr["pe_per_atom"], "ke_per_atom": pr["ke_per_atom"]}


def no_reorder(marks=(2000, 10000, 100000)) -> dict:
    """Table 8's experiment: system S (shell 0.6, the Sec. 5.1 equilibration)
    run with and without reordering; atom-steps/s over the 1000 steps ending
    at each mark.  Without reordering the atoms keep their start order, which
    loses its spatial order as they diffuse."""
    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.md import System
    wl = I.system_s(0.6)
    n = wl.n
    out = {"workload": wl.name, "n_atoms": n, "marks": list(marks)}
    for name, reorder in (("reorder", True), ("no_reorder", False)):
        s = System(wl.pos, wl.vel, wl.box, shell=wl.shell, dt=wl.dt, even_cells=True,
                   reorder=reorder)
        s.equilibrate_run(500, wl.temperature)
        done = 500
        rates = []
        for m in marks:
            s.step(m - 1000 - done)
            s.props()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(1000)
            s.props()
            rates.append(1000 * n / (time.perf_counter() - t0))
            done = m
            print(f"# {name}: steps {m - 1000}-{m}: {rates[-1]:.4g} atom-steps/s",
                  file=sys.stderr, flush=True)
        s.close()
        out[name] = {"atom_steps_per_s": rates,
                     "us_per_atom_step": [1e6 / r for r in rates]}
    out["slowdown"] = [a / b for a, b in zip(out["reorder"]["atom_steps_per_s"],
                                             out["no_reorder"]["atom_steps_per_s"])]
    # the paper's FX770M figures (Table 8, us per atom-step without reordering)
    out["paper_no_reorder_us"] = {"1e3": 0.088, "1e5": 0.249}
    return out


def reorder_interval(intervals=(0, 50, 100, 250, 500, 1000, 2000), steps=6000) -> dict:
    """Table 7's experiment: system S (shell 0.6, the Sec. 5.1 equilibration),
    then ``steps`` timed steps with the reordering done at the first rebuild
    N_R steps after the last one (0: at every rebuild)."""
    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.md import System
    wl = I.system_s(0.6)
    n = wl.n
    rows = []
    for nr in intervals:
        s = System(wl.pos, wl.vel, wl.box, shell=wl.shell, dt=wl.dt, even_cells=True,
                   reorder_interval=nr)
        s.equilibrate_run(500, wl.temperature)
        p0 = s.props()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        p1 = s.props()
        el = time.perf_counter() - t0
        s.close()
        rows.append({"reorder_interval": nr, "atom_steps_per_s": n * steps / el,
                     "us_per_atom_step": el / (n * steps) * 1e6,
                     "rebuilds": p1["n_rebuilds"] - p0["n_rebuilds"]})
        print(f"# N_R {nr}: {rows[-1]['atom_steps_per_s']:.4g} atom-steps/s",
              file=sys.stderr, flush=True)
    # the paper's FX770M figures (Table 7, us per atom-step)
    paper = {50: 0.066, 100: 0.067, 250: 0.070, 500: 0.075, 1000: 0.081, 2000: 0.094}
    for r in rows:
        r["paper_us_per_atom_step"] = paper.get(r["reorder_interval"])
    return {"workload": wl.name, "n_atoms": n, "steps": steps, "rows": rows}


def no_window(steps=2000) -> dict:
    """The analogue of the paper's texture-cache experiment (Sec. 5): system
    S (shell 0.6, the Sec. 5.1 equilibration) with and without the LDS
    window, ``steps`` timed steps each."""
    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.md import System
    wl = I.system_s(0.6)
    n = wl.n
    out = {"workload": wl.name, "n_atoms": n, "steps": steps}
    for name, window in (("window", True), ("no_window", False)):
        s = System(wl.pos, wl.vel, wl.box, shell=wl.shell, dt=wl.dt, even_cells=True,
                   window=window)
        s.equilibrate_run(500, wl.temperature)
        s.props()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        s.props()
        el = time.perf_counter() - t0
        s.close()
        out[name] = {"atom_steps_per_s": n * steps / el, "us_per_atom_step": el / (n * steps) * 1e6}
        print(f"# {name}: {out[name]['atom_steps_per_s']:.4g} atom-steps/s", file=sys.stderr,
              flush=True)
    out["slowdown"] = out["window"]["atom_steps_per_s"] / out["no_window"]["atom_steps_per_s"]
    out["paper_texture_off_slowdown"] = 1.85
    return out


def newton3_ab(reps: int) -> dict:
    """The paper's neighbour-list trades on this GPU: at an evolved state of
    the 256k soft-sphere bench system and of the LJ r_c = 3.0 system (N_e =
    48), build a plain storage-index list full (atom by atom), half, or full
    cell by cell (one workgroup per cell, one thread per occupant: Table 3's
    "old" organisation), and time the builds and the force loop without
    reactions (full) and with atomic reactions (half); the production step
    kernel's launches are timed beside them."""
    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.md import System
    out = []
    sp = I.sp_256k()
    pos, L = I.sc_lattice(48, 0.38)
    cases = [("sp_256000", sp.pos, sp.vel, sp.box, dict(shell=0.4), 200, None),
             ("lj_rc3.0_110592", pos, I.random_velocities(len(pos), 1.2, 8), L,
              dict(r_cut=3.0, shell=0.8, even_cells=True), 500, 1.2)]
    for name, p, v, box, kw, warm, temp in cases:
        s = System(p, v, box, **kw)
        if temp:
            s.equilibrate_run(warm, temp)
        else:
            s.step(warm)
        s.props()
        s.profile(True)
        s.step(200)
        s.props()
        launches, ms = s.kernel_time()
        s.profile(False)
        pr = s.props()
        full = s.newton3_ab("full", reps)
        half = s.newton3_ab("half", reps)
        cells = s.newton3_ab("cells", reps)
        n = len(p)
        out.append({"system": name, "n_atoms": n, "pairs": pr["n_pairs"],
                    "full": {"build_us": full["build_ms"] * 1e3, "force_us": full["force_ms"] * 1e3,
                             "entries": full["n_entries"]},
                    "half": {"build_us": half["build_ms"] * 1e3, "force_us": half["force_ms"] * 1e3,
                             "entries": half["n_entries"]},
                    "cells": {"build_us": cells["build_ms"] * 1e3,
                              "force_us": cells["force_ms"] * 1e3,
                              "entries": cells["n_entries"]},
                    "half_over_full_force": half["force_ms"] / full["force_ms"],
                    "cells_over_full_build": cells["build_ms"] / full["build_ms"],
                    "step_kernel_mean_us": ms / max(launches, 1) * 1e3})
        s.close()
        torch.cuda.synchronize()
    return {"reps": reps, "cases": out}


def mixture(steps: int) -> dict:
    """A soft-sphere binary mixture of the bench size (inputs.mixture_256k)
    against the same start with one species: the cost of the per-pair
    parameters (species staged with the window, a table lookup per pair)."""
    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.md import System
    wl, species = I.mixture_256k()
    eps, sig, rc, sh = I.binary_wca()
    out = {}
    for name in ("mixture", "one_species"):
        s = System(wl.pos, wl.vel, wl.box, r_cut=float(rc.max()) if name == "mixture" else
                   I.RC_SOFT_SPHERE, shell=wl.shell, dt=wl.dt)
        if name == "mixture":
            s.set_species(species, eps, sig, rc, sh)
        s.step(200)
        p0 = s.props()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        pr = s.props()
        el = time.perf_counter() - t0
        s.close()
        out[name] = {"atom_steps_per_s": wl.n * steps / el,
                     "mean_neighbours": 2.0 * pr["n_pairs"] / wl.n,
                     "steps_per_rebuild": steps / max(pr["n_rebuilds"] - p0["n_rebuilds"], 1),
                     "pe_per_atom": pr["pe_per_atom"]}
    out["ratio"] = out["mixture"]["atom_steps_per_s"] / out["one_species"]["atom_steps_per_s"]
    out.update({"n_atoms": wl.n, "steps": steps, "species_b_fraction": 0.5,
                "sigma": sig.tolist(), "epsilon": eps.tolist()})
    return out


def _oracle_replica(args):
    """One replica stepped by the oracle in 25-step chunks for budget_s."""
    pos, vel, box, shell, dt, budget_s = args
    from oracle import oracle as O
    sim = O.Sim(pos, vel, box, shell=shell, dt=dt)
    steps = 0
    t0 = time.perf_counter()
    while True:
        sim.run(25)
        steps += 25
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    sim.close()
    return len(pos) * steps, el


def cpu_baseline_replicas(systems, budget_s: float) -> dict:
    """The oracle on the replica workload: independent replicas, one per host
    core (the oracle is single-threaded), each stepping for budget_s; the
    aggregate is the sum of their rates.  Runs before the GPU is touched."""
    from concurrent.futures import ProcessPoolExecutor
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    sample = systems[:cores]
    jobs = [(s.pos, s.vel, s.box, s.shell, s.dt, budget_s) for s in sample]
    with ProcessPoolExecutor(cores) as ex:
        res = list(ex.map(_oracle_replica, jobs))
    rate = sum(a / el for a, el in res)
    return {"value": rate, "unit": "atom-steps/s", "cores": cores, "kind": "oracle",
            "host": host_info(),
            "sample": f"replicas 1..{cores} of the batch (N {min(s.n for s in sample)}.."
                      f"{max(s.n for s in sample)}), one oracle process per core, "
                      f"{budget_s:.0f} s each from their starts"}


def host_info() -> dict:
    """The host the oracle ran on: CPU model, logical CPUs, CPUs this process
    may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(),
            "usable_cpus": len(os.sched_getaffinity(0))}


def cpu_baseline(sys_in, budget_s: float):
    """The FP64 oracle on this host: same system, steps from the start until
    the time budget is used (at least 50 steps).  Its state after the first
    25 steps is also set beside the GPU's after the same 25 steps, for the
    error of each output."""
    import numpy as np
    from oracle import oracle as O
    from paper_0911_5631_amd.md import System
    n = sys_in.n
    sim = O.Sim(sys_in.pos, sys_in.vel, sys_in.box, shell=sys_in.shell, dt=sys_in.dt)
    steps = 0
    t0 = time.perf_counter()
    parity = None
    while True:
        tr = sim.run(25)
        steps += 25
        el = time.perf_counter() - t0
        if parity is None:
            t_stop = time.perf_counter()
            rp, rv, rf, _ = sim.state()
            g = System(sys_in.pos, sys_in.vel, sys_in.box, shell=sys_in.shell, dt=sys_in.dt,
                       precision=sys_in.precision)
            g.step(25)
            gp, gv, gf, _ = g.get_state()
            pr = g.props()
            g.close()
            L = sys_in.box
            d = gp - rp
            d -= L * np.round(d / L)
            scale = np.maximum(np.linalg.norm(rf, axis=1), np.sqrt((rf ** 2).sum(1).mean()))
            parity = {
                "step": 25,
                "force_rel_err_max": float((np.linalg.norm(gf - rf, axis=1) / scale).max()),
                "pe_per_atom_abs_err": abs(pr["pe"] - tr[-1, 1]) / n,
                "virial_per_atom_abs_err": abs(pr["virial"] - tr[-1, 2]) / n,
                "ke_per_atom_abs_err": abs(pr["ke"] - tr[-1, 0]) / n,
                "position_abs_err_max": float(np.abs(d).max()),
                "velocity_abs_err_max": float(np.abs(gv - rv).max()),
                "pairs_equal": int(pr["n_pairs"]) == int(tr[-1, 4]),
                "pe_per_atom": tr[-1, 1] / n}
            t0 += time.perf_counter() - t_stop      # the comparison is not oracle time
            el = time.perf_counter() - t0
        if el >= budget_s and steps >= 50:
            break
    sim.close()
    return {"value": n * steps / el, "unit": "atom-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"N={n}, steps 1..{steps} from the fcc start ({el:.1f} s, one thread, "
                      f"FP64, linked-list cells + 14-cell half list + Newton's third law)",
            "host": host_info(), "parity": parity}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--melt", type=int, default=200,
                    help="untimed steps from the fcc start before the warm-up (input "
                         "preparation: the fluid's steady rebuild rate)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="launch-configuration cache to read (and to write when tuning)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="time budget of the CPU-oracle sample (0: skip)")
    ap.add_argument("--workload", default="sp_4m",
                    choices=["sp_256k", "sp_4m", "sp_33m", "sp_small", "batch", "served",
                             "equil", "lj", "newton3", "mixture", "tune", "noreorder"],
                    help="single system (default sp_4m); 'tune' autotunes the single-system "
                         "workloads' launch configuration into the cache; "
                         "'batch' / 'served' run only the full "
                         "batched-replica or served-stream workload and print its JSON line; "
                         "'equil' the paper's system S with equilibration and block averages; "
                         "'lj' the Lennard-Jones runs of Tables 1 and 3; 'newton3' the full- vs "
                         "half-list force A/B; 'mixture' a binary soft-sphere mixture")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the reduced batched and served sections of the default run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run one plain device copy of MIB MiB (a counter calibration "
                         "point for profilers), untimed")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: each system runs on a single MI355X "
              "(sharding a system over several GPUs is not implemented); run with --gpus 1",
              file=sys.stderr)
        return 2

    cpu_rep = None
    if args.workload == "batch" and args.cpu_seconds > 0:
        from paper_0911_5631_amd import inputs as I
        cpu_rep = cpu_baseline_replicas(I.replica_batch(n_replicas=256, steps=5000),
                                        args.cpu_seconds)
        print(f"# oracle on the replicas: {cpu_rep['value']:.4g} atom-steps/s on "
              f"{cpu_rep['cores']} cores", file=sys.stderr, flush=True)

    import torch
    from paper_0911_5631_amd import inputs as I
    from paper_0911_5631_amd.md import System

    torch.cuda.set_device(0)
    if args.workload == "tune":
        from paper_0911_5631_amd import tune as TU
        out = {}
        for make in (I.sp_256k, I.sp_4m):
            wl = make()
            s = System(wl.pos, wl.vel, wl.box, shell=wl.shell, dt=wl.dt, precision=wl.precision)
            s.step(args.melt)
            key = TU.cache_key(gpu_arch(), "single", wl.n)
            r = TU.autotune_system(s, wl.n, cache_path=args.tune_cache, key=key)
            out[wl.name] = {"key": key, "best": r["best"], "trials": r["trials"]}
            s.close()
            print(f"# tuned {wl.name}: {r['best']}", file=sys.stderr, flush=True)
        print(json.dumps({"metric": "launch-configuration autotuning", "value": None,
                          "unit": "atom-steps/s", "n_gpus": 1, "data": "synthetic",
                          "config": {"workload": "tune"}, "tune": out}), flush=True)
        return 0
    if args.workload == "batch":
        r = batched(256, 5000, 32, 1000, args.tune_cache)
        line = {"metric": "atom-steps/s, 256 batched replicas", "value": r["atom_steps_per_s"],
                "unit": "atom-steps/s", "n_gpus": 1, "higher_is_better": True,
                "data": "synthetic", "config": {"workload": "replica_batch_256"}, "batched": r}
        if cpu_rep:
            line["cpu_baseline"] = cpu_rep
        print(json.dumps(line), flush=True)
        return 0
    if args.workload == "served":
        r = served(256, 50.0, 50, 1000, 20000, 32.0)
        print(json.dumps({"metric": "served request latency p50/p99 and atom-steps/s",
                          "value": r["atom_steps_per_s"], "unit": "atom-steps/s", "n_gpus": 1,
                          "higher_is_better": True, "data": "synthetic",
                          "config": {"workload": "served_stream_256"}, "served": r}), flush=True)
        return 0
    if args.workload == "equil":
        r = equilibrated(0.6)
        print(json.dumps({"metric": "atom-steps/s, system S equilibrated with block averages",
                          "value": r["atom_steps_per_s"], "unit": "atom-steps/s", "n_gpus": 1,
                          "higher_is_better": True, "dtype": "fp32-force/fp64-state",
                          "data": "synthetic (seeded simple cubic start)",
                          "config": {"workload": r["workload"]}, "equil": r}), flush=True)
        return 0
    if args.workload == "lj":
        # Table 3: N_e = 48, r_c = 3.0 / 2.5 / 2.2; Table 1: N_e = 64, r_c = 3.0
        runs = [lennard_jones(rc, 48, 2000) for rc in (3.0, 2.5, 2.2)]
        runs.append(lennard_jones(3.0, 64, 2000))
        paper_us = {(3.0, 48): 0.270, (2.5, 48): 0.176, (2.2, 48): 0.137, (3.0, 64): 0.254}
        for r in runs:
            r["paper_us_per_atom_step"] = paper_us[(r["r_cut"], round(r["n_atoms"] ** (1 / 3)))]
        print(json.dumps({"metric": "atom-steps/s, Lennard-Jones rho 0.38 (r_c 3.0, N = 110 592)",
                          "value": runs[0]["atom_steps_per_s"], "unit": "atom-steps/s",
                          "n_gpus": 1, "higher_is_better": True, "dtype": "fp32-force/fp64-state",
                          "data": "synthetic (seeded simple cubic start)",
                          "config": {"workload": "lj_rc3.0_110592"}, "lj": runs}), flush=True)
        return 0
    if args.workload == "noreorder":
        r = no_reorder()
        ri = reorder_interval()
        nw = no_window()
        print(json.dumps({"metric": "atom-steps/s with and without reordering (Table 8)",
                          "value": r["no_reorder"]["atom_steps_per_s"][-1],
                          "unit": "atom-steps/s", "n_gpus": 1, "higher_is_better": True,
                          "dtype": "fp32-force/fp64-state",
                          "data": "synthetic (seeded simple cubic start)",
                          "config": {"workload": "no_reorder_" + r["workload"]},
                          "no_reorder": r, "reorder_interval": ri, "no_window": nw}),
              flush=True)
        return 0
    if args.workload == "mixture":
        r = mixture(4000)
        print(json.dumps({"metric": "atom-steps/s, binary soft-sphere mixture (N = 256 000)",
                          "value": r["mixture"]["atom_steps_per_s"], "unit": "atom-steps/s",
                          "n_gpus": 1, "higher_is_better": True,
                          "dtype": "fp32-force/fp64-state", "data": "synthetic",
                          "config": {"workload": "binary_wca_256000"}, "mixture": r}), flush=True)
        return 0
    if args.workload == "newton3":
        r = newton3_ab(50)
        print(json.dumps({"metric": "force-phase time, full list vs half list with atomics",
                          "value": r["cases"][0]["half_over_full_force"], "unit": "ratio",
                          "n_gpus": 1, "higher_is_better": False,
                          "dtype": "fp32-force/fp64-state", "data": "synthetic",
                          "config": {"workload": "newton3_ab"}, "newton3": r}), flush=True)
        return 0
    if args.calibrate_copy > 0:
        # a plain device-to-device copy of known size whose source is no
        # longer in the last-level cache (a 1 GiB buffer is written after it)
        nel = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        flush = torch.full((1 << 28,), 2.0, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst, flush
    wl = {"sp_256k": I.sp_256k, "sp_4m": I.sp_4m, "sp_33m": I.sp_33m,
          "sp_small": I.sp_small_cells}[args.workload]()
    n = wl.n
    s = System(wl.pos, wl.vel, wl.box, shell=wl.shell, dt=wl.dt, precision=wl.precision)
    print(f"# created {wl.name}: N={n} L={wl.box:.4f}", file=sys.stderr, flush=True)
    from paper_0911_5631_amd import tune as TU
    launch = TU.apply_cached(s, args.tune_cache, TU.cache_key(gpu_arch(), "single", n))
    # input preparation: the fcc start melts (its first rebuilds come late,
    # while every atom still moves at the initial speed)
    if args.melt > 0:
        s.step(args.melt)
        s.props()
    s.step(args.warmup)
    p0 = s.props()
    torch.cuda.synchronize()

    # timed region: K steps replayed from the captured step graphs
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    pr = s.props()                       # synchronises the library's stream
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    el = t1 - t0
    value = n * args.steps / el
    print(f"# timed {args.steps} steps in {el:.4f} s: {value:.4g} atom-steps/s",
          file=sys.stderr, flush=True)
    # second timed region of the same length with every force-kernel launch
    # bracketed by HIP events on the library's stream
    s.profile(True)
    t2 = time.perf_counter()
    s.step(args.steps)
    s.props()
    t3 = time.perf_counter()
    launches, kern_ms = s.kernel_time()
    s.profile(False)
    print(f"# profiled {args.steps} steps in {t3 - t2:.4f} s; force kernel {launches} launches, "
          f"{kern_ms / max(launches, 1) * 1e3:.2f} us avg", file=sys.stderr, flush=True)

    mean_m = 2.0 * pr["n_pairs"] / n
    rebuild_frac = (pr["n_rebuilds"] - p0["n_rebuilds"]) / args.steps
    avg_s = kern_ms * 1e-3 / max(launches, 1)
    bytes_launch = step_bytes_per_atom(mean_m, rebuild_frac) * n
    achieved = bytes_launch / avg_s / 1e9
    traffic = traffic_per_launch(n)
    model_b = model_bytes_per_atom_step(mean_m, rebuild_frac)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32-force/fp64-state" if wl.precision == "fp32" else "fp64",
        "data": "synthetic (seeded fcc start, random velocity directions)",
        "config": {"workload": wl.name, "n_atoms": n, "density": wl.rho,
                   "temperature": wl.temperature, "shell": wl.shell, "dt": wl.dt,
                   "box": wl.box, "parallelism": "single-gpu",
                   "start": f"fcc, melted {args.melt} untimed steps before the warm-up",
                   "launch_config": launch or "library default"},
        "roofline": {"bound": "hbm", "kernel": "k_step", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": bytes_launch,
                     "avg_launch_us": avg_s * 1e6, "launches": launches,
                     "profiled_region_atom_steps_per_s": n * args.steps / (t3 - t2),
                     "mean_neighbours": mean_m, "rebuild_fraction": rebuild_frac},
        "step_model": {"bytes_per_atom_step": model_b,
                       "roofline_atom_steps_per_s": HBM_PEAK_GBS * 1e9 / model_b,
                       "frac": value * model_b / (HBM_PEAK_GBS * 1e9)},
        "props": {"ke_per_atom": pr["ke_per_atom"], "pe_per_atom": pr["pe_per_atom"],
                  "n_rebuilds": pr["n_rebuilds"], "step": pr["step"]},
    }
    s.close()
    if not args.no_extras:
        # the replica workload at its full size (256 systems, 5000 steps) and
        # the served workload's distribution in a trace of 64 requests, so the
        # default run stays within minutes (256 requests: --workload served)
        out["batched"] = batched(256, 5000, 32, 1000, args.tune_cache)
        out["batched"]["single_system_atom_steps_per_s"] = value
        print(f"# batched: {out['batched']['atom_steps_per_s']:.4g} atom-steps/s "
              f"({out['batched']['speedup_vs_sequential']:.1f}x sequential)", file=sys.stderr,
              flush=True)
        out["served"] = served(64, 50.0, 50, 1000, 20000, 32.0)
        print(f"# served: p50 {out['served']['p50_latency_s']:.3f} s, p99 "
              f"{out['served']['p99_latency_s']:.3f} s, GPU busy "
              f"{out['served']['gpu_busy_fraction']:.3f}", file=sys.stderr, flush=True)
    if args.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
