"""Throughput of the short-range MD step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload lj1m|kg2m|kg1k]

Default workload: LJ fluid of 1,048,576 particles (FCC 64^3, density 0.8442,
uniform jitter 0.05, T = 0.72), rc = 2.5 shifted, skin 0.3, NVE dt = 0.005,
FP32 pair math, FP64 positions / velocities / reductions.  A "step" is one
pass of the whole hot path: gated cell sort + Verlet-list rebuild, fused
force + velocity-Verlet kernel, FP64 energy/virial reduction.  Inputs are
resident in HBM before the timed region.

Prints one JSON line with the metric, a "roofline" object for the dominant
(fused force+integrate) kernel, timed with HIP events on the library's
stream over the timed region, and a "cpu_baseline" object: the FP64 oracle
timed on this host on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per atom-step of the plain method (half Verlet list in
# int32, compulsory FP64 x/v streams, FP32 force), per workload:
#   LJ 1M:  NL 4 + 38.8*4 = 159, positions 24, force 12, integration 132 -> 327
#   KG 2M:  NL 4 + 6.3*4 = 29, positions 24, force 12, topology 16,
#           integration 132 -> 213
#   surrogate 1M: 2 descriptor-list passes 2 x (4 + 43.4 x 4) = 355, a_i write
#           + read 256, positions 48, force 12, bonded 16, integration 132 -> 819
ALG_BYTES = {"lj1m": 327.0, "kg2m": 213.0, "kg1k": 213.0, "sur1m": 819.0}
# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (scaled by a 512 MiB copy: x2.0 and x1.0), valid only for
# the kernel source they were taken on (SHA-256 prefix of md_kernels.hip).
TRAFFIC = {"lj1m": {"bytes": 226635.5 * 2.0 * 1024 + 87480.0 * 1024, "source": "8c23e66d09ea82f3"},
           "kg2m": {"bytes": 232674.2 * 2.0 * 1024 + 174642.0 * 1024, "source": "8c23e66d09ea82f3"}}


def kernel_source_hash():
    import hashlib
    p = os.path.join(ROOT, "paper_2608_14911_amd", "csrc", "md_kernels.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="lj1m", choices=["lj1m", "kg2m", "kg1k", "batch", "sur1m"])
    ap.add_argument("--sur-precision", default="bf16", choices=["fp32", "bf16"],
                    help="sur1m: network precision of the surrogate")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch: keep the sampler's skin and the library's automatic cells and list build")
    ap.add_argument("--no-events", action="store_true",
                    help="time with a hipGraph replay and no per-kernel events")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--cell-factor", type=int, default=0, help="cells per list radius (1 or 2; 0 = library default)")
    ap.add_argument("--nl-build", default="auto", choices=["auto", "tiles", "per-particle"],
                    help="Verlet-list build: one wavefront per 64-particle tile, one particle per lane, "
                         "or the library's choice by cell occupancy")
    ap.add_argument("--calib-copy", action="store_true",
                    help="after the run, copy 512 MiB three times (torch copy kernel) so that hardware "
                         "byte counters can be scaled against a transfer of known size")
    return ap.parse_args()


def log(msg, quiet=False):
    if not quiet:
        print("[bench] " + msg, file=sys.stderr, flush=True)


def make_system(name, quiet, cell_factor=0, flags=0):
    from paper_2608_14911_amd import inputs
    from paper_2608_14911_amd.system import from_workload
    if name == "lj1m":
        w = inputs.workload_lj(ncell=64, seed=1001)
        s = from_workload(w, precision="fp32", cell_factor=cell_factor, flags=flags)
        return w, s
    if name == "kg2m":
        w = inputs.workload_kg(2000, 1000, seed=1002)
    elif name == "sur1m":
        w = inputs.workload_kg(1000, 1000, seed=1014)
    else:
        w = inputs.workload_kg1k()
        w["k_bend"] = 1.5
    # push-off on the GPU (capped WCA ladder, then uncapped), then the run
    # parameters of the workload.  Raw random walks overlap, so the push-off
    # list needs a large capacity; the timed system is re-created from the
    # pushed-off state with the capacity sized from the density.
    from paper_2608_14911_amd.system import push_off
    w0 = dict(w)
    w0["caprad"] = 1.0
    w0["dt"] = 0.002
    w0["gamma"] = 1.0
    w0["vel"] = np.zeros_like(w["pos"])
    s = from_workload(w0, precision="fp32", cell_factor=cell_factor, nl_capacity=256, flags=flags)
    t0 = time.time()
    push_off(s, w["rc"], log=lambda m: log(m, quiet))
    s.set_params(dt=w["dt"], gamma=w["gamma"])
    s.step(200)
    st = s.get_state()
    s.close()
    w1 = dict(w)
    w1["pos"], w1["vel"] = st["pos"], st["vel"]
    extra = {"list_cutoff": 2.5, "surrogate": True} if name == "sur1m" else {}
    s = from_workload(w1, precision="fp32", cell_factor=cell_factor, flags=flags, **extra)
    s.set_state(st)
    s.step(1)
    if s.status() != 0:
        raise RuntimeError("KG system after push-off: status %d" % s.status())
    log("push-off done in %.1f s" % (time.time() - t0), quiet)
    return w1, s


def cpu_baseline(w, name, budget_s, quiet):
    """The FP64 oracle (linked cells, OpenMP) on this host, on a bounded
    number of steps of the same workload; extrapolated to atom-steps/s."""
    import oracle
    n = w["pos"].shape[0]
    st = {"pos": w["pos"].copy(), "vel": w["vel"].copy(), "image": np.zeros((n, 3), dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    par = {"box": w["box"], "pp": oracle.pair_params(w["eps"], w["sigma"], w["rc"], w["shift"], 0.0),
           "ntypes": 1, "mass_by_type": np.array([1.0]), "dt": w["dt"],
           "integrator": oracle.LANGEVIN if w["integrator"] == "langevin" else oracle.NVE,
           "temperature": w["temperature"], "gamma": w["gamma"], "seed": w["seed"],
           "bonds": w.get("bonds"), "angles": w.get("angles"), "k_bend": w.get("k_bend", 0.0)}
    threads = oracle.nthreads_default()
    t0 = time.time()
    oracle.run(st, par, 1)          # untimed: first touch
    t1 = time.time()
    oracle.run(st, par, 1)
    one = time.time() - t1
    k = max(1, min(50, int(budget_s / max(one, 1e-6))))
    t2 = time.time()
    oracle.run(st, par, k)
    el = time.time() - t2
    steps = k + 1
    secs = el + one
    log("cpu oracle: %d steps in %.2f s on %d threads (setup %.1f s)" % (steps, secs, threads, t1 - t0), quiet)
    return {"value": n * steps / secs, "unit": "atom-steps/s", "cores": threads, "kind": "oracle",
            "sample": "%d steps of the same %d-particle workload (FP64 linked cells, OpenMP), "
                      "after 1 untimed step" % (steps, n)}


def member_alg_bytes(m, n, skin):
    """Algorithmic bytes per atom-step of one member: half Verlet list
    (int32) at its density and list radius, FP64 x / v streams, FP32 force,
    topology for melts."""
    rc = m["pair"][(0, 0)][2]
    rv = rc + skin
    rho = n / float(m["box"][0]) ** 3
    half = rho * 2.0 / 3.0 * math.pi * rv ** 3
    return 4 + 4 * half + 24 + 12 + 132 + (16 if m.get("kind") == "kg" else 0)


def bench_batch(a):
    import torch
    from paper_2608_14911_amd import autotune, inputs
    from paper_2608_14911_amd.system import Batch, System, lj_pair, nl_build_flags, prepare_replica
    t0 = time.time()
    reps = inputs.batch_replicas(256, seed=1003)
    out = []
    for k, r in enumerate(reps):
        out.append(prepare_replica(r))
        if k % 32 == 31:
            log("replicas prepared: %d / %d (%.0f s)" % (k + 1, len(reps), time.time() - t0), a.quiet)
    reps = out
    if a.no_autotune:
        choice = {"lj": (0.3, 0, "auto"), "kg": (0.4, 0, "auto")}
        table = []
    else:
        choice, table = autotune.tune(reps, steps=30, log=lambda m: log(m, a.quiet))
    reps = autotune.apply(reps, choice)
    ntot = sum(r["pos"].shape[0] for r in reps)
    b = Batch(reps)
    b.step(a.warmup)
    o0 = b.observables()
    b.timing(True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    b.step(a.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - ts
    tm = b.timing()
    b.timing(False)
    o1 = b.observables()
    b.close()
    # the same members one by one (graph-replayed standalone handles)
    t_sum = 0.0
    for r in reps:
        s = System(r["pos"], r["box"], r["vel"], pair=r["pair"], bonds=r.get("bonds"), angles=r.get("angles"),
                   k_bend=r.get("k_bend", 0.0), dt=r["dt"], skin=r["skin"], integrator=r["integrator"],
                   temperature=r["temperature"], gamma=r["gamma"], seed=r["seed"], cell_factor=r["cell_factor"],
                   flags=nl_build_flags(r["nl_build"]))
        s.step(4)
        s.stream.synchronize()
        t1 = time.perf_counter()
        s.step(20)
        s.stream.synchronize()
        t_sum += (time.perf_counter() - t1) / 20
        s.close()
    value = ntot * a.steps / el
    k_ms = tm["ms_step_kernels"] / max(tm["n_step_kernels"], 1)
    alg = sum(member_alg_bytes(r, r["pos"].shape[0], r["skin"]) * r["pos"].shape[0] for r in reps)
    ach = alg / (k_ms * 1e-3) / 1e9
    rec = {
        "metric": "atom-steps/s (1M LJ, 2M KG melt)",
        "value": value, "unit": "atom-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "batch of 256 replicas (128 LJ fluids, 128 polymer melts), %d particles" % ntot,
                   "n_particles": ntot, "replicas": len(reps), "sizes": "log-uniform 2048..65536",
                   "precision": "FP32 pair/bonded math, FP64 positions, velocities and reductions",
                   "parallelism": "single GPU",
                   "autotuned": {k: {"skin": v[0], "cell_factor": v[1] or "auto", "nl_build": v[2]}
                                 for k, v in choice.items()}},
        "standalone_sum_atom_steps_per_s": ntot / t_sum,
        "batched_over_standalone": value / (ntot / t_sum),
        "n_rebuilds_total": sum(x["n_rebuilds"] - y["n_rebuilds"] for x, y in zip(o1, o0)),
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_batch_step (fused forces + integration, all replicas)", "kernel_ms": k_ms,
                     "alg_bytes_per_launch": alg},
        "kernel_breakdown_ms_per_step": {
            "rebuild_stage": tm["ms_rebuild"] / max(tm["n_rebuild"], 1), "step_kernel": k_ms,
            "finalize": tm["ms_finalize"] / max(tm["n_finalize"], 1)},
        "autotune_trials": table,
    }
    if not a.no_cpu_baseline:
        w = dict(reps[0])
        eps, sig, rc, shift, cap = w["pair"][(0, 0)]
        w.update({"eps": eps, "sigma": sig, "rc": rc, "shift": shift})
        rec["cpu_baseline"] = cpu_baseline(w, "batch", a.cpu_seconds, a.quiet)
        rec["cpu_baseline"]["sample"] += " (replica 0 of the batch)"
    print(json.dumps(rec), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.workload == "batch":
        return bench_batch(a)
    from paper_2608_14911_amd import md as md_
    nl_flags = {"auto": 0, "tiles": md_.MD_CFG_NL_TILES, "per-particle": md_.MD_CFG_NL_PER_PARTICLE}[a.nl_build]
    w, s = make_system(a.workload, a.quiet, a.cell_factor, nl_flags)
    n = s.n
    if a.workload == "sur1m":
        # the surrogate replaces the WCA pair force: the network trained by
        # surrogate_experiment.py on a 100k-bead plain-method melt (without
        # excluded volume from a trained network the FENE bonds collapse the
        # chains, so random weights cannot be timed over many steps)
        wpath = os.path.join(ROOT, "paper_2608_14911_amd", "data", "surrogate_kg.npz")
        if not os.path.exists(wpath):
            raise SystemExit("missing %s: python -m paper_2608_14911_amd.surrogate_experiment --save %s"
                             % (wpath, wpath))
        wd = np.load(wpath)
        s.sur_set(wd["theta_" + a.sur_precision], wd["g_mean"], wd["g_istd"], a.sur_precision)
        s.set_pair_mode("surrogate")
    s.step(a.warmup)
    o0 = s.observables()
    s.history()
    timing = not a.no_events
    if timing:
        s.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(a.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = s.timing() if timing else None
    if timing:
        s.timing(False)
    o1 = s.observables()
    hist = s.history()
    value = n * a.steps / el
    ms = 1e3 * el / a.steps
    from paper_2608_14911_amd import md as md_
    plan = md_.md_plan_config(s.cfg)
    rec = {
        "metric": "atom-steps/s (1M LJ, 2M KG melt)" if a.workload != "sur1m" else
                  "atom-steps/s (1M KG melt, learned surrogate pair force)",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w["name"], "n_particles": n, "rc": w["rc"], "skin": w["skin"],
                   "dt": w["dt"], "integrator": w["integrator"],
                   "precision": "FP32 pair/bonded math, FP64 positions, velocities and reductions",
                   "parallelism": "single GPU", "cell_factor": plan["cell_factor"],
                   "cells_per_side": plan["cells"][0], "list_build": plan["nl_build"],
                   "list_capacity": plan["nl_capacity"]},
        "n_rebuilds": o1["n_rebuilds"] - o0["n_rebuilds"],
        "energy_drift_per_particle": (o1["e_total"] - o0["e_total"]) / n,
        "nl_max_count": o1["nl_max_count"],
    }
    if tm:
        k_ms = tm["ms_step_kernels"] / max(tm["n_step_kernels"], 1)
        alg = ALG_BYTES[a.workload] * n
        ach = alg / (k_ms * 1e-3) / 1e9
        tr = TRAFFIC.get(a.workload)
        traffic = tr["bytes"] if tr and tr["source"] == kernel_source_hash() else None
        rec["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel": ("k_step (fused pair+bonded forces, velocity Verlet, reductions)"
                                      if a.workload != "sur1m" else
                                      "surrogate force stage (k_sur_desc, k_sur_mlp, k_sur_force, k_step_ext)"),
                           "kernel_ms": k_ms, "alg_bytes_per_launch": alg}
        rec["kernel_breakdown_ms_per_step"] = {
            "rebuild_stage": tm["ms_rebuild"] / max(tm["n_rebuild"], 1),
            "step_kernel": k_ms,
            "finalize": tm["ms_finalize"] / max(tm["n_finalize"], 1)}
    if a.calib_copy:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["calib_copy_bytes"] = src.numel() * 4
    if not a.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, a.workload, a.cpu_seconds, a.quiet)
    s.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
