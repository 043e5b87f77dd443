"""Throughput of the short-range MD step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload default|lj1m|kg2m|batch|sur1m|dpd1m|adress1m|kg1k]

The headline workload is the LJ fluid of 1,048,576 particles (FCC 64^3,
density 0.8442, uniform jitter 0.05, T = 0.72), rc = 2.5 shifted, skin 0.3,
NVE dt = 0.005, FP32 pair math, FP64 positions / velocities / reductions.
A "step" is one pass of the whole hot path: gated cell sort + Verlet-list
rebuild, fused force + velocity-Verlet kernel, FP64 energy/virial reduction.
Inputs are resident in HBM before a timed region starts.

Each workload is timed twice over K steps after W warm-up steps:
  1. the product path: md_step replaying its two-step hipGraph, no events ->
     ``value`` and ``ms_per_step``;
  2. an evented pass: the same K steps launched kernel by kernel with HIP
     events on the library's stream around each stage -> the per-stage
     breakdown and the ``roofline`` of the fused force + integrate kernel.
The breakdown splits the rebuild stage into binning + cell sort and the
neighbour-list build.  The default run prints one JSON line for the LJ fluid
with the other workloads (2M-bead melt, 256-replica batch with its members
also run one by one, learned surrogate on a 1M-bead melt, DPD fluid under
Lees-Edwards shear, AdResS fluid) as sub-records under "workloads", and a
"cpu_baseline" object: the FP64 oracle timed on this host on a bounded
sample, with all threads and with one.
"""
import argparse
import hashlib
import json
import math
import os
import platform
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
#   DPD + shear 1M (density 3, rc_d 1, skin 0.3): NL 4 + 13.8*4 = 59,
#           positions 24, neighbour velocities 24 and ids 4, force 12,
#           integration 132 -> 255
#   AdResS LJ 1M: the LJ fluid's 327 (the weights come from the positions)
ALG_BYTES = {"lj1m": 327.0, "kg2m": 213.0, "kg1k": 213.0, "sur1m": 819.0, "dpd1m": 255.0, "adress1m": 327.0}
STEP_KERNEL = {"lj1m": "k_step_fast (fused pair forces, velocity Verlet, reductions)",
               "kg2m": "k_step_fast_bonded (fused pair + bonded forces, velocity Verlet, reductions)",
               "kg1k": "k_step_fast_bonded (fused pair + bonded forces, velocity Verlet, reductions)",
               "dpd1m": "k_step_gen (tabulated pair force, DPD pair thermostat, Lees-Edwards image and "
                        "crossing, velocity Verlet, reductions) with its velocity snapshot",
               "adress1m": "k_step_gen (AdResS mix of LJ and a tabulated CG pair force, velocity Verlet, "
                           "reductions)"}
# The surrogate's force stage is bound by vector ALU issue (counters: VALU
# busy 95-100 % in the descriptor and pair-force kernels), so it is priced in
# FP32 vector operations against the chip's FP32 vector peak.  Algorithmic
# operations per bead-step, FMA = 2, over the 55.6 ordered pairs within
# r_d = 2.5 at density 0.85: descriptors 134 per pair (32 Gaussians by
# recurrence 70, 32 FMAs into G 64) and pair force 262 per pair (basis 70,
# g' 64, two 32-term dot products 128): (134 + 262) x 55.6 = 22.0k.  The
# network's 24.8k operations per bead run on the matrix cores and are left
# out of this figure.
SUR_VALU_FLOPS = 22.0e3
FP32_VECTOR_PEAK_TFLOPS = 157.3
# HBM bytes per launch of the fused kernel from rocprofv3 FETCH_SIZE and
# WRITE_SIZE passes (each scaled by what the counter reads for a 512 MiB
# copy: x2.0 and x1.0), valid only for the sources the kernel is compiled
# from (SHA-256 prefix over KERNEL_SOURCES); null once they change.
KERNEL_SOURCES = ("md_kernels.hip", "md_device.h", "md_internal.h", "md_api.hip")
TRAFFIC = {"lj1m": {"bytes": 555358863, "read": 465777455, "write": 89581408, "source": "69393c115cf2c192"},
           "kg2m": {"bytes": 657338658, "read": 478474626, "write": 178864032, "source": "69393c115cf2c192"}}


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_14911_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="default",
                    choices=["default", "lj1m", "kg2m", "kg1k", "batch", "sur1m", "dpd1m", "adress1m"],
                    help="default: the LJ fluid with kg2m, batch and sur1m as sub-records")
    ap.add_argument("--sur-precision", default="bf16", choices=["fp32", "bf16"],
                    help="sur1m: network precision of the surrogate")
    ap.add_argument("--batch-start", default="lattice", choices=["lattice", "pushoff"],
                    help="batch: melt replicas laid on a lattice (no push-off) or pushed-off random walks")
    ap.add_argument("--autotune", default="cache", choices=["cache", "tune", "none"],
                    help="the autotuner's cached choice (batch members; LJ 1M and KG 2M cells, list build "
                         "and force-kernel block), a fresh tuning run, or the library defaults")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="CPU oracle budget per leg")
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


# ---------------------------------------------------------------- systems
# autotuner keys of the single-system workloads: (kind, N, density, rc); the
# surrogate's key carries its descriptor cutoff, and its skin is tuned too
# (the descriptor list's skin is a performance choice, not part of the model)
TUNE_KEYS = {"lj1m": ("lj", 1048576, 0.8442, 2.5), "kg2m": ("kg", 2000000, 0.85, 2.0 ** (1.0 / 6.0)),
             "sur1m": ("sur", 1000000, 0.85, 2.5)}
SUR_SKINS = (0.2, 0.25, 0.3, 0.4)
_PUSHED = {}   # pushed-off melt states, reused by the tuner's trials


def surrogate_on(s, a):
    """The surrogate replaces the WCA pair force: the network trained by
    surrogate_experiment.py on a 100k-bead plain-method melt."""
    wpath = os.path.join(ROOT, "paper_2608_14911_amd", "data", "surrogate_kg.npz")
    wd = np.load(wpath)
    s.sur_set(wd["theta_" + a.sur_precision], wd["g_mean"], wd["g_istd"], a.sur_precision)
    s.set_pair_mode("surrogate")
    return s


def make_system(name, quiet, cell_factor=0, flags=0, block_size=0, skin=None):
    from paper_2608_14911_amd import inputs
    from paper_2608_14911_amd.system import from_workload, push_off
    if name == "lj1m":
        w = inputs.workload_lj(ncell=64, seed=1001)
        return w, from_workload(w, precision="fp32", cell_factor=cell_factor, flags=flags, block_size=block_size)
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
    t0 = time.time()
    if name not in _PUSHED:
        w0 = dict(w, caprad=1.0, dt=0.002, gamma=1.0, vel=np.zeros_like(w["pos"]))
        s = from_workload(w0, precision="fp32", nl_capacity=256)
        push_off(s, w["rc"], log=lambda m: log(m, quiet))
        s.set_params(dt=w["dt"], gamma=w["gamma"])
        s.step(200)
        _PUSHED[name] = s.get_state()
        s.close()
    st = _PUSHED[name]
    w1 = dict(w, pos=st["pos"], vel=st["vel"])
    if skin is not None:
        w1["skin"] = skin
    extra = {"list_cutoff": 2.5, "surrogate": True} if name == "sur1m" else {}
    s = from_workload(w1, precision="fp32", cell_factor=cell_factor, flags=flags, block_size=block_size, **extra)
    s.set_state(st)
    s.step(1)
    if s.status() != 0:
        raise RuntimeError("KG system after push-off: status %d" % s.status())
    log("%s: push-off done in %.1f s" % (name, time.time() - t0), quiet)
    return w1, s


def make_ext_system(name):
    """The extended-method workloads (one GPU, 1,048,576 particles each).
    dpd1m: a DPD fluid at density 3 (random start, Maxwell-Boltzmann
    velocities at kT = 1 plus the imposed profile) with the soft repulsion
    u = a (1 - r)^2 / 2, a = 25, as a 256-point pair table, DPD thermostat
    gamma 4.5 with rc_d 1, Lees-Edwards shear rate 0.1, dt 0.01, skin 0.3.
    adress1m: the LJ fluid of lj1m with an AdResS slab (atomistic zone
    L/8 either side of the box centre, hybrid zones L/8 wide) and a soft CG
    pair table u = a (1 - r / rc)^2 / 2, a = 20, rc 2.0, NVE."""
    from paper_2608_14911_amd import inputs
    from paper_2608_14911_amd.system import System, lj_pair
    n = 1048576
    if name == "dpd1m":
        rho, rate, seed = 3.0, 0.1, 1020
        L = (n / rho) ** (1.0 / 3.0)
        box = np.array([L, L, L])
        pos = inputs.random_positions(n, box, seed=seed)
        vel = inputs.maxwell_boltzmann(n, 1.0, seed=seed)
        vel[:, 0] += rate * (pos[:, 1] - 0.5 * L)
        s = System(pos, box, vel, pair={(0, 0): lj_pair(rc=1.0)}, skin=0.3, dt=0.01, integrator="dpd",
                   temperature=1.0, gamma=4.5, seed=seed, dpd_rc=1.0, shear_rate=rate, table_points=256)
        r = np.linspace(0.0, 1.0, 256)
        s.set_pair_table(0, 0, 12.5 * (1.0 - r) ** 2, 25.0 * (1.0 - r), 0.0)
        w = {"name": "DPD fluid 1048576 particles, density 3, soft tabulated repulsion a = 25, gamma 4.5, "
                     "Lees-Edwards shear rate 0.1", "rc": 1.0, "skin": 0.3, "dt": 0.01, "integrator": "dpd"}
        return w, s
    w = inputs.workload_lj(ncell=64, seed=1001)
    L = w["box"][0]
    s = System(w["pos"], w["box"], w["vel"], pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, dt=0.005, table_points=512,
               adress=(0.5 * L, L / 8.0, L / 8.0))
    rc_cg = 2.0
    r = np.linspace(0.0, rc_cg, 512)
    s.set_cg_table(0, 0, 10.0 * (1.0 - r / rc_cg) ** 2, 20.0 * (1.0 - r / rc_cg) / rc_cg, 0.0, rc_cg)
    w2 = {"name": "LJ fluid 1048576 particles (FCC 64^3), rho 0.8442, AdResS slab: atomistic L/8 either side "
                  "of the centre, hybrid L/8, soft tabulated CG pair (a = 20, rc 2.0)",
          "rc": 2.5, "skin": 0.3, "dt": 0.005, "integrator": "nve"}
    return w2, s


def bench_ext(name, a):
    t0 = time.time()
    w, s = make_ext_system(name)
    log("%s: %d particles ready in %.1f s" % (name, s.n, time.time() - t0), a.quiet)
    rec = single_record(name, a, w, s)
    rec["config"]["block_size"] = 256
    rec["config"]["tuning"] = "library defaults"
    s.close()
    del s
    free_gpu()
    log("%s: %.3g atom-steps/s, %.3f ms/step" % (name, rec["value"], rec["ms_per_step"]), a.quiet)
    return w, rec


def free_gpu():
    import gc

    import torch
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# ---------------------------------------------------------------- CPU baseline
def cpu_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cpus_available": avail}


def cpu_oracle_rate(w, budget_s, nthreads, quiet, max_steps=50):
    """The FP64 oracle (linked cells, OpenMP over particles) advancing the
    same workload for a bounded number of steps; returns (atom-steps/s,
    steps, seconds, threads)."""
    import oracle
    n = w["pos"].shape[0]
    st = {"pos": w["pos"].copy(), "vel": w["vel"].copy(), "image": np.zeros((n, 3), dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    par = {"box": w["box"], "pp": oracle.pair_params(w["eps"], w["sigma"], w["rc"], w["shift"], 0.0),
           "ntypes": 1, "mass_by_type": np.array([1.0]), "dt": w["dt"],
           "integrator": oracle.LANGEVIN if w["integrator"] == "langevin" else oracle.NVE,
           "temperature": w["temperature"], "gamma": w["gamma"], "seed": w["seed"],
           "bonds": w.get("bonds"), "angles": w.get("angles"), "k_bend": w.get("k_bend", 0.0)}
    threads = nthreads or oracle.nthreads_default()
    oracle.run(st, par, 1, nthreads=threads)          # untimed: first touch
    t1 = time.time()
    oracle.run(st, par, 1, nthreads=threads)
    one = time.time() - t1
    k = max(0, min(max_steps - 1, int(budget_s / max(one, 1e-6)) - 1))
    t2 = time.time()
    if k:
        oracle.run(st, par, k, nthreads=threads)
    secs = (time.time() - t2) + one
    steps = k + 1
    log("cpu oracle: %d steps of %d particles in %.2f s on %d threads" % (steps, n, secs, threads), quiet)
    return n * steps / secs, steps, secs, threads


def cpu_baseline(w, budget_s, quiet):
    n = w["pos"].shape[0]
    v_all, s_all, t_all, th = cpu_oracle_rate(w, budget_s, 0, quiet)
    v_one, s_one, t_one, _ = cpu_oracle_rate(w, budget_s, 1, quiet, max_steps=10)
    rec = {"value": v_all, "unit": "atom-steps/s", "cores": th, "kind": "oracle",
           "sample": "%d steps (%.1f s) of the same %d-particle workload with %d OpenMP threads, and %d steps "
                     "(%.1f s) with 1 thread; FP64 linked cells, after 1 untimed step"
                     % (s_all, t_all, n, th, s_one, t_one),
           "value_1thread": v_one}
    rec.update(cpu_info())
    return rec


# ---------------------------------------------------------------- single systems
def time_system(s, steps, warmup, quiet):
    """Graph-replayed timed region, then an evented pass of the same length."""
    import torch
    s.step(warmup)
    o0 = s.observables()
    s.history()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    o1 = s.observables()
    hist = s.history()
    # evented pass: kernel-by-kernel launches, events around each stage
    s.timing(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s.step(steps)
    torch.cuda.synchronize()
    el_ev = time.perf_counter() - t1
    tm = s.timing()
    s.timing(False)
    o2 = s.observables()
    return el, el_ev, tm, o0, o1, o2, hist


def breakdown(tm, step_key, k_ms):
    """Per-step milliseconds of the evented pass: the gated rebuild stage
    (binning and cell sort, then the neighbour-list build; both run every
    step and return at once unless a rebuild is due), the step kernel, the
    finalize."""
    nr = max(tm["n_rebuild"], 1)
    reb = tm["ms_rebuild"] / nr
    srt = tm["ms_bin_sort"] / nr
    return {"rebuild_stage": reb, "binning_sort": srt, "neighbour_build": reb - srt, step_key: k_ms,
            "finalize": tm["ms_finalize"] / max(tm["n_finalize"], 1)}


def single_record(name, a, w, s):
    from paper_2608_14911_amd import md as md_
    n = s.n
    el, el_ev, tm, o0, o1, o2, hist = time_system(s, a.steps, a.warmup, a.quiet)
    plan = md_.md_plan_config(s.cfg)
    k_ms = tm["ms_step_kernels"] / max(tm["n_step_kernels"], 1)
    alg = ALG_BYTES[name] * n
    ach = alg / (k_ms * 1e-3) / 1e9
    tr = TRAFFIC.get(name)
    traffic = tr["bytes"] if tr and tr["source"] == kernel_source_hash() else None
    sur = name == "sur1m"
    rec = {
        "metric": "atom-steps/s (1M LJ, 2M KG melt); surrogate vs plain at stated force RMSE",
        "value": n * a.steps / el, "unit": "atom-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * el / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": w["name"] + (", learned surrogate pair force (%s network)" % a.sur_precision
                                            if sur else ""),
                   "n_particles": n, "rc": w["rc"], "skin": w["skin"], "dt": w["dt"],
                   "integrator": w["integrator"],
                   "precision": "FP32 pair/bonded math, FP64 positions, velocities and reductions",
                   "parallelism": "single GPU", "cell_factor": plan["cell_factor"],
                   "cells_per_side": plan["cells"][0], "list_build": plan["nl_build"],
                   "list_capacity": plan["nl_capacity"]},
        "timing": "value and ms_per_step: md_step replaying its two-step hipGraph (no events); roofline and "
                  "breakdown: a second pass of the same steps launched kernel by kernel with HIP events",
        "n_rebuilds": o1["n_rebuilds"] - o0["n_rebuilds"],
        "energy_drift_per_particle": (o1["e_total"] - o0["e_total"]) / n,
        "nl_max_count": o1["nl_max_count"],
        "evented_pass": {"ms_per_step": 1e3 * el_ev / a.steps, "n_rebuilds": o2["n_rebuilds"] - o1["n_rebuilds"]},
        "roofline": ({"bound": "alu", "achieved": SUR_VALU_FLOPS * n / (k_ms * 1e-3) / 1e12,
                      "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": SUR_VALU_FLOPS * n / (k_ms * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                      "traffic": None,
                      "kernel": "surrogate force stage (k_sur_desc2 with the BF16 network, k_sur_step)",
                      "kernel_ms": k_ms, "alg_flops_per_particle": SUR_VALU_FLOPS,
                      "hbm_alg_bytes_per_particle": ALG_BYTES[name]} if sur else
                     {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                      "kernel": STEP_KERNEL[name],
                      "kernel_ms": k_ms, "alg_bytes_per_launch": alg,
                      "alg_bytes_per_particle": ALG_BYTES[name]}),
        "kernel_breakdown_ms_per_step": breakdown(tm, "step_kernel" if not sur else "force_stage_and_step", k_ms),
    }
    if name == "kg2m" or name == "kg1k":
        rec["kernel_breakdown_note"] = ("pair and bonded forces and the integration are fused into one kernel "
                                        "(step_kernel); the rebuild stage is binning_sort + neighbour_build")
    return rec


def single_choice(name, a):
    """(cell_factor, list-build flags, block_size, source) of a single-system
    workload: the command line's, the autotuner's cache entry, a fresh tuning
    run, or the library defaults."""
    from paper_2608_14911_amd import autotune
    from paper_2608_14911_amd import md as md_
    from paper_2608_14911_amd.system import nl_build_flags
    nl_flags = {"auto": 0, "tiles": md_.MD_CFG_NL_TILES, "per-particle": md_.MD_CFG_NL_PER_PARTICLE}[a.nl_build]
    if a.cell_factor or a.nl_build != "auto" or a.autotune == "none" or name not in TUNE_KEYS:
        return a.cell_factor, nl_flags, 0, None, "command line / library defaults", None
    kind, n, rho, rc = TUNE_KEYS[name]
    sur = name == "sur1m"
    if a.autotune == "tune":
        if sur:
            make = lambda cf, fl, sk: surrogate_on(make_system(name, True, cf, fl, 0, sk)[1], a)
            (cf, build, bs, skin), table = autotune.tune_system(make, n, rho, rc, kind, steps=20, blocks=(),
                                                                skins=SUR_SKINS, log=lambda m: log(m, a.quiet))
        else:
            make = lambda cf, fl: make_system(name, True, cf, fl)[1]
            (cf, build, bs, skin), table = autotune.tune_system(make, n, rho, rc, kind, steps=30,
                                                                log=lambda m: log(m, a.quiet))
            skin = None
        return cf, nl_build_flags(build), bs, skin, "autotuner (fresh run)", table
    c = autotune.cached_system_choice(kind, n, rho, rc)
    if c is None:
        return 0, 0, 0, None, "library defaults (no autotuner cache entry)", None
    return c[0], nl_build_flags(c[1]), c[2], (c[3] if sur else None), \
        "autotuner cache (%s, cell factor %d, %s, block %d, skin %.2f)" % (
            autotune.key_of(kind, n, rho, rc), c[0], c[1], c[2], c[3]), None


def bench_single(name, a):
    cf, nl_flags, bs, skin, how, table = single_choice(name, a)
    t0 = time.time()
    w, s = make_system(name, a.quiet, cf, nl_flags, bs, skin)
    if name == "sur1m":
        surrogate_on(s, a)
    log("%s: %d particles ready in %.1f s" % (name, s.n, time.time() - t0), a.quiet)
    rec = single_record(name, a, w, s)
    rec["config"]["block_size"] = bs or 256
    rec["config"]["tuning"] = how
    if table:
        rec["autotune_trials"] = table
    s.close()
    del s
    free_gpu()
    log("%s: %.3g atom-steps/s, %.3f ms/step" % (name, rec["value"], rec["ms_per_step"]), a.quiet)
    return w, rec


# ---------------------------------------------------------------- batch
def member_alg_bytes(m, n, skin):
    """Algorithmic bytes per atom-step of one member: half Verlet list
    (int32) at its density and list radius, FP64 x / v streams, FP32 force,
    topology for melts."""
    rc = m["pair"][(0, 0)][2]
    rv = rc + skin
    rho = n / float(m["box"][0]) ** 3
    half = rho * 2.0 / 3.0 * math.pi * rv ** 3
    return 4 + 4 * half + 24 + 12 + 132 + (16 if m.get("kind") == "kg" else 0)


def lattice_replica(r):
    """A melt replica's chains laid on a simple cubic lattice at its own
    density and chain length (no overlapping beads, no push-off)."""
    from paper_2608_14911_amd import inputs
    lc = r["chain_len"]
    w = inputs.lattice_melt(r["pos"].shape[0] // lc, lc, r["density"], jitter=0.05, seed=r["seed"])
    out = dict(r)
    out.update(pos=w["pos"], box=w["box"], bonds=w["bonds"], angles=w["angles"])
    return out


def bench_batch(a):
    import torch
    from paper_2608_14911_amd import autotune, inputs
    from paper_2608_14911_amd.system import Batch, prepare_replica
    t0 = time.time()
    reps = inputs.batch_replicas(256, seed=1003)
    if a.batch_start == "lattice":
        reps = [lattice_replica(r) if r["kind"] == "kg" else r for r in reps]
    else:
        reps = [prepare_replica(r) for r in reps]
    log("batch: replicas ready in %.1f s" % (time.time() - t0), a.quiet)
    table = []
    if a.autotune == "none":
        choice = {}
        how = "each replica's own skin, the library's automatic cells and list build"
    elif a.autotune == "tune":
        choice, table = autotune.tune(reps, steps=30, log=lambda m: log(m, a.quiet))
        how = "tuned in this run"
    else:
        choice, src = autotune.cached_choice(reps)
        how = "autotuner cache (%s)" % src
    reps = autotune.apply(reps, choice)
    ntot = sum(r["pos"].shape[0] for r in reps)
    b = Batch(reps)
    b.step(a.warmup)
    o0 = b.observables()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    b.step(a.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - ts
    o1 = b.observables()
    b.timing(True)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    b.step(a.steps)
    torch.cuda.synchronize()
    el_ev = time.perf_counter() - ts
    tm = b.timing()
    b.timing(False)
    b.close()
    del b
    free_gpu()
    k_ms = tm["ms_step_kernels"] / max(tm["n_step_kernels"], 1)
    alg = sum(member_alg_bytes(r, r["pos"].shape[0], r["skin"]) * r["pos"].shape[0] for r in reps)
    ach = alg / (k_ms * 1e-3) / 1e9
    rec = {
        "value": ntot * a.steps / el, "unit": "atom-steps/s", "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * el / a.steps,
        "config": {"workload": "batch of 256 replicas (128 LJ fluids, 128 polymer melts), %d particles" % ntot,
                   "n_particles": ntot, "replicas": len(reps), "sizes": "log-uniform 2048..65536",
                   "melt_start": ("chains laid on a simple cubic lattice" if a.batch_start == "lattice"
                                  else "random walks pushed off on the GPU"),
                   "precision": "FP32 pair/bonded math, FP64 positions, velocities and reductions",
                   "parameters": how,
                   "choice": {k: {"skin": v[0], "cell_factor": v[1] or "auto", "nl_build": v[2]}
                              for k, v in sorted(choice.items())}},
        "n_rebuilds_total": sum(x["n_rebuilds"] - y["n_rebuilds"] for x, y in zip(o1, o0)),
        "evented_pass": {"ms_per_step": 1e3 * el_ev / a.steps},
        "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": ach / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_batch_step (fused forces + integration, all replicas)", "kernel_ms": k_ms,
                     "alg_bytes_per_launch": alg},
        "kernel_breakdown_ms_per_step": breakdown(tm, "step_kernel", k_ms),
    }
    t_one = standalone_seconds_per_step(reps)
    free_gpu()
    rec["vs_members_one_by_one"] = {
        "method": "each member as its own handle (plain step kernels, graph-replayed md_step), 4 untimed "
                  "and 20 timed steps from the same start, summed time per step",
        "ms_per_step": 1e3 * t_one, "atom_steps_per_s": ntot / t_one,
        "batched_over_one_by_one": rec["value"] / (ntot / t_one)}
    if table:
        rec["autotune_trials"] = table
    log("batch: %.3g atom-steps/s, %.3f ms/step (%.1fx the members one by one)" % (
        rec["value"], rec["ms_per_step"], rec["vs_members_one_by_one"]["batched_over_one_by_one"]), a.quiet)
    return reps, rec


def standalone_seconds_per_step(reps, steps=20, warm=4):
    """The batch's members advanced one by one, each as its own handle with
    the same parameters: the summed wall time per step."""
    from paper_2608_14911_amd.system import System, nl_build_flags
    t_sum = 0.0
    for r in reps:
        s = System(r["pos"], r["box"], r.get("vel"), pair=r.get("pair"), bonds=r.get("bonds"), angles=r.get("angles"),
                   k_bend=r.get("k_bend", 0.0), dt=r.get("dt", 0.005), skin=r.get("skin", 0.3),
                   integrator=r.get("integrator", "nve"), temperature=r.get("temperature", 1.0),
                   gamma=r.get("gamma", 0.0), seed=r.get("seed", 0), masses=r.get("masses", (1.0,)),
                   nl_capacity=r.get("nl_capacity", 0), cell_factor=r.get("cell_factor", 0),
                   flags=nl_build_flags(r.get("nl_build", "auto")))
        s.step(warm)
        s.stream.synchronize()
        t1 = time.perf_counter()
        s.step(steps)
        s.stream.synchronize()
        t_sum += (time.perf_counter() - t1) / steps
        s.close()
    return t_sum


# ---------------------------------------------------------------- main
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
        reps, rec = bench_batch(a)
        rec.update({"metric": "atom-steps/s (1M LJ, 2M KG melt); surrogate vs plain at stated force RMSE",
                    "n_gpus": 1, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                    "dtype": "f32+f64", "data": "synthetic"})
        if not a.no_cpu_baseline:
            w = dict(reps[0])
            eps, sig, rc, shift, _ = w["pair"][(0, 0)]
            w.update({"eps": eps, "sigma": sig, "rc": rc, "shift": shift})
            rec["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds, a.quiet)
            rec["cpu_baseline"]["sample"] += " (replica 0 of the batch)"
        print(json.dumps(rec), flush=True)
        return
    main_name = "lj1m" if a.workload == "default" else a.workload
    if main_name in ("dpd1m", "adress1m"):
        w, rec = bench_ext(main_name, a)
    else:
        w, rec = bench_single(main_name, a)
    if a.workload == "default":
        subs = {}
        _, subs["kg2m"] = bench_single("kg2m", a)
        _, subs["batch"] = bench_batch(a)
        _, subs["sur1m"] = bench_single("sur1m", a)
        subs["sur1m"]["vs_plain_kg"] = "plain WCA kernel on a melt of the same density: workloads.kg2m"
        _, subs["dpd1m"] = bench_ext("dpd1m", a)
        _, subs["adress1m"] = bench_ext("adress1m", a)
        rec["workloads"] = subs
    if a.calib_copy:
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        rec["calib_copy_bytes"] = src.numel() * 4
    if not a.no_cpu_baseline and main_name not in ("dpd1m", "adress1m"):
        rec["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds, a.quiet)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
