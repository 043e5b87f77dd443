"""Kremer-Grest start states pushed off by the FP64 oracle (never by the GPU).

Push-off modelled on the paper's example (section "Example usage": capped
LJ warm-up at a small time step, then the uncapped potential): capped WCA with
the capping radius lowered 1.0, 0.95, 0.9, 0.85, 0.8 (Langevin gamma=1,
dt 0.002), then uncapped WCA at dt 0.005.  FENE (K=30, R0=1.5) and, when
asked, bending stay on throughout.  A raw random walk overlaps beads, so the
ladder starts from a soft cap; a single cap at 0.9 breaks FENE bonds.
"""
import functools

import numpy as np

import oracle
from paper_2608_14911_amd import inputs

WCA = 2.0 ** (1.0 / 6.0)


PUSHOFF = ((1.0, 0.002, 500), (0.95, 0.002, 500), (0.9, 0.002, 1000), (0.85, 0.002, 1000),
           (0.8, 0.002, 1000), (0.0, 0.005, 1000))


def pushoff(w, k_bend=0.0, seed=77, schedule=PUSHOFF):
    n = w["pos"].shape[0]
    st = {"pos": w["pos"].copy(), "vel": np.zeros((n, 3)), "image": np.zeros((n, 3), dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    base = {"box": w["box"], "ntypes": 1, "mass_by_type": np.array([1.0]), "integrator": oracle.LANGEVIN,
            "temperature": 1.0, "gamma": 1.0, "seed": seed, "bonds": w["bonds"], "angles": w["angles"],
            "fene_K": 30.0, "fene_R0": 1.5, "k_bend": k_bend}
    for caprad, dt, ns in schedule:
        oracle.run(st, dict(base, pp=oracle.pair_params(rc=WCA, caprad=caprad), dt=dt), ns)
    return st


@functools.lru_cache(maxsize=None)
def kg1k_state(k_bend=0.0):
    """1,000-bead melt (20 x 50) at density 0.85 after push-off; returns
    (workload dict with pos/vel replaced, unwrapped-free state)."""
    w = inputs.workload_kg1k()
    st = pushoff(w, k_bend=k_bend)
    out = dict(w)
    out["pos"] = st["pos"].copy()
    out["vel"] = st["vel"].copy()
    out["k_bend"] = k_bend
    return out
