"""GPU tests of the HIP-event timing mode (md_timing_enable / md_timing_read
and the batch's pair), which bench.py's per-stage breakdown and roofline
come from: every step is counted once per stage, the binning-and-sort part
lies inside the rebuild stage, and the evented launches advance the same
trajectory, bit for bit, as the graph-replayed steps they replace."""
import numpy as np
import pytest

from gpu_helpers import WCA, banner
from kg_fixture import kg1k_state
from paper_2608_14911_amd import inputs
from paper_2608_14911_amd.system import Batch, System, lj_pair

pytestmark = pytest.mark.gpu


def lj_system(seed=21):
    pos, box = inputs.fcc_lattice(8, 0.8442, jitter=0.05, seed=seed)
    vel = inputs.maxwell_boltzmann(pos.shape[0], 1.2, seed=seed)
    return pos, box, vel


def check_counts(tm, steps):
    assert tm["n_step_kernels"] == steps and tm["n_rebuild"] == steps and tm["n_finalize"] == steps
    for k in ("ms_step_kernels", "ms_rebuild", "ms_finalize"):
        assert tm[k] > 0.0, k
    assert 0.0 < tm["ms_bin_sort"] <= tm["ms_rebuild"]


def test_timing_counts_and_trajectory():
    banner("timing mode: counts, sort inside the rebuild stage, same trajectory as the graph")
    pos, box, vel = lj_system()
    steps = 40
    runs = []
    for timed in (False, True):
        s = System(pos, box, vel, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, dt=0.005)
        s.step(2)
        s.timing(timed)
        s.step(steps)
        tm = s.timing() if timed else None
        o = s.observables()
        runs.append((s.get_state(), o, tm))
        s.close()
    (g0, o0, _), (g1, o1, tm) = runs
    check_counts(tm, steps)
    assert o1["n_rebuilds"] >= 3, "the run must cross several rebuilds"
    assert o0["n_rebuilds"] == o1["n_rebuilds"]
    for key in ("pos", "vel", "image", "pos_build"):
        assert np.array_equal(g0[key], g1[key]), key
    # a second read returns what was timed since the first (nothing)
    s = System(pos, box, vel, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, dt=0.005)
    s.timing(True)
    s.step(3)
    assert s.timing()["n_step_kernels"] == 3
    assert s.timing()["n_step_kernels"] == 0
    s.close()


def test_batch_timing_counts_and_trajectory():
    banner("batch timing mode: counts and the same trajectory as the graph")
    pos, box, vel = lj_system(22)
    w = kg1k_state(0.0)
    members = [{"pos": pos, "box": box, "vel": vel, "pair": {(0, 0): lj_pair(rc=2.5)}, "dt": 0.005, "skin": 0.3,
                "integrator": "nve", "seed": 22},
               {"pos": w["pos"], "box": w["box"], "vel": w["vel"], "bonds": w["bonds"],
                "pair": {(0, 0): lj_pair(rc=WCA)}, "dt": 0.01, "skin": 0.4, "integrator": "langevin",
                "temperature": 1.0, "gamma": 0.5, "seed": 23}]
    steps = 30
    runs = []
    for timed in (False, True):
        b = Batch(members)
        b.step(2)
        b.timing(timed)
        b.step(steps)
        tm = b.timing() if timed else None
        runs.append(([b.get_state(k) for k in range(2)], tm))
        b.close()
    (st0, _), (st1, tm) = runs
    check_counts(tm, steps)
    for k in range(2):
        for key in ("pos", "vel", "image"):
            assert np.array_equal(st0[k][key], st1[k][key]), (k, key)
