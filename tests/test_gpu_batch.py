"""GPU tests of batches (md_batch_*): every member advanced inside a batch
follows, bit for bit, the trajectory a standalone handle with the same
configuration computes (same cells, list, rebuild steps, kernels and noise);
observables agree to FP64 summation order."""
import numpy as np
import pytest

from gpu_helpers import WCA, banner, rel
from kg_fixture import kg1k_state
from paper_2608_14911_amd import inputs
from paper_2608_14911_amd.system import Batch, System, lj_pair, prepare_replica

pytestmark = pytest.mark.gpu


def lj_member(ncell, rho, temp, seed, cf=0):
    pos, box = inputs.fcc_lattice(ncell, rho, jitter=0.05, seed=seed)
    return {"kind": "lj", "pos": pos, "box": box, "vel": inputs.maxwell_boltzmann(pos.shape[0], temp, seed=seed),
            "pair": {(0, 0): lj_pair(rc=2.5)}, "dt": 0.005, "skin": 0.3, "integrator": "nve", "seed": seed,
            "cell_factor": cf}


def kg_member(k_bend, temp, seed, cf=0):
    w = kg1k_state(k_bend)
    return {"kind": "kg", "pos": w["pos"], "box": w["box"], "vel": w["vel"], "bonds": w["bonds"],
            "angles": w["angles"] if k_bend else None, "k_bend": k_bend, "pair": {(0, 0): lj_pair(rc=WCA)},
            "dt": 0.01, "skin": 0.4, "integrator": "langevin", "temperature": temp, "gamma": 0.5, "seed": seed,
            "cell_factor": cf}


def standalone(m):
    return System(m["pos"], m["box"], m["vel"], pair=m["pair"], bonds=m.get("bonds"), angles=m.get("angles"),
                  k_bend=m.get("k_bend", 0.0), dt=m["dt"], skin=m["skin"], integrator=m["integrator"],
                  temperature=m.get("temperature", 1.0), gamma=m.get("gamma", 0.0), seed=m["seed"],
                  cell_factor=m.get("cell_factor", 0))


def members():
    # ragged sizes: 500, 864, 1372 LJ particles; 1,000-bead melts with and
    # without bending; cell factors 1 and 2 both present
    return [lj_member(5, 0.8442, 0.72, 11), kg_member(0.0, 1.0, 12), lj_member(6, 0.75, 1.0, 13, cf=1),
            kg_member(1.5, 1.1, 14, cf=1), lj_member(7, 0.85, 0.9, 15), kg_member(1.5, 0.8, 16)]


def test_batch_members_follow_their_standalone_trajectories():
    ms = members()
    banner("batch of %d members vs standalone, 61 steps" % len(ms))
    b = Batch(ms)
    b.step(61)
    ob = b.observables()
    for k, m in enumerate(ms):
        s = standalone(m)
        s.step(61)
        os_ = s.observables()
        sb, ss = b.get_state(k), s.get_state()
        for key in ("pos", "vel", "image", "pos_build"):
            assert np.array_equal(sb[key], ss[key]), (k, key)
        assert sb["step"] == ss["step"] == 61
        assert ob[k]["n_rebuilds"] == os_["n_rebuilds"], k
        for key in ("e_pair", "e_bond", "e_angle", "e_kin", "virial", "pressure"):
            if os_[key] != 0.0:
                assert rel(ob[k][key], os_[key]) < 1e-12, (k, key)
        s.close()
    b.close()


def test_batch_of_sampled_replicas_runs_and_conserves_lj_energy():
    """Eight replicas from the uneven-size sampler (4 LJ NVE, 4 pushed-off
    melts): the batch runs 200 steps without a device error, and each LJ
    replica conserves its total energy."""
    reps = inputs.batch_replicas(8, seed=1003, n_min=2048, n_max=8192)
    banner("sampled replicas: sizes %s" % [r["pos"].shape[0] for r in reps])
    reps = [prepare_replica(r) for r in reps]
    b = Batch(reps)
    o0 = b.observables()
    b.step(200)
    o1 = b.observables()
    for k, r in enumerate(reps):
        assert o1[k]["step"] == 200
        if r["kind"] == "lj":
            n = r["pos"].shape[0]
            assert abs(o1[k]["e_total"] - o0[k]["e_total"]) / n < 5e-3, k
    b.close()
