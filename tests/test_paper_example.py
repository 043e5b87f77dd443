"""The paper's only worked example (section "Example usage") as a fixture.

The script prints no numbers, only parameters; they are stored under
tests/golden/paper_example.json with their citation.  Checks: the synthetic
workload reproduces those parameters, the cutoff is the WCA cutoff 2^(1/6)
to the printed precision, and the oracle's capped warm-up starts from the
random configuration without blowing up.
"""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2608_14911_amd import inputs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_example.json")


def load():
    with open(GOLD) as f:
        return json.load(f)


def test_workload_matches_printed_parameters():
    g = load()
    w = inputs.workload_paper_example()
    assert w["pos"].shape == (g["num_particles"], 3)
    np.testing.assert_array_equal(w["box"], g["box"])
    assert w["rc"] == g["rc"] and w["skin"] == g["skin"] and w["caprad"] == g["LJcaprad"]
    assert w["dt"] == g["warmup_dt"] and w["temperature"] == g["temperature"]
    assert w["gamma"] == g["gamma"]
    assert np.all(w["vel"] == 0.0)
    assert np.all((w["pos"] >= 0) & (w["pos"] < 20.0))
    # printed cutoff is 2^(1/6) to five decimals (the WCA cutoff)
    assert abs(g["rc"] - 2 ** (1 / 6)) < 5e-6


def test_capped_warmup_is_finite_on_random_start():
    g = load()
    n = 2000                       # same density as the paper's 10,000 in 20^3
    L = (n / (g["num_particles"] / 20.0 ** 3)) ** (1 / 3)
    box = np.array([L, L, L])
    pos = inputs.random_positions(n, box, seed=5)
    st = {"pos": pos, "vel": np.zeros((n, 3)), "image": np.zeros((n, 3), dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    par = {"box": box, "pp": oracle.pair_params(g["epsilon"], g["sigma"], g["rc"], caprad=g["LJcaprad"]),
           "ntypes": 1, "mass_by_type": np.array([g["mass"]]), "dt": g["warmup_dt"],
           "integrator": oracle.LANGEVIN, "temperature": g["temperature"], "gamma": g["gamma"], "seed": 5}
    h = oracle.run(st, par, 200)
    assert np.all(np.isfinite(h))
    # the capped force is bounded by its value at the capping radius
    _, fcap = oracle.pair_eval(par["pp"], g["LJcaprad"])
    F, _ = oracle.forces(st["pos"], box, par["pp"])
    assert np.all(np.isfinite(F))
    assert fcap > 0
