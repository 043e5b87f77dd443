"""GPU tests of the autotuner and of the parameters it picks.

The tuned parameters change cost, not physics: the list build (tiles or one
particle per lane on the same cells) and the force kernel's block size leave
every trajectory bitwise unchanged; the skin and the cell size change only
the order of the FP32 force sums, so trajectories agree to rounding.  The
tuner's cache is keyed by (arch, kind, N bucket, density bucket, rc).
"""
import json

import numpy as np
import pytest

from gpu_helpers import WCA, banner
from kg_fixture import kg1k_state
from paper_2608_14911_amd import autotune, inputs
from paper_2608_14911_amd.system import Batch, System, lj_pair, nl_build_flags

pytestmark = pytest.mark.gpu


def lj_member(ncell, rho, temp, seed):
    pos, box = inputs.fcc_lattice(ncell, rho, jitter=0.05, seed=seed)
    return {"kind": "lj", "pos": pos, "box": box, "vel": inputs.maxwell_boltzmann(pos.shape[0], temp, seed=seed),
            "pair": {(0, 0): lj_pair(rc=2.5)}, "dt": 0.005, "skin": 0.3, "integrator": "nve", "seed": seed}


def kg_member(temp, seed):
    w = kg1k_state(1.5)
    return {"kind": "kg", "pos": w["pos"], "box": w["box"], "vel": w["vel"], "bonds": w["bonds"],
            "angles": w["angles"], "k_bend": 1.5, "pair": {(0, 0): lj_pair(rc=WCA)}, "dt": 0.01, "skin": 0.4,
            "integrator": "langevin", "temperature": temp, "gamma": 0.5, "seed": seed}


def run_state(system, steps):
    system.step(steps)
    st = system.get_state()
    o = system.observables()
    system.close()
    return st, o


@pytest.mark.parametrize("kind", ["lj", "kg"])
def test_force_kernel_block_sizes_leave_trajectories_unchanged(kind):
    banner("force-kernel block sizes, %s" % kind)
    if kind == "lj":
        m = lj_member(9, 0.8442, 0.72, 21)            # 2,916 particles: a ragged last block at every size
        make = lambda bs: System(m["pos"], m["box"], m["vel"], pair=m["pair"], dt=0.005, skin=0.3, block_size=bs)
    else:
        m = kg_member(1.0, 22)
        make = lambda bs: System(m["pos"], m["box"], m["vel"], pair=m["pair"], bonds=m["bonds"], angles=m["angles"],
                                 k_bend=1.5, dt=0.01, skin=0.4, integrator="langevin", gamma=0.5, seed=22,
                                 block_size=bs)
    ref, oref = run_state(make(0), 40)
    assert oref["n_rebuilds"] >= 1
    for bs in (64, 128, 512):
        st, o = run_state(make(bs), 40)
        for key in ("pos", "vel", "image"):
            assert np.array_equal(st[key], ref[key]), (bs, key)
        for key in ("e_pair", "e_bond", "e_angle", "e_kin", "virial"):
            assert abs(o[key] - oref[key]) <= 1e-12 * max(abs(oref[key]), 1.0), (bs, key)
    # switched in place (md_set_params) between steps: still the same trajectory
    s = make(0)
    s.step(15)
    s.set_params(block_size=64)
    s.step(15)
    s.set_params(block_size=512)
    st, _ = run_state(s, 10)
    for key in ("pos", "vel", "image"):
        assert np.array_equal(st[key], ref[key]), ("switched", key)


def test_tune_batch_writes_cache_and_keeps_physics(tmp_path):
    banner("autotune a 4-member batch")
    ms = [lj_member(6, 0.84, 0.9, 31), kg_member(1.0, 32), lj_member(7, 0.82, 0.8, 33), kg_member(1.2, 34)]
    path = str(tmp_path / "cache.json")
    choice, table = autotune.tune(ms, steps=6, skins=(0.3, 0.4), path=path)
    keys = {autotune.member_key(m) for m in ms}
    assert set(choice) == keys and len(keys) == 2
    assert all(k.startswith("gfx950|") and "|rho0.8|" in k for k in keys)
    assert len(table) >= 2 * 3 * 2 - 2
    cache = json.load(open(path))
    for k in keys:
        e = cache[k]
        assert (e["skin"], e["cell_factor"], e["nl_build"]) == tuple(choice[k])
        assert e["skin"] in (0.3, 0.4) and e["nl_build"] in ("tiles", "per_particle")
    again, _ = autotune.cached_choice(ms, path=path)
    assert again == {k: tuple(v) for k, v in choice.items()}
    # the tuned batch against the default one: the same physics to rounding
    tuned = Batch(autotune.apply(ms, choice))
    plain = Batch(ms)
    tuned.step(20)
    plain.step(20)
    ot, op = tuned.observables(), plain.observables()
    for k, m in enumerate(ms):
        a, b = tuned.get_state(k), plain.get_state(k)
        d = np.abs(a["pos"] - b["pos"])
        d = np.minimum(d, m["box"] - d)
        assert d.max() < 1e-4, (k, d.max())
        assert abs(ot[k]["e_total"] - op[k]["e_total"]) <= 1e-5 * abs(op[k]["e_total"]) + 1e-3
    tuned.close()
    plain.close()
    # the list build alone changes nothing: tuned choice with the other build, bit for bit
    other = {k: (sk, cf, "per_particle" if bld == "tiles" else "tiles") for k, (sk, cf, bld) in choice.items()}
    x, y = Batch(autotune.apply(ms, choice)), Batch(autotune.apply(ms, other))
    x.step(20)
    y.step(20)
    for k in range(len(ms)):
        sx, sy = x.get_state(k), y.get_state(k)
        for key in ("pos", "vel", "image"):
            assert np.array_equal(sx[key], sy[key]), (k, key)
    x.close()
    y.close()


def test_tune_system_caches_cells_build_and_block(tmp_path):
    banner("autotune a single LJ system")
    m = lj_member(10, 0.8442, 0.72, 41)
    n = m["pos"].shape[0]
    path = str(tmp_path / "cache.json")

    def make(cf, flags):
        return System(m["pos"], m["box"], m["vel"], pair=m["pair"], dt=0.005, skin=0.3, cell_factor=cf, flags=flags)

    (cf, build, bs, skin), table = autotune.tune_system(make, n, 0.8442, 2.5, "lj", steps=8, path=path)
    assert bs in autotune.BLOCKS and build in ("tiles", "per_particle") and cf in (1, 2) and skin == 0.3
    assert len(table) >= 2 + len(autotune.BLOCKS)
    assert autotune.cached_system_choice("lj", n, 0.8442, 2.5, path=path) == (cf, build, bs, skin)
    # the winner and the defaults: the same trajectory up to FP32 summation order
    a, _ = run_state(System(m["pos"], m["box"], m["vel"], pair=m["pair"], dt=0.005, skin=0.3, cell_factor=cf,
                            flags=nl_build_flags(build), block_size=bs), 20)
    b, _ = run_state(make(0, 0), 20)
    d = np.abs(a["pos"] - b["pos"])
    d = np.minimum(d, m["box"] - d)
    assert d.max() < 1e-4
    # a skin dimension (a workload whose skin is a performance choice)
    path2 = str(tmp_path / "cache2.json")

    def make_s(cf, flags, skin):
        return System(m["pos"], m["box"], m["vel"], pair=m["pair"], dt=0.005, skin=skin, cell_factor=cf, flags=flags)

    (cf2, build2, bs2, skin2), table2 = autotune.tune_system(make_s, n, 0.8442, 2.5, "lj", steps=6, blocks=(256,),
                                                             skins=(0.2, 0.4), path=path2)
    assert skin2 in (0.2, 0.4) and {t["skin"] for t in table2} == {0.2, 0.4}
    assert autotune.cached_system_choice("lj", n, 0.8442, 2.5, path=path2) == (cf2, build2, bs2, skin2)
