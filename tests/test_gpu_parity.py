"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Neighbour sets must equal the oracle's bit for bit (same FP64 positions,
same IEEE operations for r^2); forces, energies and virial must agree within
1e-12 (FP64 pair path) and 1e-5 (FP32 pair path, condition-aware per
particle); short trajectories in FP64 within 1e-9 on unwrapped positions.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import WCA, assert_forces_close, banner, oracle_pp, rel, unwrap
from kg_fixture import kg1k_state
from paper_2608_14911_amd import inputs
from paper_2608_14911_amd.system import System, from_workload, lj_pair

pytestmark = pytest.mark.gpu


def tricky(seed, n, L, rv):
    g = np.random.default_rng(seed)
    pos = g.uniform(0, L, size=(n, 3))
    pos[0] = [0.0, 0.0, 0.0]
    pos[1] = [np.nextafter(L, 0), 0.5, 0.5]
    pos[2] = [L / 2, np.nextafter(L, 0), 0.0]
    base = np.array([L / 3, L / 3, L / 3])
    for k, r in enumerate([rv, np.nextafter(rv, 0), np.nextafter(rv, 10)]):
        pos[3 + 2 * k] = base + [0, 0, 1.3 * k]
        pos[4 + 2 * k] = base + [r, 0, 1.3 * k]
    return inputs.wrap_into_box(pos, [L, L, L])


@pytest.mark.parametrize("seed,n,L,cf", [(0, 300, 7.0, 1), (1, 2000, 12.0, 1), (2, 5000, 15.3, 1),
                                         (3, 2000, 12.0, 2), (4, 300, 7.2, 2), (5, 4000, 14.0, 2)])
def test_neighbor_sets_bitexact_random(seed, n, L, cf):
    banner("NL random seed=%d n=%d L=%g cell_factor=%d" % (seed, n, L, cf))
    rc, skin = WCA, 0.3
    rv = rc + skin
    pos = tricky(seed, n, L, rv)
    s = System(pos, [L, L, L], pair={(0, 0): lj_pair(rc=rc, caprad=0.8)}, skin=skin, nl_capacity=64,
               cell_factor=cf)
    got = s.neighbors(cap=64)
    ref = oracle.neighbors(pos, [L, L, L], rv)
    for i in range(n):
        assert np.array_equal(got[i], ref[i]), i
    # the longest row, which the build keeps with one conditional atomic per
    # wavefront, is the oracle's
    assert s.observables()["nl_max_count"] == max(len(r) for r in ref)
    s.close()


def test_neighbor_sets_bitexact_kg1k_and_paper_density():
    w = inputs.workload_kg1k()
    banner("NL kg1k")
    s = from_workload(w, precision="fp64")
    got = s.neighbors(cap=64)
    ref = oracle.neighbors(w["pos"], w["box"], w["rc"] + w["skin"])
    assert all(np.array_equal(a, b) for a, b in zip(got, ref))
    s.close()
    banner("NL paper-example density")
    w = inputs.workload_paper_example(n=3000)
    L = (3000 / 1.25) ** (1 / 3)
    pos = inputs.random_positions(3000, [L, L, L], seed=3)
    s = System(pos, [L, L, L], pair={(0, 0): lj_pair(rc=1.12246, caprad=0.8)}, skin=0.3)
    got = s.neighbors(cap=128)
    ref = oracle.neighbors(pos, [L, L, L], 1.12246 + 0.3)
    assert all(np.array_equal(a, b) for a, b in zip(got, ref))
    s.close()


TILE_BUILD_CASES = [
    # (name, n, density, rc, cell_factor, nl_capacity, box aspect)
    ("wca_cf2", 3000, 0.8442, WCA, 2, 40, (1.0, 1.0, 1.0)),
    ("wca_cf1", 3000, 0.8442, WCA, 1, 40, (1.0, 1.0, 1.0)),
    ("lj_cf1", 4000, 0.8442, 2.5, 1, 152, (1.0, 1.0, 1.0)),
    ("lj_cf2", 4000, 0.8442, 2.5, 2, 248, (1.0, 1.0, 1.0)),
    ("lj_noncubic", 4000, 0.8442, 2.5, 1, 160, (1.0, 1.15, 0.87)),
    ("lj_dense", 2000, 1.2, 2.5, 1, 256, (1.0, 1.0, 1.0)),
    ("box_3_cells", 200, 0.3, 2.5, 1, 200, (1.0, 1.0, 1.0)),
]


@pytest.mark.parametrize("case", TILE_BUILD_CASES, ids=[c[0] for c in TILE_BUILD_CASES])
def test_tile_list_build_equals_per_particle_build(case):
    """The tile list build (one wavefront per 64 particles, candidates through
    the scalar cache, 16-bit prefilter) yields the per-particle build's rows
    entry for entry (same order), and trajectories over several rebuilds are
    then bitwise equal."""
    from paper_2608_14911_amd import md
    name, n, rho, rc, cf, cap, asp = case
    banner("tile NL %s n=%d cap=%d cf=%d" % (name, n, cap, cf))
    L0 = (n / rho / (asp[0] * asp[1] * asp[2])) ** (1.0 / 3.0)
    box = [L0 * a for a in asp]
    skin = 0.3
    pos = tricky(11, n, min(box), rc + skin)
    pos = inputs.wrap_into_box(pos * (np.asarray(box) / min(box)), box)
    vel = np.random.default_rng(12).normal(size=(n, 3))
    vel -= vel.mean(0)
    sys = []
    for flags in (md.MD_CFG_NL_TILES, md.MD_CFG_NL_PER_PARTICLE):
        sys.append(System(pos, box, vel, pair={(0, 0): lj_pair(rc=rc, caprad=0.8)}, skin=skin,
                          dt=0.002, nl_capacity=cap, cell_factor=cf, flags=flags, precision="fp32"))
    rows = [s.neighbors(cap=cap, sort=False) for s in sys]
    assert sum(len(r) for r in rows[0]) > 0
    for i in range(n):
        assert np.array_equal(rows[0][i], rows[1][i]), i
    ref = oracle.neighbors(pos, box, rc + skin)
    for i in range(n):
        assert np.array_equal(np.sort(rows[0][i]), ref[i]), i
    for s in sys:
        assert s.observables()["nl_max_count"] == max(len(r) for r in ref)
    for s in sys:
        s.step(40)
    st = [s.get_state() for s in sys]
    nr = [s.observables()["n_rebuilds"] for s in sys]
    assert nr[0] == nr[1] and nr[0] >= 2
    assert np.array_equal(st[0]["pos"], st[1]["pos"])
    assert np.array_equal(st[0]["vel"], st[1]["vel"])
    rows = [s.neighbors(cap=cap, sort=False) for s in sys]
    for i in range(n):
        assert np.array_equal(rows[0][i], rows[1][i]), i
    for s in sys:
        s.close()


@pytest.mark.parametrize("cf", [1, 2])
def test_tile_list_build_equals_per_particle_build_kg1k(cf):
    """Same for the bonded melt: rows and the bond/angle remap feed bitwise
    equal trajectories."""
    from paper_2608_14911_amd import md
    w = kg1k_state(1.5)
    banner("tile NL kg1k (pushed off, bending on) cf=%d" % cf)
    sys = [from_workload(w, precision="fp32", flags=f, cell_factor=cf)
           for f in (md.MD_CFG_NL_TILES, md.MD_CFG_NL_PER_PARTICLE)]
    rows = [s.neighbors(cap=64, sort=False) for s in sys]
    assert all(np.array_equal(a, b) for a, b in zip(*rows))
    for s in sys:
        s.step(200)
    st = [s.get_state() for s in sys]
    assert sys[0].observables()["n_rebuilds"] >= 2
    assert np.array_equal(st[0]["pos"], st[1]["pos"])
    assert np.array_equal(st[0]["vel"], st[1]["vel"])
    for s in sys:
        s.close()


def test_nl_overflow_is_reported_with_needed_capacity():
    banner("NL overflow")
    from paper_2608_14911_amd import md
    pos, box = inputs.fcc_lattice(6, 0.8442)
    with pytest.raises(md.MDError) as e:
        System(pos, box, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, nl_capacity=40)
    assert e.value.code == md.MD_ERR_NL_OVERFLOW
    # the longest row, and the capacity to ask for: rounded up to a multiple of 8
    assert "has 78 neighbours" in str(e.value) and ">= 80" in str(e.value)


def test_fcc_lattice_counts_and_sums():
    banner("FCC 6^3 lattice sums")
    pos, box = inputs.fcc_lattice(6, 0.8442)
    n = pos.shape[0]
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        s = System(pos, box, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, precision=prec)
        nl = s.neighbors(cap=128)
        assert all(len(x) == 78 for x in nl)
        o = s.observables()
        assert rel(o["e_pair"] / n, -6.332811992580958) < tol
        assert rel(o["virial"] / n, -22.158199254035495) < tol
        assert o["nl_max_count"] == 78
        F = s.forces()
        assert np.abs(F).max() < (1e-9 if prec == "fp64" else 2e-4)
        s.close()


def lj_liquid(ncell=6, seed=4, jitter=0.2):
    pos, box = inputs.fcc_lattice(ncell, 0.8442, jitter=jitter, seed=seed)
    return pos, box


@pytest.mark.parametrize("prec,tol,cf", [("fp64", 1e-12, 1), ("fp32", 1e-5, 1), ("fp32", 1e-5, 2)])
def test_lj_forces_energy_virial(prec, tol, cf):
    banner("LJ forces %s cell_factor=%d" % (prec, cf))
    pos, box = lj_liquid(ncell=8)
    s = System(pos, box, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, precision=prec, cell_factor=cf)
    Fg = s.forces()
    o = s.observables()
    Fo, oo = oracle.forces(pos, box, oracle_pp(rc=2.5), want_fscale=True)
    assert_forces_close(Fg, Fo, oo["fscale"], tol, "LJ " + prec)
    assert rel(o["e_pair"], oo["e_pair"]) < tol
    assert rel(o["virial"], oo["virial"]) < tol
    np.testing.assert_allclose(o["virial_tensor"], oo["virial_tensor"], rtol=tol * 10,
                               atol=tol * abs(oo["virial"]))
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_kg_forces_with_bonds_angles_capped(prec, tol):
    banner("KG raw-walk forces %s" % prec)
    w = inputs.random_walk_chains(20, 50, 0.85, seed=9)
    pos, box = w["pos"], w["box"]
    s = System(pos, box, pair={(0, 0): lj_pair(rc=WCA, caprad=0.8)}, bonds=w["bonds"], angles=w["angles"],
               skin=0.4, precision=prec, k_bend=1.5)
    Fg = s.forces()
    o = s.observables()
    Fo, oo = oracle.forces(pos, box, oracle_pp(rc=WCA, caprad=0.8), bonds=w["bonds"], angles=w["angles"],
                           k_bend=1.5, want_fscale=True)
    assert_forces_close(Fg, Fo, oo["fscale"], tol, "KG " + prec)
    for k in ("e_pair", "e_bond", "e_angle", "virial"):
        assert rel(o[k], oo[k]) < tol * 10, k
    s.close()


def test_multitype_forces():
    banner("multi-type forces")
    g = np.random.default_rng(12)
    pos, box = lj_liquid(ncell=6, seed=6)
    n = pos.shape[0]
    types = g.integers(0, 3, size=n).astype(np.int32)
    rows = {(0, 0): (1.0, 1.0, 2.5, math.nan, 0.0), (0, 1): (0.5, 1.1, 2.2, math.nan, 0.0),
            (1, 1): (1.5, 0.9, 2.0, 0.0, 0.0), (0, 2): (0.8, 1.0, WCA, math.nan, 0.0),
            (1, 2): (0.0, 1.0, 1.5, math.nan, 0.0), (2, 2): (1.2, 1.05, 2.4, math.nan, 0.0)}
    pp = oracle.pair_table(3, {k: oracle.pair_params(*v) for k, v in rows.items()})
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5)):
        s = System(pos, box, types=types, n_types=3, pair=rows, masses=(1.0, 2.0, 0.5), skin=0.3,
                   precision=prec)
        Fg = s.forces()
        Fo, oo = oracle.forces(pos, box, pp, ntypes=3, type=types, want_fscale=True)
        assert_forces_close(Fg, Fo, oo["fscale"], tol, "multitype " + prec)
        assert rel(s.observables()["e_pair"], oo["e_pair"]) < tol
        s.close()


def oracle_params(w, pp, integrator):
    return {"box": w["box"], "pp": pp, "ntypes": 1, "mass_by_type": np.array([1.0]), "dt": w["dt"],
            "integrator": integrator, "temperature": w["temperature"], "gamma": w["gamma"],
            "seed": w["seed"], "bonds": w.get("bonds"), "angles": w.get("angles"),
            "fene_K": w.get("fene_K", 30.0), "fene_R0": w.get("fene_R0", 1.5), "k_bend": w.get("k_bend", 0.0)}


@pytest.mark.parametrize("k_bend", [0.0, 1.5])
def test_trajectory_fp64_langevin_kg1k(k_bend):
    banner("trajectory KG1k fp64 langevin 100 steps k_bend=%g" % k_bend)
    w = kg1k_state(k_bend)
    pp = oracle_pp(rc=WCA)
    s = from_workload(w, precision="fp64")
    s.step(100)
    assert s.status() == 0
    hg = s.history()
    sg = s.get_state()
    n = w["pos"].shape[0]
    st = {"pos": w["pos"].copy(), "vel": w["vel"].copy(), "image": np.zeros((n, 3), dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    ho = oracle.run(st, oracle_params(w, pp, oracle.LANGEVIN), 100)
    assert sg["step"] == 100 and st["step"] == 100
    np.testing.assert_allclose(unwrap(sg, w["box"]), unwrap(st, w["box"]), rtol=0, atol=1e-9)
    np.testing.assert_allclose(sg["vel"], st["vel"], rtol=0, atol=1e-8)
    assert len(hg) == 100
    for k in range(100):
        assert hg[k]["step"] == k
        for key, col in (("e_pair", 0), ("e_bond", 1), ("e_angle", 2), ("e_kin", 3), ("virial", 4)):
            assert abs(hg[k][key] - ho[k, col]) <= 1e-9 * max(1.0, abs(ho[k, col])), (k, key)
    assert hg[-1]["n_rebuilds"] >= 2
    s.close()


def test_trajectory_fp64_nve_lj():
    banner("trajectory LJ fp64 NVE 200 steps")
    w = inputs.workload_lj(ncell=6, seed=21)
    s = from_workload(w, precision="fp64")
    s.step(200)
    sg = s.get_state()
    hg = s.history()
    st = {"pos": w["pos"].copy(), "vel": w["vel"].copy(), "image": np.zeros(w["pos"].shape, dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    ho = oracle.run(st, oracle_params(w, oracle_pp(rc=2.5), oracle.NVE), 200)
    np.testing.assert_allclose(unwrap(sg, w["box"]), unwrap(st, w["box"]), rtol=0, atol=1e-8)
    e = np.array([h["e_pair"] + h["e_kin"] for h in hg])
    eo = ho[:, 0] + ho[:, 3]
    np.testing.assert_allclose(e, eo, rtol=1e-9)
    s.close()


def test_fp32_step_parity_and_statistics_lj():
    banner("LJ fp32 single step + short run")
    w = inputs.workload_lj(ncell=6, seed=22)
    s = from_workload(w, precision="fp32")
    s.step(1)
    sg = s.get_state()
    st = {"pos": w["pos"].copy(), "vel": w["vel"].copy(), "image": np.zeros(w["pos"].shape, dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    oracle.run(st, oracle_params(w, oracle_pp(rc=2.5), oracle.NVE), 1)
    # one step moves x by dt^2/2 F: FP32 force error 1e-5 relative -> tiny
    np.testing.assert_allclose(unwrap(sg, w["box"]), unwrap(st, w["box"]), rtol=0, atol=1e-8)
    s.step(399)
    h = s.history()
    e = np.array([x["e_total"] for x in h])
    n = w["pos"].shape[0]
    assert np.abs(e - e[0]).max() / n < 2e-3
    s.close()


def test_determinism_and_checkpoint_bitwise():
    banner("determinism + checkpoint resume")
    w = kg1k_state(1.5)
    runs = []
    for _ in range(2):
        s = from_workload(w, precision="fp32")
        s.step(120)
        runs.append(s.get_state())
        s.close()
    assert np.array_equal(runs[0]["pos"], runs[1]["pos"]) and np.array_equal(runs[0]["vel"], runs[1]["vel"])
    s = from_workload(w, precision="fp32")
    s.step(60)
    ck = s.get_state()
    s.close()
    s2 = from_workload(w, precision="fp32")
    s2.set_state(ck)
    s2.step(60)
    r = s2.get_state()
    assert r["step"] == 120
    assert np.array_equal(r["pos"], runs[0]["pos"])
    assert np.array_equal(r["vel"], runs[0]["vel"])
    assert np.array_equal(r["image"], runs[0]["image"])
    s2.close()


def test_gpu_pushoff_kg_melt():
    """The GPU push-off ladder on raw random walks (200 chains x 50 beads at
    density 0.85) leaves no bead pair closer than 0.75 and no bond longer
    than 1.3, checked on the oracle's brute-force neighbour sets."""
    from paper_2608_14911_amd.system import push_off
    w = inputs.workload_kg(200, 50, seed=31)
    banner("push-off KG 200x50 seed=31")
    w0 = dict(w, caprad=1.0, dt=0.002, gamma=1.0, vel=np.zeros_like(w["pos"]))
    s = from_workload(w0, precision="fp32", nl_capacity=256)
    push_off(s, w["rc"])
    st = s.get_state()
    s.close()
    pos = st["pos"]
    L = w["box"]
    b = w["bonds"]
    d = pos[b[:, 1]] - pos[b[:, 0]]
    d -= L * np.round(d / L)
    assert np.sqrt((d * d).sum(1)).max() < 1.3
    nl = oracle.neighbors(pos, L, 0.75)
    assert all(len(r) == 0 for r in nl)


@pytest.mark.parametrize("build", ["tiles", "per_particle"])
def test_degenerate_systems(build):
    """Edge cases through both list builds: one particle (no neighbour, zero
    force, free flight); a pair exactly at the cutoff and one ulp inside it;
    65 particles (a full tile and a tile of one); particles farther apart
    than the list radius (every list empty)."""
    from paper_2608_14911_amd import md
    from paper_2608_14911_amd.system import nl_build_flags
    flags = nl_build_flags(build)
    banner("degenerate systems, %s build" % build)
    L = 10.0
    # one particle
    s = System(np.array([[1.0, 2.0, 3.0]]), [L, L, L], np.array([[0.5, -0.25, 0.125]]),
               pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, dt=0.01, flags=flags)
    assert [len(r) for r in s.neighbors(cap=8)] == [0]
    assert np.abs(s.forces()).max() == 0.0
    s.step(10)
    st = s.get_state()
    np.testing.assert_allclose(st["pos"][0], [1.05, 1.975, 3.0125], rtol=0, atol=1e-12)
    s.close()
    # a pair at the cutoff (no force, listed) and one ulp inside it (force)
    for r, expect_force in [(2.5, False), (np.nextafter(2.5, 0.0), True)]:
        # 0.5 + r is exact at both distances, so the FP64 difference is r itself
        pos = np.array([[0.5, 5.0, 5.0], [0.5 + r, 5.0, 5.0]])
        assert pos[1, 0] - pos[0, 0] == r
        s = System(pos, [L, L, L], pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, precision="fp64", flags=flags)
        F = s.forces()
        Fo, _ = oracle.forces(pos, [L, L, L], oracle_pp(rc=2.5))
        assert np.array_equal(F != 0.0, Fo != 0.0) and (np.abs(F).max() > 0) == expect_force
        np.testing.assert_allclose(F, Fo, rtol=1e-12, atol=0)
        assert [len(x) for x in s.neighbors(cap=8)] == [1, 1]
        s.close()
    # 65 particles: a full tile and a tile of one
    g = np.random.default_rng(21)
    pos = g.uniform(0, L, size=(65, 3))
    s = System(pos, [L, L, L], pair={(0, 0): lj_pair(rc=2.5, caprad=0.8)}, skin=0.3, flags=flags)
    ref = oracle.neighbors(pos, [L, L, L], 2.8)
    assert all(np.array_equal(a, b) for a, b in zip(s.neighbors(cap=64), ref))
    Fo, oo = oracle.forces(pos, [L, L, L], oracle_pp(rc=2.5, caprad=0.8), want_fscale=True)
    assert_forces_close(s.forces(), Fo, oo["fscale"], 1e-5, "65 particles")
    s.close()
    # sparse: a 4x4x4 lattice of spacing 3 > rv in a box of 12
    grid = np.stack(np.meshgrid(*[np.arange(4) * 3.0 + 0.5] * 3, indexing="ij"), -1).reshape(-1, 3)
    s = System(grid, [12.0] * 3, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, flags=flags)
    assert all(len(x) == 0 for x in s.neighbors(cap=8))
    assert np.abs(s.forces()).max() == 0.0
    assert s.observables()["nl_max_count"] == 0
    s.close()


def test_odd_list_capacity_rows_in_last_batch():
    """A requested capacity that is not a multiple of 8, set just above the
    longest row, so that the longest rows end inside the last batch of 8
    slots the fast FP32 kernel streams.  The library rounds the capacity up
    to 8; forces equal a run with a roomy capacity bit for bit (same rows, same
    order) and agree with the oracle within the FP32 tolerance."""
    banner("odd list capacity (LJ fast path, tiles and per-particle builds)")
    from paper_2608_14911_amd import md
    pos, box = lj_liquid(ncell=8, seed=5)
    ref = oracle.neighbors(pos, box, 2.8)
    longest = max(len(r) for r in ref)
    cap = longest + 1 if (longest + 1) % 8 else longest + 2
    assert cap % 8 != 0 and longest > (cap & ~7)
    Fo, oo = oracle.forces(pos, box, oracle_pp(rc=2.5), want_fscale=True)
    for flags in (md.MD_CFG_NL_TILES, md.MD_CFG_NL_PER_PARTICLE):
        got = []
        for c in (cap, 256):
            s = System(pos, box, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, nl_capacity=c, flags=flags)
            assert md.md_plan_config(s.cfg)["nl_capacity"] == (c + 7) // 8 * 8
            got.append((s.forces(), s.observables()))
            s.close()
        assert np.array_equal(got[0][0], got[1][0])
        assert got[0][1]["e_pair"] == got[1][1]["e_pair"] and got[0][1]["nl_max_count"] == longest
        assert_forces_close(got[0][0], Fo, oo["fscale"], 1e-5, "odd capacity")
        print("odd capacity %d (rounded %d), longest row %d: max |dF| / scale %.2e" % (
            cap, (cap + 7) // 8 * 8, longest,
            (np.linalg.norm(got[0][0] - Fo, axis=1) / oo["fscale"]).max()), flush=True)


def test_set_params_rejects_a_skin_change():
    """md_set_params keeps the list radius and the half-skin rebuild threshold
    of md_init, so a different skin is an argument error (a larger cutoff with
    a smaller skin would keep the old threshold and miss pairs)."""
    banner("md_set_params skin change rejected")
    from paper_2608_14911_amd import md
    pos, box = lj_liquid(ncell=6)
    s = System(pos, box, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3)
    with pytest.raises(md.MDError) as e:
        s.set_params(pair={(0, 0): lj_pair(rc=2.7)}, skin=0.1)
    assert e.value.code == md.MD_ERR_ARG and "skin" in str(e.value)
    s.cfg.skin = 0.3
    with pytest.raises(md.MDError) as e:
        s.set_params(pair={(0, 0): lj_pair(rc=2.7)})
    assert e.value.code == md.MD_ERR_ARG
    # a smaller cutoff with the same skin is accepted and gives the oracle's forces
    s.set_params(pair={(0, 0): lj_pair(rc=2.2)})
    Fo, oo = oracle.forces(pos, box, oracle_pp(rc=2.2), want_fscale=True)
    assert_forces_close(s.forces(), Fo, oo["fscale"], 1e-5, "rc 2.2 after set_params")
    s.close()
