"""Trajectory-level parity of the HIP path against the FP64 oracle.

* The 1,000-bead Kremer-Grest melt (20 x 50, WCA + FENE, Langevin T = 1,
  gamma = 1, dt = 0.01, skin 0.3) over its full 1,000 steps from the oracle's
  pushed-off state: block averages (10 blocks of 100 steps) of the pair and
  bond energies per bead, the pressure and the temperature, and the
  bond-length histogram, agree with the oracle's within 3 combined standard
  errors.  The FP64 path runs with the oracle's thermostat seed; the FP32 path
  with another seed, so its statistics are an independent sample.  The
  temperature also equals the thermostat's kT = 1 within 3 standard errors
  plus 0.01 (the O(dt) bias of the on-step velocity at dt = 0.01).
* One Langevin step of the bonded melt through the fused FP32 kernel the
  2M-bead benchmark times (single type, cubic box: the fast bonded kernel),
  against the oracle's FP64 step from the same state and noise.  A force
  error dF_i moves x by dt^2/(2m) dF_i and the half-step velocity by
  dt/(2m) dF_i in that step, so with |dF_i| <= 1e-5 sum_j |f_ij| the
  per-particle bounds follow; after k steps the position bound is
  k^2 dt^2 1e-5 max_i sum_j |f_ij|.
* One step of sampled batch members (LJ fluids and melts) against the oracle
  with each member's own parameters, with the same per-particle bounds.
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import WCA, banner, oracle_pp, unwrap
from kg_fixture import kg1k_state
from paper_2608_14911_amd import inputs
from paper_2608_14911_amd.system import Batch, from_workload

pytestmark = pytest.mark.gpu

TOL = 1e-5          # FP32 force tolerance, relative to sum_j |f_ij|
NBLOCK = 10
EDGES = np.linspace(0.80, 1.20, 21)


def kg_oracle_params(w, seed=None):
    return {"box": w["box"], "pp": oracle_pp(rc=w["rc"]), "ntypes": 1, "mass_by_type": np.array([1.0]),
            "dt": w["dt"], "integrator": oracle.LANGEVIN if w["integrator"] == "langevin" else oracle.NVE,
            "temperature": w["temperature"], "gamma": w["gamma"],
            "seed": w["seed"] if seed is None else seed, "bonds": w.get("bonds"), "angles": w.get("angles"),
            "fene_K": w.get("fene_K", 30.0), "fene_R0": w.get("fene_R0", 1.5), "k_bend": w.get("k_bend", 0.0)}


def bond_lengths(pos, bonds, box):
    d = pos[bonds[:, 1]] - pos[bonds[:, 0]]
    d -= box * np.round(d / box)
    return np.sqrt((d * d).sum(1))


def series_stats(hist, bl, n, V):
    """Block means and standard errors of U_pair/N, U_bond/N, P, T and the
    bond-length histogram.  hist columns: e_pair, e_bond, e_angle, e_kin, W."""
    K, W = hist[:, 3], hist[:, 4]
    out = {"upair": hist[:, 0] / n, "ubond": hist[:, 1] / n, "P": (2 * K + W) / (3 * V), "T": 2 * K / (3 * n)}
    res = {}
    for k, x in out.items():
        blk = x.reshape(NBLOCK, -1).mean(1)
        res[k] = (blk.mean(), blk.std(ddof=1) / np.sqrt(NBLOCK))
    h = np.array([np.histogram(x, EDGES)[0] / x.size for x in bl]).reshape(NBLOCK, -1, len(EDGES) - 1).mean(1)
    res["hist"] = (h.mean(0), h.std(0, ddof=1) / np.sqrt(NBLOCK))
    return res


def oracle_series(w, nsteps, every):
    n = w["pos"].shape[0]
    st = {"pos": w["pos"].copy(), "vel": w["vel"].copy(), "image": np.zeros((n, 3), dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    par = kg_oracle_params(w)
    H, B = [], []
    for _ in range(nsteps // every):
        H.append(oracle.run(st, par, every))
        B.append(bond_lengths(st["pos"], w["bonds"], w["box"]))
    return np.concatenate(H), np.array(B)


def gpu_series(w, nsteps, every, precision):
    s = from_workload(w, precision=precision)
    B = []
    for _ in range(nsteps // every):
        s.step(every)
        B.append(bond_lengths(s.get_state()["pos"], w["bonds"], w["box"]))
    h = s.history()
    assert s.status() == 0 and len(h) == nsteps
    H = np.array([[x["e_pair"], x["e_bond"], x["e_angle"], x["e_kin"], x["virial"]] for x in h])
    nreb = s.observables()["n_rebuilds"]
    s.close()
    return H, np.array(B), nreb


@pytest.mark.parametrize("precision,seed_shift", [("fp64", 0), ("fp32", 7)])
def test_kg1k_1000_steps_statistical_parity(precision, seed_shift):
    w = kg1k_state(0.0)
    n = w["pos"].shape[0]
    V = float(np.prod(w["box"]))
    banner("KG1k 1000-step statistics, GPU %s (seed +%d) vs oracle" % (precision, seed_shift))
    Ho, Bo = oracle_series(w, 1000, 10)
    Hg, Bg, nreb = gpu_series(dict(w, seed=w["seed"] + seed_shift), 1000, 10, precision)
    so, sg = series_stats(Ho, Bo, n, V), series_stats(Hg, Bg, n, V)
    for k in ("upair", "ubond", "P", "T"):
        (mg, eg), (mo, eo) = sg[k], so[k]
        z = abs(mg - mo) / np.hypot(eg, eo)
        print("%-6s GPU %.5f +- %.5f  oracle %.5f +- %.5f  |diff|/se %.2f" % (k, mg, eg, mo, eo, z), flush=True)
        assert abs(mg - mo) <= 3.0 * np.hypot(eg, eo), k
    for name, st in (("GPU", sg), ("oracle", so)):
        m, e = st["T"]
        assert abs(m - 1.0) <= 3.0 * e + 0.01, (name, m, e)
    (hg, eg), (ho, eo) = sg["hist"], so["hist"]
    z = np.abs(hg - ho) / np.maximum(np.hypot(eg, eo), 1e-12)
    print("bond-length histogram |diff|/se per bin:", np.round(z, 2), flush=True)
    assert np.all(np.abs(hg - ho) <= 3.0 * np.hypot(eg, eo) + 2e-4)
    assert hg.sum() > 1.0 - 1e-3 and ho.sum() > 1.0 - 1e-3   # the range holds (nearly) every bond
    assert nreb >= 20
    if precision == "fp64":
        # same seed: the FP64 trajectory tracks the oracle's through the first 100 steps
        np.testing.assert_allclose(Hg[:100, :2], Ho[:100, :2], rtol=1e-9, atol=1e-9)


def step_bounds(w, fscale, k=1):
    dt, m = w["dt"], 1.0
    return TOL * dt * dt / (2 * m) * fscale, TOL * dt / (2 * m) * fscale


def test_fp32_kg_langevin_steps_through_fast_bonded_kernel():
    from paper_2608_14911_amd import md
    w = kg1k_state(1.5)
    n = w["pos"].shape[0]
    banner("KG1k FP32 Langevin steps (fast bonded kernel) vs oracle FP64")
    s = from_workload(w, precision="fp32")
    assert s.cfg.force_precision == md.MD_FP32 and s.cfg.n_types == 1
    _, oo = oracle.forces(w["pos"], w["box"], oracle_pp(rc=WCA), bonds=w["bonds"], angles=w["angles"],
                          k_bend=1.5, want_fscale=True)
    st = {"pos": w["pos"].copy(), "vel": w["vel"].copy(), "image": np.zeros((n, 3), dtype=np.int32),
          "step": 0, "vel_half": 0, "type": None}
    par = kg_oracle_params(w)
    s.step(1)
    g = s.get_state()
    oracle.run(st, par, 1)
    bx, bv = step_bounds(w, oo["fscale"])
    dx = np.abs(unwrap(g, w["box"]) - unwrap(st, w["box"])).max(1)
    dv = np.abs(g["vel"] - st["vel"]).max(1)
    print("1 step: max |dx| %.3e (bound ratio %.3f), max |dv| %.3e (bound ratio %.3f)" % (
        dx.max(), (dx / (bx + 1e-12)).max(), dv.max(), (dv / (bv + 1e-12)).max()), flush=True)
    assert np.all(dx <= bx + 1e-12) and np.all(dv <= bv + 1e-12)
    assert dx.max() < 1e-8
    # four more steps: positions within k^2 dt^2 TOL max_i fscale_i
    s.step(4)
    g = s.get_state()
    oracle.run(st, par, 4)
    k = 5
    bound = k * k * w["dt"] ** 2 * TOL * oo["fscale"].max()
    dx = np.abs(unwrap(g, w["box"]) - unwrap(st, w["box"])).max()
    print("5 steps: max |dx| %.3e, bound %.3e" % (dx, bound), flush=True)
    assert dx <= bound
    s.close()


def lattice_replica(r):
    lc = r["chain_len"]
    m = inputs.lattice_melt(r["pos"].shape[0] // lc, lc, r["density"], jitter=0.05, seed=r["seed"])
    out = dict(r)
    out.update(pos=m["pos"], box=m["box"], bonds=m["bonds"], angles=m["angles"])
    return out


def test_batch_members_one_step_vs_oracle():
    """16 members (8 LJ fluids, 8 melts on lattices, 2,048..8,192 particles)
    advance one step in one batch; every member's positions and half-step
    velocities match the oracle's step of that member."""
    reps = inputs.batch_replicas(16, seed=77, n_min=2048, n_max=8192)
    reps = [lattice_replica(r) if r["kind"] == "kg" else r for r in reps]
    banner("batch of 16 members, one step vs oracle (%d particles)" % sum(r["pos"].shape[0] for r in reps))
    b = Batch(reps)
    b.step(1)
    for k, r in enumerate(reps):
        g = b.get_state(k)
        n = r["pos"].shape[0]
        row = r["pair"][(0, 0)]
        w = {"box": r["box"], "rc": row[2], "dt": r["dt"], "integrator": r["integrator"],
             "temperature": r["temperature"], "gamma": r["gamma"], "seed": r["seed"], "bonds": r.get("bonds"),
             "angles": r.get("angles"), "k_bend": r.get("k_bend", 0.0)}
        kw = dict(bonds=r["bonds"], angles=r["angles"], k_bend=r["k_bend"]) if r["kind"] == "kg" else {}
        _, oo = oracle.forces(r["pos"], r["box"], oracle_pp(rc=row[2]), want_fscale=True, **kw)
        st = {"pos": r["pos"].copy(), "vel": r["vel"].copy(), "image": np.zeros((n, 3), dtype=np.int32),
              "step": 0, "vel_half": 0, "type": None}
        oracle.run(st, kg_oracle_params(w), 1)
        bx, bv = step_bounds(w, oo["fscale"])
        dx = np.abs(unwrap(g, r["box"]) - unwrap(st, r["box"])).max(1)
        dv = np.abs(g["vel"] - st["vel"]).max(1)
        print("member %2d (%s, n=%d): max |dx| %.2e ratio %.3f, max |dv| %.2e ratio %.3f" % (
            k, r["kind"], n, dx.max(), (dx / (bx + 1e-12)).max(), dv.max(), (dv / (bv + 1e-12)).max()), flush=True)
        assert g["step"] == 1
        assert np.all(dx <= bx + 1e-12) and np.all(dv <= bv + 1e-12), k
    b.close()
