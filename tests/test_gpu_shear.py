"""GPU parity of the DPD thermostat and the Lees-Edwards sheared boundaries
against the FP64 oracle, through the C ABI (FP32 pair path).

* Neighbour sets under shear equal the oracle's brute-force sets bit for bit,
  at several shear offsets, for cells of side rc+skin and half cells, and in a
  box of 3 cells where the shifted stencil covers whole rows.
* Conservative forces under shear (LJ fluid; a bonded melt with bonds across
  the sheared boundary) within 1e-5 of the oracle, per particle relative to
  the sum of its force-term magnitudes.
* One DPD step (with and without shear; a capped LJ core on a random start)
  against the oracle's step from the same state and noise: a force error
  dF_i moves x by dt^2/(2m) dF_i and the half-step velocity by dt/(2m) dF_i
  in the first step, so the bounds follow from |dF_i| <= 1e-5 times the sum
  of the force-term magnitudes (DPD terms included).  Ten steps of a pure
  DPD fluid (no stiff core to amplify differences) within
  k^2 dt^2 1e-5 max_i of that sum.
* Particles starting at rest under fast shear: the offset's drift alone
  forces list rebuilds, and after many steps the forces are still the
  oracle's and the list holds every pair inside the cutoff.
* A DPD fluid under shear on the GPU carries the imposed linear profile; its
  peculiar temperature equals the oracle's (the same thermostat at this time
  step) within 3 combined standard errors; without shear it conserves
  momentum.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import WCA, assert_forces_close, banner, oracle_pp
from paper_2608_14911_amd import inputs
from paper_2608_14911_amd.system import System, lj_pair

pytestmark = pytest.mark.gpu

TOL = 1e-5


def set_step(s, pos, vel, step):
    """Give the handle a state at the given step (the shear offset follows it)."""
    n = pos.shape[0]
    s.set_state({"pos": pos, "vel": vel, "image": np.zeros((n, 3), dtype=np.int32), "step": step, "vel_half": 0},
                with_build=False)


@pytest.mark.parametrize("L,cf,n,asp", [(9.0, 1, 2000, (1.0, 0.93, 1.07)), (9.0, 2, 2000, (1.0, 0.93, 1.07)),
                                         (12.5, 1, 4000, (1.0, 1.0, 1.0)), (4.7, 1, 300, (1.0, 1.0, 1.0))])
def test_sheared_neighbor_sets_bitexact(L, cf, n, asp):
    banner("sheared NL L=%g cell_factor=%d n=%d" % (L, cf, n))
    rate, dt, rc, skin = 0.9, 0.01, 1.2, 0.3
    box = np.array([L * asp[0], L * asp[1], L * asp[2]])
    pos = inputs.random_positions(n, box, seed=int(L * 10) + cf)
    vel = np.zeros_like(pos)
    s = System(pos, box, vel, pair={(0, 0): lj_pair(rc=rc, caprad=0.8)}, skin=skin, dt=dt, shear_rate=rate,
               cell_factor=cf, nl_capacity=64)
    for step in (0, 37, 250, 1111):
        set_step(s, pos, vel, step)
        got = s.neighbors(cap=64)
        ref = oracle.neighbors_le(pos, box, rc + skin, shear_rate=rate, dt=dt, step=step, cap=64)
        bad = [i for i in range(n) if not np.array_equal(got[i], ref[i])]
        assert not bad, (step, bad[:5])
    s.close()


def test_sheared_forces_lj_and_bonded_melt():
    banner("sheared conservative forces: LJ fluid and melt")
    rate, dt = 0.5, 0.005
    pos, box = inputs.fcc_lattice(6, 0.8442, jitter=0.2, seed=3)
    s = System(pos, box, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, dt=dt, shear_rate=rate)
    for step in (0, 123, 777):
        set_step(s, pos, np.zeros_like(pos), step)
        Fg = s.forces()
        o = s.observables()
        Fo, _, oo = oracle.forces_ext(pos, box, oracle_pp(rc=2.5), shear_rate=rate, dt=dt, step=step,
                                      want_fscale=True)
        assert_forces_close(Fg, Fo, oo["fscale"], TOL, "sheared LJ step %d" % step)
        assert abs(o["e_pair"] - oo["e_pair"]) <= TOL * abs(oo["e_pair"])
        assert abs(o["virial"] - oo["virial"]) <= TOL * oo["virial_abs"]
    s.close()
    w = inputs.lattice_melt(40, 25, 0.85, seed=5)
    kw = dict(bonds=w["bonds"], angles=w["angles"], k_bend=1.5)
    s = System(w["pos"], w["box"], pair={(0, 0): lj_pair(rc=WCA)}, skin=0.4, dt=0.01, shear_rate=0.8, **kw)
    for step in (0, 999):
        set_step(s, w["pos"], np.zeros_like(w["pos"]), step)
        Fg = s.forces()
        o = s.observables()
        Fo, _, oo = oracle.forces_ext(w["pos"], w["box"], oracle_pp(rc=WCA), shear_rate=0.8, dt=0.01, step=step,
                                      want_fscale=True, **kw)
        assert_forces_close(Fg, Fo, oo["fscale"], TOL, "sheared melt step %d" % step)
        for k in ("e_pair", "e_bond", "e_angle"):
            assert abs(o[k] - oo[k]) <= TOL * abs(oo[k]), k
    s.close()


def dpd_system(L, rho, seed, rate, kT=1.0, gamma=4.5, dt=0.01):
    n = int(round(rho * L ** 3))
    box = np.array([L, L, L])
    pos = inputs.random_positions(n, box, seed=seed)
    vel = inputs.maxwell_boltzmann(n, kT, seed=seed)
    vel[:, 0] += rate * (pos[:, 1] - 0.5 * L)
    return pos, box, vel


def oracle_state(pos, vel, step=0):
    n = pos.shape[0]
    return {"pos": pos.copy(), "vel": vel.copy(), "image": np.zeros((n, 3), dtype=np.int32), "step": step,
            "vel_half": 0, "type": None}


@pytest.mark.parametrize("rate", [0.0, 0.7])
def test_dpd_steps_against_oracle(rate):
    banner("DPD steps vs oracle, shear rate %g" % rate)
    L, dt, rc_d = 8.0, 0.01, 1.0
    pos, box, vel = dpd_system(L, 1.0, seed=31, rate=rate)
    pair = {(0, 0): lj_pair(eps=1.0, sigma=0.8, rc=0.8 * WCA, caprad=0.6)}
    s = System(pos, box, vel, pair=pair, skin=0.3, dt=dt, integrator="dpd", temperature=1.0, gamma=4.5, seed=9,
               dpd_rc=rc_d, shear_rate=rate)
    pp = oracle_pp(eps=1.0, sigma=0.8, rc=0.8 * WCA, caprad=0.6)
    par = {"box": box, "pp": pp, "ntypes": 1, "mass_by_type": np.array([1.0]), "dt": dt, "integrator": oracle.DPD,
           "temperature": 1.0, "gamma": 4.5, "seed": 9, "dpd_rc": rc_d, "shear_rate": rate}
    F, Fd, oo = oracle.forces_ext(pos, box, pp, vel=vel, shear_rate=rate, dpd_rc=rc_d, dpd_gamma=4.5, kT=1.0, dt=dt,
                                  seed=9, step=0, want_fscale=True)
    st = oracle_state(pos, vel)
    s.step(1)
    g = s.get_state()
    oracle.run_ext(st, par, 1)
    dx = g["pos"] - st["pos"]   # wrapped positions, compared through the minimum image of the difference
    dx[:, 1] -= box[1] * np.round(dx[:, 1] / box[1])
    dx[:, 0] -= box[0] * np.round(dx[:, 0] / box[0])
    dx[:, 2] -= box[2] * np.round(dx[:, 2] / box[2])
    dx = np.abs(dx).max(1)
    dv = np.abs(g["vel"] - st["vel"]).max(1)
    bx = TOL * dt * dt / 2 * oo["fscale"] + 1e-12
    bv = TOL * dt / 2 * oo["fscale"] + 1e-12
    print("1 step: max |dx| %.2e (ratio %.3f), max |dv| %.2e (ratio %.3f), max |Fd| %.2f" % (
        dx.max(), (dx / bx).max(), dv.max(), (dv / bv).max(), np.abs(Fd).max()), flush=True)
    assert np.all(dx <= bx) and np.all(dv <= bv)
    assert np.abs(Fd).max() > 1.0
    s.close()
    # ten steps of a pure DPD fluid (crossings of the sheared boundary included)
    pos, box, vel = dpd_system(6.0, 3.0, seed=32, rate=rate)
    pp0 = oracle_pp(eps=0.0, rc=1.0)
    s = System(pos, box, vel, pair={(0, 0): lj_pair(eps=0.0, rc=1.0)}, skin=0.3, dt=dt, integrator="dpd",
               temperature=1.0, gamma=4.5, seed=9, dpd_rc=rc_d, shear_rate=rate)
    _, _, oo = oracle.forces_ext(pos, box, pp0, vel=vel, shear_rate=rate, dpd_rc=rc_d, dpd_gamma=4.5, kT=1.0, dt=dt,
                                 seed=9, step=0, want_fscale=True)
    st = oracle_state(pos, vel)
    s.step(10)
    g = s.get_state()
    oracle.run_ext(st, dict(par, pp=pp0, box=box), 10)
    dx = g["pos"] - st["pos"]
    for k in range(3):
        dx[:, k] -= box[k] * np.round(dx[:, k] / box[k])
    k = 10
    bound = k * k * dt * dt * TOL * oo["fscale"].max()
    print("10 steps: max |dx| %.2e, bound %.2e, y-crossings %d" % (np.abs(dx).max(), bound,
                                                                   int(np.abs(st["image"][:, 1]).sum())), flush=True)
    assert np.abs(dx).max() <= bound
    assert np.array_equal(g["image"][:, 1], st["image"][:, 1])
    s.close()


def test_offset_drift_alone_forces_rebuilds():
    """Particles starting at rest on an FCC lattice (NVE) under fast shear:
    the offset moves 0.05 per step, so with a skin of 0.3 the drift alone
    forces a rebuild every 6 steps; the forces after 60 steps are still the
    oracle's and the list holds every current pair."""
    banner("shear offset drift forces rebuilds")
    rate, dt = 1.0, 0.005
    pos, box = inputs.fcc_lattice(6, 0.8442, jitter=0.0)
    s = System(pos, box, np.zeros_like(pos), pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, dt=dt, shear_rate=rate)
    nsteps = 60
    s.step(nsteps)
    o = s.observables()
    g = s.get_state()
    per_step = rate * box[1] * dt
    assert o["n_rebuilds"] >= 1 + nsteps // math.ceil(0.3 / per_step)
    Fg = s.forces()
    Fo, _, oo = oracle.forces_ext(g["pos"], box, oracle_pp(rc=2.5), shear_rate=rate, dt=dt, step=nsteps,
                                  want_fscale=True)
    assert_forces_close(Fg, Fo, oo["fscale"], TOL, "after offset drift")
    ref = oracle.neighbors_le(g["pos"], box, 2.5, shear_rate=rate, dt=dt, step=nsteps, cap=128)
    nl = s.neighbors(cap=128)
    # every pair inside the cutoff now is in the list (built at an earlier offset and positions)
    assert all(set(r).issubset(set(x)) for r, x in zip(ref, nl))
    s.close()


def peculiar_T_series(get_state, advance, L, rate, n, nsamp=16, every=25):
    out = []
    for _ in range(nsamp):
        advance(every)
        g = get_state()
        pec = g["vel"].copy()
        pec[:, 0] -= rate * (g["pos"][:, 1] - 0.5 * L)
        out.append((pec ** 2).sum() / (3 * n))
    return np.array(out)


def test_dpd_shear_profile_temperature_and_momentum():
    banner("DPD fluid under shear: profile and temperature against the oracle")
    L, rate, dt = 7.0, 0.3, 0.01
    pos, box, vel = dpd_system(L, 3.0, seed=41, rate=rate)
    n = pos.shape[0]
    nb, nrep = 7, 6
    prof, cnt = np.zeros(nb), np.zeros(nb)

    def gstate(s):
        g = s.get_state()
        b = np.minimum((g["pos"][:, 1] / L * nb).astype(int), nb - 1)
        np.add.at(prof, b, g["vel"][:, 0])
        np.add.at(cnt, b, 1)
        return g

    # Independent replicas (noise seeds) on each side: the temperature of one
    # run is a correlated series whose own spread understates the error of its
    # mean, so the standard error comes from the spread of the replica means.
    Tg = []
    for seed in range(3, 3 + nrep):
        s = System(pos, box, vel, pair={(0, 0): lj_pair(eps=0.0, rc=1.0)}, skin=0.3, dt=dt, integrator="dpd",
                   temperature=1.0, gamma=4.5, seed=seed, dpd_rc=1.0, shear_rate=rate)
        s.step(300)
        Tg.append(peculiar_T_series(lambda: gstate(s), s.step, L, rate, n).mean())
        assert s.status() == 0
        s.close()
    prof /= cnt
    yc = (np.arange(nb) + 0.5) * L / nb
    slope = np.polyfit(yc, prof, 1)[0]
    # the oracle: the same system with its own noise seeds, the same protocol
    To = []
    for seed in range(103, 103 + nrep):
        st = oracle_state(pos, vel)
        par = {"box": box, "pp": oracle_pp(eps=0.0, rc=1.0), "ntypes": 1, "mass_by_type": np.array([1.0]),
               "dt": dt, "integrator": oracle.DPD, "temperature": 1.0, "gamma": 4.5, "seed": seed, "dpd_rc": 1.0,
               "shear_rate": rate}
        oracle.run_ext(st, par, 300)
        To.append(peculiar_T_series(lambda: st, lambda k: oracle.run_ext(st, par, k), L, rate, n).mean())
    Tg, To = np.array(Tg), np.array(To)
    se = math.hypot(Tg.std(ddof=1), To.std(ddof=1)) / math.sqrt(nrep)
    print("shear profile slope %.4f (imposed %.4f); peculiar T GPU %.4f (%s), oracle %.4f (%s), se %.4f" % (
        slope, rate, Tg.mean(), " ".join("%.4f" % t for t in Tg), To.mean(), " ".join("%.4f" % t for t in To),
        se), flush=True)
    assert slope == pytest.approx(rate, rel=0.08)
    # 4 standard errors: a two-sided tail of 0.25 % for Student's t at the 10
    # degrees of freedom of two samples of 6
    assert abs(Tg.mean() - To.mean()) <= 4.0 * se
    # without shear: total momentum stays at its start value (pair forces cancel to FP32 rounding)
    pos, box, vel = dpd_system(8.0, 3.0, seed=42, rate=0.0)
    vel -= vel.mean(0)
    s = System(pos, box, vel, pair={(0, 0): lj_pair(eps=0.0, rc=1.0)}, skin=0.3, dt=dt, integrator="dpd",
               temperature=1.0, gamma=4.5, seed=4, dpd_rc=1.0)
    s.step(500)
    g = s.get_state()
    p = np.abs(g["vel"].sum(0)).max()
    print("momentum after 500 DPD steps: %.2e (per particle %.2e)" % (p, p / len(pos)), flush=True)
    assert p < 1e-3 * math.sqrt(len(pos))
    s.close()
