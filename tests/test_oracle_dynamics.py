"""Pins of the oracle's integrator: VelocityVerlet with the LangevinThermostat
extension (section "Example usage": integrator.addExtension(thermostat)).

Reading of the scheme (the paper gives none): the Langevin force
-gamma m v' + sqrt(2 gamma m kT/dt) xi joins the conservative force inside
velocity Verlet, v' being the half-step velocity.  Facts used:
  * NVE: the fluctuation of the total energy scales with dt^2 and the map is
    time reversible;
  * free particle, derived from the scheme: on-step <v^2> = kT/m exactly,
    half-step <v'^2> = (kT/m)/(1 - gamma dt/2) and <v'_{n+1} v'_n> =
    (1 - gamma dt) <v'^2>.
"""
import numpy as np
import pytest

import oracle
from paper_2608_14911_amd import inputs

WCA = 2.0 ** (1.0 / 6.0)


def lj_state(ncell=4, rho=0.8442, T=0.72, seed=3, rc=2.5):
    pos, box = inputs.fcc_lattice(ncell, rho, jitter=0.05, seed=seed)
    vel = inputs.maxwell_boltzmann(pos.shape[0], T, seed=seed)
    st = {"pos": pos, "vel": vel, "image": np.zeros(pos.shape, dtype=np.int32), "step": 0,
          "vel_half": 0, "type": None}
    par = {"box": box, "pp": oracle.pair_params(rc=rc), "ntypes": 1, "mass_by_type": np.array([1.0]),
           "dt": 0.005, "integrator": oracle.NVE}
    return st, par


def copy_state(s):
    return {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in s.items()}


def test_nve_energy_fluctuation_scales_with_dt_squared():
    st0, par = lj_state(rc=WCA, ncell=5)
    # equilibrate a little
    oracle.run(st0, par, 200)
    fl = []
    for dt, n in ((0.004, 250), (0.002, 500)):
        s = copy_state(st0)
        p = dict(par, dt=dt)
        h = oracle.run(s, p, n)
        e = h[1:, 0] + h[1:, 1] + h[1:, 2] + h[1:, 3]
        fl.append(np.sqrt(np.mean((e - e.mean()) ** 2)))
    ratio = fl[0] / fl[1]
    assert 4.0 * 0.7 < ratio < 4.0 * 1.3, ratio


def test_nve_conserves_energy_lj_rc25():
    # shifted energy with an unshifted force: crossings of rc cost a little
    # energy, far below the kinetic-energy fluctuation a wrong kick would give
    st, par = lj_state(rc=2.5, ncell=5)
    oracle.run(st, par, 200)
    h = oracle.run(st, par, 400)
    e = h[:, 0] + h[:, 3]
    n = st["pos"].shape[0]
    assert np.abs(e - e[0]).max() / n < 1e-3
    assert e.std() < 0.05 * h[:, 3].std()


def test_time_reversibility():
    st, par = lj_state(rc=2.5, ncell=4)
    x0 = st["pos"].copy()
    img0 = st["image"].copy()
    k = 60
    oracle.run(st, par, k)
    # convert the half-step velocity to the on-step one and reverse it
    F, _ = oracle.forces(st["pos"], par["box"], par["pp"])
    v_on = st["vel"] + 0.5 * par["dt"] * F
    st["vel"] = np.ascontiguousarray(-v_on)
    st["vel_half"] = 0
    oracle.run(st, par, k)
    L = par["box"][0]
    back = st["pos"] + st["image"] * L
    np.testing.assert_allclose(back, x0 + img0 * L, rtol=0, atol=1e-9)


def free_particles(n=2000, gamma=10.0, dt=0.01, T=1.0, seed=7):
    box = np.array([30.0, 30.0, 30.0])
    pos = inputs.random_positions(n, box, seed=seed)
    st = {"pos": pos, "vel": np.zeros((n, 3)), "image": np.zeros((n, 3), dtype=np.int32), "step": 0,
          "vel_half": 0, "type": None}
    par = {"box": box, "pp": oracle.pair_params(eps=0.0, rc=1.0), "ntypes": 1,
           "mass_by_type": np.array([2.0]), "dt": dt, "integrator": oracle.LANGEVIN,
           "temperature": T, "gamma": gamma, "seed": seed}
    return st, par


def test_langevin_free_particle_moments():
    gamma, dt, T, m = 10.0, 0.01, 1.3, 2.0
    st, par = free_particles(gamma=gamma, dt=dt, T=T)
    oracle.run(st, par, 300)            # relax from v = 0 (tau = 10 steps)
    n = st["pos"].shape[0]
    half2, onstep, ac = [], [], []
    prev = None
    for _ in range(400):
        h = oracle.run(st, par, 1)
        onstep.append(2.0 * h[0, 3] / (3 * n))      # m <v_n^2> per component
        v = st["vel"].copy()
        half2.append(m * np.mean(v * v))
        if prev is not None:
            ac.append(np.mean(v * prev) / np.mean(prev * prev))
        prev = v
    on = np.mean(onstep)
    hf = np.mean(half2)
    # on-step equipartition is exact for this scheme
    assert on == pytest.approx(T, rel=0.01)
    assert hf == pytest.approx(T / (1 - 0.5 * gamma * dt), rel=0.01)
    assert hf / on == pytest.approx(1.0 / (1 - 0.5 * gamma * dt), rel=0.01)
    assert np.mean(ac) == pytest.approx(1 - gamma * dt, abs=0.01)


def test_langevin_noise_is_keyed_by_step_and_tag():
    st, par = free_particles(n=50)
    s2 = copy_state(st)
    oracle.run(st, par, 5)
    oracle.run(s2, par, 2)
    oracle.run(s2, par, 3)
    assert np.array_equal(st["pos"], s2["pos"]) and np.array_equal(st["vel"], s2["vel"])
    s3 = copy_state(st)
    oracle.run(s3, dict(par, seed=par["seed"] + 1), 1)
    oracle.run(st, par, 1)
    assert not np.array_equal(st["vel"], s3["vel"])
