"""GPU parity of the tabulated pair and angle potentials, AngularCosineSquared
and TabulatedSubEnsAngular against the FP64 oracle (same tables), through
the C ABI.  Tables are stored in FP32 on the device; forces must agree
within 1e-5 per particle relative to the sum of the particle's force-term
magnitudes, energies within 1e-5.
"""
import math

import numpy as np
import pytest

import oracle
from gpu_helpers import WCA, assert_forces_close, banner, oracle_pp
from paper_2608_14911_amd import inputs, md
from paper_2608_14911_amd.system import System, lj_pair

pytestmark = pytest.mark.gpu

TOL = 1e-5


def lj_table(n, rmin, rc, eps=1.0, sigma=1.0):
    pp = oracle.pair_params(eps=eps, sigma=sigma, rc=rc)
    r = rmin + np.arange(n) * (rc - rmin) / (n - 1)
    uf = np.array([oracle.pair_eval(pp, x) for x in r[:-1]] + [(0.0, 0.0)])
    return uf[:, 0], uf[:, 1]


def test_tabulated_pair_lj_fluid_and_mixture():
    banner("tabulated pair potentials: LJ fluid, three-type mixture")
    pos, box = inputs.fcc_lattice(6, 0.8442, jitter=0.15, seed=7)
    u, f = lj_table(1500, 0.8, 2.5)
    s = System(pos, box, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3, table_points=2048)
    s.set_pair_table(0, 0, u, f, 0.8)
    Fg = s.forces()
    o = s.observables()
    tabs = oracle.tables(pair={(0, 0): (0.8, u, f)})
    Fo, _, oo = oracle.forces_ext(pos, box, oracle_pp(rc=2.5), tabs=tabs, want_fscale=True)
    assert_forces_close(Fg, Fo, oo["fscale"], TOL, "tabulated LJ")
    assert abs(o["e_pair"] - oo["e_pair"]) <= TOL * abs(oo["e_pair"])
    assert abs(o["virial"] - oo["virial"]) <= TOL * oo["virial_abs"]
    # the table sampled from LJ reproduces the plain LJ path closely
    s2 = System(pos, box, pair={(0, 0): lj_pair(rc=2.5)}, skin=0.3)
    assert np.abs(s2.forces() - Fg).max() < 2e-3 * np.abs(Fg).max()
    s2.close()
    s.close()
    # mixture: type pair (0, 1) tabulated (a soft repulsion), the others LJ
    g = np.random.default_rng(3)
    types = g.integers(0, 3, size=pos.shape[0]).astype(np.int32)
    rows = {(0, 0): (1.0, 1.0, 2.5, math.nan, 0.0), (0, 1): (1.0, 1.0, 2.0, math.nan, 0.0),
            (1, 1): (0.8, 1.1, 2.4, math.nan, 0.0), (0, 2): (1.0, 0.9, WCA * 0.9, math.nan, 0.0),
            (1, 2): (0.5, 1.0, 2.2, math.nan, 0.0), (2, 2): (1.2, 1.0, 2.5, math.nan, 0.0)}
    rs = np.linspace(0.5, 2.0, 300)
    us = 20.0 * (1.0 - rs / 2.0) ** 2
    fs = 20.0 * (1.0 - rs / 2.0)         # -du/dr
    s = System(pos, box, types=types, n_types=3, pair=rows, masses=(1.0, 2.0, 0.5), skin=0.3, table_points=512)
    s.set_pair_table(1, 0, us, fs, 0.5)
    Fg = s.forces()
    pp = oracle.pair_table(3, {k: oracle.pair_params(*v) for k, v in rows.items()})
    tabs = oracle.tables(ntypes=3, pair={(0, 1): (0.5, us, fs)})
    Fo, _, oo = oracle.forces_ext(pos, box, pp, ntypes=3, type=types, tabs=tabs, want_fscale=True)
    assert_forces_close(Fg, Fo, oo["fscale"], TOL, "tabulated mixture")
    assert abs(s.observables()["e_pair"] - oo["e_pair"]) <= TOL * abs(oo["e_pair"])
    s.close()


def cos2_table(K, phi0, n):
    phi = np.arange(n) * math.pi / (n - 1)
    u = K * (np.cos(phi) - math.cos(phi0)) ** 2
    g = -2.0 * K * (np.cos(phi) - math.cos(phi0)) * np.sin(phi)
    return u, g


@pytest.mark.parametrize("kind", ["cosine_squared", "tabulated", "subens"])
def test_angle_kinds_on_a_melt(kind):
    banner("angle kind %s on a melt" % kind)
    w = inputs.lattice_melt(40, 25, 0.85, jitter=0.12, seed=6)
    K, phi0 = 4.0, math.radians(115.0)
    kw = dict(bonds=w["bonds"], angles=w["angles"])
    if kind == "cosine_squared":
        s = System(w["pos"], w["box"], pair={(0, 0): lj_pair(rc=WCA)}, skin=0.4, dt=0.005,
                   angle_kind=md.MD_ANGLE_COSINE_SQUARED, angle_K=K, angle_phi0=phi0, **kw)
        tabs = oracle.tables(angle_kind=oracle.ANGLE_COSINE_SQUARED, angle_K=K, angle_phi0=phi0)
    else:
        u1, g1 = cos2_table(K, phi0, 721)
        s = System(w["pos"], w["box"], pair={(0, 0): lj_pair(rc=WCA)}, skin=0.4, dt=0.005,
                   angle_kind=md.MD_ANGLE_TABULATED, table_points=1024, **kw)
        if kind == "tabulated":
            s.set_angle_table(u1, g1)
            tabs = oracle.tables(angle_kind=oracle.ANGLE_TABULATED, angle_u=u1, angle_g=g1)
        else:
            u2, g2 = cos2_table(1.5, math.radians(160.0), 721)
            wts = np.array([0.25, 0.75])
            s.set_angle_subens(np.stack([u1, u2]), np.stack([g1, g2]), wts)
            uc, gc = oracle.angle_tables_combine(np.stack([u1, u2]), np.stack([g1, g2]), wts)
            tabs = oracle.tables(angle_kind=oracle.ANGLE_TABULATED, angle_u=uc, angle_g=gc)
    Fg = s.forces()
    o = s.observables()
    Fo, _, oo = oracle.forces_ext(w["pos"], w["box"], oracle_pp(rc=WCA), tabs=tabs, want_fscale=True, **kw)
    assert_forces_close(Fg, Fo, oo["fscale"], TOL, "angle kind " + kind)
    for k in ("e_pair", "e_bond", "e_angle"):
        assert abs(o[k] - oo[k]) <= TOL * abs(oo[k]), (k, o[k], oo[k])
    assert abs(o["virial"] - oo["virial"]) <= TOL * oo["virial_abs"]
    # one step of Langevin dynamics through the generic kernel
    s.set_params(integrator="langevin", gamma=1.0, temperature=1.0, seed=5)
    s.step(1)
    g = s.get_state()
    n = w["pos"].shape[0]
    st = {"pos": w["pos"].copy(), "vel": np.zeros((n, 3)), "image": np.zeros((n, 3), dtype=np.int32), "step": 0,
          "vel_half": 0, "type": None}
    par = {"box": w["box"], "pp": oracle_pp(rc=WCA), "ntypes": 1, "mass_by_type": np.array([1.0]), "dt": 0.005,
           "integrator": oracle.LANGEVIN, "temperature": 1.0, "gamma": 1.0, "seed": 5, "tabs": tabs, **kw}
    oracle.run_ext(st, par, 1)
    dx = np.abs(g["pos"] - st["pos"])
    dx = np.minimum(dx, w["box"] - dx).max(1)
    assert np.all(dx <= TOL * 0.005 ** 2 / 2 * oo["fscale"] + 1e-12)
    s.close()


def test_tabulated_angle_needs_its_table():
    w = inputs.lattice_melt(4, 25, 0.85, seed=6)
    s = System(w["pos"], w["box"], pair={(0, 0): lj_pair(rc=WCA)}, skin=0.4, bonds=w["bonds"], angles=w["angles"],
               angle_kind=md.MD_ANGLE_TABULATED, table_points=64)
    with pytest.raises(md.MDError) as e:
        s.step(1)
    assert e.value.code == md.MD_ERR_STATE
    s.close()
