"""Pins of the oracle's tabulated pair and angle potentials and of the
AngularCosineSquared angle (section "Functionality": tabulated potentials;
section "New Features": AngularCosineSquared, TabulatedSubEnsAngular).

* A pair table sampled from the (pinned) Lennard-Jones closed form gives the
  LJ energy and force exactly at the grid points, the mean of two nodes half
  way between them, the rmin values below rmin, nothing from rc on, and on a
  fine grid the LJ forces of a whole fluid within the interpolation error.
* AngularCosineSquared: u = K cos^2(phi0) at a right angle, zero energy and
  force at phi0; its forces are minus the gradient of the total energy
  (central differences).
* An angle table sampled from that closed form gives its energy and forces
  exactly at the nodes.
* TabulatedSubEnsAngular: the combined table's energies and forces are the
  weighted sums of those of the separate tables.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2608_14911_amd import inputs

L = np.array([20.0, 20.0, 20.0])


def lj_table(n, rmin=0.8, rc=2.5):
    pp = oracle.pair_params(rc=rc)
    r = rmin + np.arange(n) * (rc - rmin) / (n - 1)
    uf = np.array([oracle.pair_eval(pp, x) for x in r[:-1]] + [(0.0, 0.0)])
    return r, uf[:, 0], uf[:, 1]


def pair_system(r):
    return np.array([[5.0, 5.0, 5.0], [5.0 + r, 5.0, 5.0]])


def test_pair_table_nodes_midpoints_and_ends():
    rc, rmin, n = 2.5, 0.8, 35
    r, u, f = lj_table(n, rmin, rc)
    tabs = oracle.tables(pair={(0, 0): (rmin, u, f)})
    pp = oracle.pair_params(rc=rc)
    for k in (0, 3, 17, n - 2):
        F, _, o = oracle.forces_ext(pair_system(r[k]), L, pp, tabs=tabs)
        ue, fe = oracle.pair_eval(pp, r[k])
        assert o["e_pair"] == pytest.approx(ue, rel=1e-12, abs=1e-14)
        assert -F[0, 0] == pytest.approx(fe, rel=1e-12, abs=1e-12)   # repulsive f > 0 pushes 0 to -x
    k = 11
    rm = 0.5 * (r[k] + r[k + 1])
    F, _, o = oracle.forces_ext(pair_system(rm), L, pp, tabs=tabs)
    assert o["e_pair"] == pytest.approx(0.5 * (u[k] + u[k + 1]), rel=1e-12)
    assert -F[0, 0] == pytest.approx(0.5 * (f[k] + f[k + 1]), rel=1e-12)
    F, _, o = oracle.forces_ext(pair_system(0.6), L, pp, tabs=tabs)        # below rmin
    assert o["e_pair"] == pytest.approx(u[0], rel=1e-12) and -F[0, 0] == pytest.approx(f[0], rel=1e-12)
    F, _, o = oracle.forces_ext(pair_system(rc), L, pp, tabs=tabs)         # at the cutoff
    assert o["e_pair"] == 0.0 and np.abs(F).max() == 0.0


def test_fine_pair_table_reproduces_lj_fluid():
    pos, box = inputs.fcc_lattice(4, 0.8442, jitter=0.15, seed=2)
    r, u, f = lj_table(200001, 0.7)
    tabs = oracle.tables(pair={(0, 0): (0.7, u, f)})
    pp = oracle.pair_params(rc=2.5)
    Ft, _, ot = oracle.forces_ext(pos, box, pp, tabs=tabs)
    Fl, ol = oracle.forces(pos, box, pp, use_cells=False)
    # linear interpolation error h^2/8 |f''|, h = 8.5e-6, |f''| < 1e7 on [0.7, 2.5]
    assert np.abs(Ft - Fl).max() < 1e-3 * 1e-2 * np.abs(Fl).max()
    assert ot["e_pair"] == pytest.approx(ol["e_pair"], rel=1e-8)


def chain(seed, n=12):
    g = np.random.default_rng(seed)
    steps = g.normal(size=(n - 1, 3))
    steps = steps / np.linalg.norm(steps, axis=1)[:, None] * 0.97
    pos = np.vstack([np.zeros(3), np.cumsum(steps, axis=0)]) + 10.0
    angles = np.array([[i, i + 1, i + 2] for i in range(n - 2)], dtype=np.int32)
    return pos, angles


def angle_energy(pos, angles, tabs, k_bend=0.0):
    pp = oracle.pair_params(eps=0.0, rc=1.0)
    _, _, o = oracle.forces_ext(pos, L, pp, angles=angles, k_bend=k_bend, tabs=tabs)
    return o["e_angle"]


def test_cosine_squared_closed_forms_and_gradient():
    K, phi0 = 3.0, math.radians(109.5)
    tabs = oracle.tables(angle_kind=oracle.ANGLE_COSINE_SQUARED, angle_K=K, angle_phi0=phi0)
    pp = oracle.pair_params(eps=0.0, rc=1.0)
    right = np.array([[11.0, 10.0, 10.0], [10.0, 10.0, 10.0], [10.0, 11.3, 10.0]])
    assert angle_energy(right, np.array([[0, 1, 2]], dtype=np.int32), tabs) == pytest.approx(
        K * math.cos(phi0) ** 2, rel=1e-14)
    at0 = np.array([[10.0 + math.cos(phi0), 10.0 + math.sin(phi0), 10.0], [10.0, 10.0, 10.0], [11.2, 10.0, 10.0]])
    F, _, o = oracle.forces_ext(at0, L, pp, angles=np.array([[0, 1, 2]], dtype=np.int32), tabs=tabs)
    assert abs(o["e_angle"]) < 1e-28 and np.abs(F).max() < 1e-13
    pos, ang = chain(3)
    F, _, _ = oracle.forces_ext(pos, L, pp, angles=ang, tabs=tabs)
    h = 1e-6
    for i in (0, 4, 11):
        for d in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[i, d] += h
            p2[i, d] -= h
            fd = -(angle_energy(p1, ang, tabs) - angle_energy(p2, ang, tabs)) / (2 * h)
            assert F[i, d] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    assert np.abs(F.sum(0)).max() < 1e-12


def cos2_table(K, phi0, n):
    phi = np.arange(n) * math.pi / (n - 1)
    u = K * (np.cos(phi) - math.cos(phi0)) ** 2
    g = -2.0 * K * (np.cos(phi) - math.cos(phi0)) * np.sin(phi)
    return phi, u, g


def test_angle_table_equals_cosine_squared_at_nodes():
    K, phi0, n = 2.0, math.radians(120.0), 181
    phi, u, g = cos2_table(K, phi0, n)
    tab = oracle.tables(angle_kind=oracle.ANGLE_TABULATED, angle_u=u, angle_g=g)
    ana = oracle.tables(angle_kind=oracle.ANGLE_COSINE_SQUARED, angle_K=K, angle_phi0=phi0)
    pp = oracle.pair_params(eps=0.0, rc=1.0)
    a = np.array([[0, 1, 2]], dtype=np.int32)
    for k in (20, 77, 150):
        p = np.array([[10.0 + 1.1 * math.cos(phi[k]), 10.0 + 1.1 * math.sin(phi[k]), 10.0], [10.0, 10.0, 10.0],
                      [10.9, 10.0, 10.0]])
        Ft, _, ot = oracle.forces_ext(p, L, pp, angles=a, tabs=tab)
        Fa, _, oa = oracle.forces_ext(p, L, pp, angles=a, tabs=ana)
        assert ot["e_angle"] == pytest.approx(oa["e_angle"], rel=1e-9, abs=1e-12)
        np.testing.assert_allclose(Ft, Fa, rtol=1e-7, atol=1e-9)


def test_subensemble_angle_tables_are_weighted_sums():
    n = 91
    _, u1, g1 = cos2_table(2.0, math.radians(100.0), n)
    _, u2, g2 = cos2_table(5.0, math.radians(150.0), n)
    w = np.array([0.3, 0.7])
    uc, gc = oracle.angle_tables_combine(np.stack([u1, u2]), np.stack([g1, g2]), w)
    pos, ang = chain(8)
    pp = oracle.pair_params(eps=0.0, rc=1.0)
    res = []
    for u, g in ((u1, g1), (u2, g2), (uc, gc)):
        F, _, o = oracle.forces_ext(pos, L, pp, angles=ang,
                                    tabs=oracle.tables(angle_kind=oracle.ANGLE_TABULATED, angle_u=u, angle_g=g))
        res.append((F, o["e_angle"]))
    assert res[2][1] == pytest.approx(w[0] * res[0][1] + w[1] * res[1][1], rel=1e-12)
    np.testing.assert_allclose(res[2][0], w[0] * res[0][0] + w[1] * res[1][0], rtol=1e-10, atol=1e-12)
