"""Pins of the oracle's AdResS force interpolation (the method the paper
names as its differentiator: sections "Statement of need" and
"Functionality"; it gives no formula and no model pair).  Reading: single-
site molecules, F_ij = w_i w_j F^AT_ij + (1 - w_i w_j) F^CG_ij with the slab
weight w(x) = 1 / cos^2 switch / 0 around x0 along x.  Pinned by:

* w: 1 in the atomistic zone, 0 in the coarse-grained zone, 1/2 half way
  through the hybrid zone, continuous at both zone edges, periodic in x;
* limits: an atomistic zone covering the box gives the plain atomistic
  forces, no atomistic zone gives the coarse-grained forces, and equal AT and
  CG potentials give that potential whatever the weights;
* a pair of particles half way through the hybrid zone feels
  F = F^AT/4 + 3 F^CG/4 (w = 1/2 each);
* Newton's third law: the net force vanishes.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2608_14911_amd import inputs

WCA = 2.0 ** (1.0 / 6.0)


def soft_cg(n=400, rmin=0.0, rc=1.5, a=15.0):
    r = rmin + np.arange(n) * (rc - rmin) / (n - 1)
    return rmin, rc, 0.5 * a * (1.0 - r / rc) ** 2, a * (1.0 - r / rc) / rc


def test_weight_zones_and_continuity():
    L, x0, dat, dhy = 20.0, 6.0, 2.0, 3.0
    w = lambda x: oracle.adress_weight(x, L, x0, dat, dhy)
    assert w(6.0) == 1.0 and w(7.99) == 1.0 and w(4.01) == 1.0
    assert w(x0 + dat + 0.5 * dhy) == pytest.approx(0.5, abs=1e-15)
    assert w(x0 - dat - 0.5 * dhy) == pytest.approx(0.5, abs=1e-15)
    assert w(x0 + dat + dhy + 1e-9) == 0.0 and w(16.0) == 0.0
    e = 1e-9
    assert abs(w(x0 + dat + e) - 1.0) < 1e-12 and abs(w(x0 + dat + dhy - e)) < 1e-12
    # periodic: x0 near the box edge
    assert oracle.adress_weight(19.5, L, 0.5, 2.0, 3.0) == 1.0
    assert oracle.adress_weight(17.0, L, 0.5, 2.0, 3.0) == pytest.approx(0.5, abs=1e-15)   # d = 3.5


def test_limits_and_newton():
    pos, box = inputs.fcc_lattice(4, 0.8, jitter=0.2, seed=4)
    pp = oracle.pair_params(rc=WCA)
    cg = {(0, 0): soft_cg()}
    Fat, _, oat = oracle.forces_ext(pos, box, pp)
    Fall, _, oall = oracle.forces_ext(pos, box, pp, tabs=oracle.tables(adress=(0.0, box[0], 1.0), cg=cg))
    np.testing.assert_allclose(Fall, Fat, rtol=1e-13, atol=1e-12)
    assert oall["e_pair"] == pytest.approx(oat["e_pair"], rel=1e-13)
    Fcg, _, ocg = oracle.forces_ext(pos, box, pp, tabs=oracle.tables(adress=(0.0, 0.0, 1e-9), cg=cg))
    # the coarse-grained forces alone: the soft potential as a pair table with the AT force switched off
    rmin, rc, u, f = soft_cg()
    Fref, _, oref = oracle.forces_ext(pos, box, oracle.pair_params(eps=1.0, rc=rc),
                                      tabs=oracle.tables(pair={(0, 0): (rmin, u, f)}))
    np.testing.assert_allclose(Fcg, Fref, rtol=1e-12, atol=1e-11)
    assert ocg["e_pair"] == pytest.approx(oref["e_pair"], rel=1e-12)
    # a hybrid zone across the box: the net force still vanishes
    Fh, _, _ = oracle.forces_ext(pos, box, pp, tabs=oracle.tables(adress=(box[0] / 2, 1.0, 2.5), cg=cg))
    assert np.abs(Fh.sum(0)).max() < 1e-12 * np.abs(Fh).sum()
    assert np.abs(Fh - Fat).max() > 1.0 and np.abs(Fh - Fcg).max() > 1.0
    # equal AT and CG potentials: the weights do not matter
    ru = np.linspace(0.7, WCA, 2001)
    uf = np.array([oracle.pair_eval(pp, x) for x in ru[:-1]] + [(0.0, 0.0)])
    same = {(0, 0): (0.7, WCA, uf[:, 0], uf[:, 1])}
    tab_at = oracle.tables(pair={(0, 0): (0.7, uf[:, 0], uf[:, 1])}, adress=(box[0] / 2, 1.0, 2.5), cg=same)
    tab_plain = oracle.tables(pair={(0, 0): (0.7, uf[:, 0], uf[:, 1])})
    Fs, _, _ = oracle.forces_ext(pos, box, pp, tabs=tab_at)
    Fp, _, _ = oracle.forces_ext(pos, box, pp, tabs=tab_plain)
    np.testing.assert_allclose(Fs, Fp, rtol=1e-12, atol=1e-10)


def test_pair_half_way_through_the_hybrid_zone():
    L, x0, dat, dhy = 20.0, 10.0, 2.0, 4.0
    xm = x0 + dat + 0.5 * dhy                      # w = 1/2
    box = np.array([L, L, L])
    pos = np.array([[xm, 5.0, 5.0], [xm, 5.0 + 1.05, 5.0]])   # separated along y: same x, same weight
    pp = oracle.pair_params(rc=2.5)
    cg = {(0, 0): soft_cg(rc=2.0)}
    F, _, o = oracle.forces_ext(pos, box, pp, tabs=oracle.tables(adress=(x0, dat, dhy), cg=cg))
    ua, fa = oracle.pair_eval(pp, 1.05)
    rmin, rc, u, f = soft_cg(rc=2.0)
    ucg = 0.5 * 15.0 * (1 - 1.05 / rc) ** 2       # the table is linear in r on its grid: compare through it
    Fc, _, oc = oracle.forces_ext(pos, box, oracle.pair_params(rc=rc), tabs=oracle.tables(pair={(0, 0): (rmin, u, f)}))
    assert o["e_pair"] == pytest.approx(0.25 * ua + 0.75 * oc["e_pair"], rel=1e-12)
    assert -F[0, 1] == pytest.approx(0.25 * fa + 0.75 * (-Fc[0, 1]), rel=1e-12)
    assert oc["e_pair"] == pytest.approx(ucg, rel=1e-4)
