"""Pins of the oracle's interaction functions against closed-form facts.

LennardJones / LennardJonesCapped with shift='auto' and the bonded terms are
the interactions of the paper's example and feature list (sections "Example
usage" and "Functionality"); the facts checked here follow from the
potentials' definitions (minimum depth and position, zero crossings, harmonic
limit, continuity at the cutoff) and from F = -dU/dr by finite differences,
not from re-evaluating the oracle's own expressions.
"""
import math

import numpy as np
import pytest

import oracle

WCA = 2.0 ** (1.0 / 6.0)


def lj(eps=1.0, sigma=1.0, rc=2.5, shift=float("nan"), caprad=0.0):
    return oracle.pair_params(eps, sigma, rc, shift, caprad)


@pytest.mark.parametrize("eps,sigma", [(1.0, 1.0), (0.7, 1.3), (2.5, 0.8)])
def test_lj_minimum_depth_and_position(eps, sigma):
    # unshifted LJ has its minimum -eps at 2^(1/6) sigma, where the force vanishes
    p = lj(eps, sigma, rc=3.0 * sigma, shift=0.0)
    u, f = oracle.pair_eval(p, WCA * sigma)
    assert u == pytest.approx(-eps, rel=1e-14)
    assert abs(f) < 1e-12 * eps / sigma
    # zero crossing at r = sigma, repulsive inside
    u1, f1 = oracle.pair_eval(p, sigma)
    assert abs(u1) < 1e-14 * eps
    assert f1 > 0
    # f(sigma) = 24 eps / sigma: the slope of 4eps[(s/r)^12-(s/r)^6] at r = sigma
    assert f1 == pytest.approx(24.0 * eps / sigma, rel=1e-14)


def test_lj_shift_auto_makes_energy_vanish_at_cutoff():
    for rc in (2.5, WCA, 1.12246):
        p = lj(rc=rc)
        u, _ = oracle.pair_eval(p, rc * (1 - 1e-12))
        assert abs(u) < 1e-9
        # outside the cutoff: nothing
        assert oracle.pair_eval(p, rc) == (0.0, 0.0)
        assert oracle.pair_eval(p, rc * 1.0000001) == (0.0, 0.0)


def test_wca_is_lj_plus_eps_and_continuous():
    p = lj(rc=WCA)
    q = lj(rc=3.0, shift=0.0)
    for r in (0.9, 1.0, 1.05, 1.1):
        u, f = oracle.pair_eval(p, r)
        u0, f0 = oracle.pair_eval(q, r)
        assert u == pytest.approx(u0 + 1.0, rel=1e-13, abs=1e-13)
        assert f == pytest.approx(f0, rel=1e-13)
    u, f = oracle.pair_eval(p, WCA * (1 - 1e-9))
    assert abs(u) < 1e-12 and abs(f) < 1e-6


@pytest.mark.parametrize("params", [dict(), dict(rc=WCA), dict(eps=0.5, sigma=1.2, rc=3.0)])
def test_lj_force_is_minus_energy_derivative(params):
    p = lj(**params)
    rc = p[2]
    for r in np.linspace(0.85, rc * 0.98, 17):
        h = 1e-6
        up, _ = oracle.pair_eval(p, r + h)
        um, _ = oracle.pair_eval(p, r - h)
        _, f = oracle.pair_eval(p, r)
        fd = -(up - um) / (2 * h)
        assert f == pytest.approx(fd, rel=1e-7, abs=1e-8)


def test_capped_lj_freezes_energy_and_force_below_caprad():
    cap = 0.8
    p = lj(rc=WCA, caprad=cap)
    q = lj(rc=WCA)
    uc, fc = oracle.pair_eval(q, cap)
    for r in (0.05, 0.3, 0.5, 0.79):
        u, f = oracle.pair_eval(p, r)
        assert u == pytest.approx(uc, rel=1e-14)
        assert f == pytest.approx(fc, rel=1e-12)
    for r in (0.81, 0.95, 1.1):
        assert oracle.pair_eval(p, r) == pytest.approx(oracle.pair_eval(q, r), rel=1e-14)


def test_fene_properties():
    K, R0 = 30.0, 1.5
    # u(0) = 0, harmonic limit u ~ K r^2 / 2, attractive force ~ -K r
    u, f = oracle.fene_eval(K, R0, 1e-4)
    assert u == pytest.approx(0.5 * K * 1e-8, rel=1e-6)
    assert f == pytest.approx(-K * 1e-4, rel=1e-6)
    # diverges at R0
    u, f = oracle.fene_eval(K, R0, R0 * (1 - 1e-9))
    assert u > 100 and f < -1e6
    # F = -dU/dr
    for r in np.linspace(0.2, 1.45, 11):
        h = 1e-6
        fd = -(oracle.fene_eval(K, R0, r + h)[0] - oracle.fene_eval(K, R0, r - h)[0]) / (2 * h)
        assert oracle.fene_eval(K, R0, r)[1] == pytest.approx(fd, rel=1e-7)
    # half the bond length at which the log argument is 1/2: u = K R0^2 ln(2) / 2
    u, _ = oracle.fene_eval(K, R0, R0 / math.sqrt(2.0))
    assert u == pytest.approx(0.5 * K * R0 * R0 * math.log(2.0), rel=1e-14)


def test_fene_broken_bond_raises():
    with pytest.raises(oracle.OracleError) as e:
        oracle.fene_eval(30.0, 1.5, 1.5)
    assert e.value.code == oracle.ERR_BOND_BROKEN


def _bend_energy(k, ra, rb, rc):
    return oracle.bend_eval(k, ra, rb, rc)[0]


def test_bending_closed_forms():
    k = 1.5
    a, b = np.array([0.0, 0, 0]), np.array([0.97, 0, 0])
    # straight chain: theta = 0, zero energy and force
    u, Fa, Fb, Fc = oracle.bend_eval(k, a, b, np.array([1.94, 0, 0]))
    assert abs(u) < 1e-15 and np.abs(np.r_[Fa, Fb, Fc]).max() < 1e-14
    # right angle: cos = 0 -> u = k
    u, *_ = oracle.bend_eval(k, a, b, np.array([0.97, 1.1, 0]))
    assert u == pytest.approx(k, rel=1e-14)
    # full fold-back: cos = -1 -> u = 2k
    u, *_ = oracle.bend_eval(k, a, b, np.array([0.1, 0, 0]))
    assert u == pytest.approx(2 * k, rel=1e-14)


def test_bending_forces_are_gradient_and_balanced():
    g = np.random.default_rng(3)
    k = 1.5
    for _ in range(20):
        r = g.normal(size=(3, 3))
        u, Fa, Fb, Fc = oracle.bend_eval(k, r[0], r[1], r[2])
        F = np.stack([Fa, Fb, Fc])
        np.testing.assert_allclose(F.sum(axis=0), 0, atol=1e-12)
        # zero torque about the origin (rotational invariance)
        np.testing.assert_allclose(np.cross(r, F).sum(axis=0), 0, atol=1e-12)
        h = 1e-6
        for p in range(3):
            for d in range(3):
                rp = r.copy(); rp[p, d] += h
                rm = r.copy(); rm[p, d] -= h
                fd = -(_bend_energy(k, *rp) - _bend_energy(k, *rm)) / (2 * h)
                assert F[p, d] == pytest.approx(fd, rel=1e-6, abs=1e-7)
