"""Parity at the full benchmark sizes, in the configuration bench.py times.

The 1,048,576-particle LJ fluid (FCC 64^3 with jitter, rc 2.5, skin 0.3,
NVE) and a 2,000,000-bead Kremer-Grest melt (2,000 chains x 1,000 beads at
density 0.85, WCA + FENE + bending 1.5, Langevin, skin 0.4) run with FP32
pair math and the library's automatic choices: cells of side rc+skin, with
the tile list build for the fluid and the per-particle build for the melt.  The FP64 oracle (linked cells, all host
threads) computes every particle's force at full size, so the check is
element by element, not sampled:

* every particle's force within 1e-5 of the oracle's, relative to the sum
  of its pair force magnitudes, and the norm of the difference within 1e-5
  of the force norm;
* pair, bond and angle energies within 1e-5 (relative), the virial within
  1e-5 of its condition, the sum of |r_ij . f_ij| over its terms, which the
  oracle returns beside W;
* neighbour rows of 4,096 sampled particles equal to the oracle's brute-
  force sets bit for bit, at the build positions;
* the same again after 40 steps with several list rebuilds.

The melt starts from chains laid on a simple cubic lattice
(``inputs.lattice_melt``), which has no overlapping beads and so needs no
push-off.  The benchmark's pushed-off random walks exercise the same
kernels.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import WCA, assert_forces_close, banner, oracle_pp, rel
from paper_2608_14911_amd import inputs, md
from paper_2608_14911_amd.system import from_workload

pytestmark = pytest.mark.gpu

TOL = 1e-5
NSAMPLE = 4096


def sampled_rows(s, sample, cap):
    """Neighbour tags of the sampled tags, sorted (rows come back by tag)."""
    cnt = torch.zeros(s.n, dtype=torch.int32, device=s.device)
    idx = torch.full((s.n, cap), -1, dtype=torch.int32, device=s.device)
    md.md_get_neighbors(s.h, cnt.data_ptr(), idx.data_ptr(), cap)
    sel = torch.as_tensor(sample, device=s.device)
    c = cnt[sel].cpu().numpy()
    m = idx[sel].cpu().numpy()
    del cnt, idx
    return [np.sort(m[k, :c[k]]) for k in range(len(sample))]


def virial_close(got, ref_obs, what=""):
    """|W - W_ref| <= TOL * sum |r_ij . f_ij|: the virial's terms have both
    signs, so its error is bounded relative to the sum of their magnitudes,
    which the oracle returns (virial_abs).  Prints both relative errors."""
    ref, scale = ref_obs["virial"], ref_obs["virial_abs"]
    d = abs(got - ref)
    print("virial %s: W %.6e, sum|r.f| %.6e, |dW|/sum|r.f| %.2e, |dW|/|W| %.2e" % (
        what, ref, scale, d / scale, d / max(abs(ref), 1e-300)), flush=True)
    return d <= TOL * scale


def check(s, w, pp, rv, cap, bonded, what, nsample=NSAMPLE):
    F = s.forces()
    o = s.observables()
    st = s.get_state()
    kw = {}
    if bonded:
        kw = dict(bonds=w["bonds"], angles=w["angles"], fene_K=w["fene_K"], fene_R0=w["fene_R0"],
                  k_bend=w["k_bend"])
    Fo, oo = oracle.forces(st["pos"], w["box"], pp, want_fscale=True, **kw)
    assert_forces_close(F, Fo, oo["fscale"], TOL, what)
    keys = ("e_pair", "e_bond", "e_angle") if bonded else ("e_pair",)
    for k in keys:
        assert rel(o[k], oo[k]) < TOL, (what, k, o[k], oo[k])
    assert virial_close(o["virial"], oo, what), (what, o["virial"], oo["virial"])
    # rows against brute force at the positions the list was built from
    g = np.random.default_rng(7)
    sample = np.sort(g.choice(s.n, size=nsample, replace=False))
    got = sampled_rows(s, sample, cap)
    ref = oracle.neighbors(st["pos_build"], w["box"], rv, query=sample, cap=cap)
    for k in range(nsample):
        assert np.array_equal(got[k], ref[k]), (what, int(sample[k]))
    return o


def test_lj_1m_full_size():
    w = inputs.workload_lj(ncell=64, seed=1001)
    banner("full-size LJ fluid n=%d" % w["pos"].shape[0])
    s = from_workload(w, precision="fp32")
    pp = oracle_pp(rc=w["rc"])
    rv = w["rc"] + w["skin"]
    check(s, w, pp, rv, 256, False, "LJ 1M start")
    s.step(40)
    o = check(s, w, pp, rv, 256, False, "LJ 1M after 40 steps")
    assert o["n_rebuilds"] >= 3 and o["status_flags"] == 0
    s.close()


def test_kg_2m_full_size():
    w = inputs.lattice_melt(2000, 1000, 0.85, jitter=0.05, seed=1002)
    w.update(inputs.kg_params(k_bend=1.5))
    w["vel"] = inputs.maxwell_boltzmann(w["pos"].shape[0], 1.0, seed=1002, zero_momentum=False, exact=False)
    w.update({"dt": 0.01, "skin": 0.4, "temperature": 1.0, "gamma": 0.5, "integrator": "langevin",
              "seed": 1002})
    banner("full-size KG melt n=%d" % w["pos"].shape[0])
    s = from_workload(w, precision="fp32")
    pp = oracle_pp(rc=WCA)
    rv = WCA + w["skin"]
    check(s, w, pp, rv, 128, True, "KG 2M start")
    s.step(40)
    o = check(s, w, pp, rv, 128, True, "KG 2M after 40 steps")
    assert o["n_rebuilds"] >= 2 and o["status_flags"] == 0
    s.close()


def lattice_replica(r):
    """A melt replica of the sampler laid on a lattice instead of pushed off:
    same bead count, chain length and density."""
    n = r["pos"].shape[0]
    lc = r["chain_len"]
    w = inputs.lattice_melt(n // lc, lc, r["density"], jitter=0.05, seed=r["seed"])
    out = dict(r)
    out.update(pos=w["pos"], box=w["box"], bonds=w["bonds"], angles=w["angles"])
    return out


def test_batch_256_full_size():
    """The benchmark's 256 replicas (4.7M particles; melts on lattices) in one
    batch with the automatic builds: after 20 steps, the observables of every
    member (evaluated at its current positions) match the oracle's energies
    and virial at those positions within 1e-5."""
    from paper_2608_14911_amd.system import Batch
    reps = inputs.batch_replicas(256, seed=1003)
    reps = [lattice_replica(r) if r["kind"] == "kg" else r for r in reps]
    banner("full-size batch: %d replicas, %d particles" % (len(reps), sum(r["pos"].shape[0] for r in reps)))
    b = Batch(reps)
    b.step(20)
    sample = range(len(reps))
    ob = b.observables()
    for k in sample:
        r, st = reps[k], b.get_state(k)
        assert st["step"] == 20 and ob[k]["step"] == 20 and ob[k]["status_flags"] == 0, k
        row = r["pair"][(0, 0)]
        pp = oracle_pp(eps=row[0], sigma=row[1], rc=row[2], shift=row[3], caprad=row[4])
        kw = {}
        if r["kind"] == "kg":
            kw = dict(bonds=r["bonds"], angles=r["angles"], k_bend=r["k_bend"])
        _, oo = oracle.forces(st["pos"], r["box"], pp, want_fscale=True, **kw)
        keys = ("e_pair", "e_bond", "e_angle") if r["kind"] == "kg" else ("e_pair",)
        for key in keys:
            assert rel(ob[k][key], oo[key]) < TOL, (k, r["kind"], key, ob[k][key], oo[key])
        assert virial_close(ob[k]["virial"], oo, "member %d" % k), (k, ob[k]["virial"], oo["virial"])
    b.close()


@pytest.mark.parametrize("prec,tol", [("bf16", 3e-2), ("fp32", 1e-5)])
def test_surrogate_1m_full_size(prec, tol):
    """The learned surrogate on a 1,000,000-bead melt (the trained weights the
    benchmark times, list radius 2.5 + skin): 256 sampled beads' forces
    against the FP64 surrogate oracle, and over all beads the total force,
    which vanishes for pair-decomposed forces (Newton's third law).  A bead's surrogate force depends on
    the beads within 2 r_d of it only, so the oracle evaluates, per sampled
    bead, the beads within 2 r_d + 0.5 of it (periodic minimum image in the
    full box) and the bead's force there is exact.  FENE and bending come
    from the plain oracle on the whole melt."""
    import os
    from oracle import surrogate as S
    w = inputs.lattice_melt(1000, 1000, 0.85, jitter=0.05, seed=1014)
    w.update(inputs.kg_params(k_bend=1.5))
    w["vel"] = inputs.maxwell_boltzmann(w["pos"].shape[0], 1.0, seed=1014, zero_momentum=False, exact=False)
    w.update({"dt": 0.01, "skin": 0.4, "temperature": 1.0, "gamma": 0.5, "integrator": "langevin",
              "seed": 1014})
    banner("full-size surrogate %s n=%d" % (prec, w["pos"].shape[0]))
    s = from_workload(w, precision="fp32", list_cutoff=2.5, surrogate=True)
    wd = np.load(os.path.join(os.path.dirname(inputs.__file__), "data", "surrogate_kg.npz"))
    th = wd["theta_" + prec]
    s.sur_set(th, wd["g_mean"], wd["g_istd"], prec)
    s.set_pair_mode("surrogate")
    Fg = s.forces()
    pos, box = s.get_state()["pos"], w["box"]
    Fb, ob = oracle.forces(pos, box, oracle_pp(eps=0.0, rc=WCA), bonds=w["bonds"], angles=w["angles"],
                           k_bend=1.5, want_fscale=True)
    g = np.random.default_rng(11)
    sample = g.choice(pos.shape[0], size=256, replace=False)
    th64 = th.astype(np.float64)
    m64, istd64 = wd["g_mean"].astype(np.float64), wd["g_istd"].astype(np.float64)
    worst = 0.0
    for i in sample:
        d = pos - pos[i]
        d -= box * np.round(d / box)
        near = np.nonzero((d * d).sum(1) < (2 * S.RD + 0.5) ** 2)[0]
        k = int(np.nonzero(near == i)[0][0])
        _, _, Fs, _, _, fs = S.energy_forces(th64, m64, istd64, pos[near], box, want_fscale=True)
        ref = Fs[k] + Fb[i]
        scale = fs[k] + ob["fscale"][i]
        err = np.linalg.norm(Fg[i] - ref)
        worst = max(worst, err / scale)
        assert err <= tol * scale + 1e-12, (prec, int(i), err, scale)
    print("%s: worst per-bead ratio %.3g" % (prec, worst))
    # every bead: the forces sum to zero up to FP32 rounding of the per-pair
    # terms (each pair's term is summed by both beads in different orders)
    tot = np.abs(Fg.sum(0)).max() / np.abs(Fg).sum()
    print("%s: |sum F| / sum |F| = %.3g" % (prec, tot))
    assert tot < 1e-6
    s.close()


def test_lj_16m_large():
    """A 16,384,000-particle LJ fluid (FCC 160^3, 16x the benchmark): list
    offsets and cell indices far beyond the benchmark's; every force against
    the oracle and sampled rows bit-exact, before and after a few steps."""
    w = inputs.workload_lj(ncell=160, seed=1007)
    banner("large LJ fluid n=%d" % w["pos"].shape[0])
    s = from_workload(w, precision="fp32")
    pp = oracle_pp(rc=w["rc"])
    rv = w["rc"] + w["skin"]
    check(s, w, pp, rv, 128, False, "LJ 16M start", nsample=512)
    s.step(12)
    o = check(s, w, pp, rv, 128, False, "LJ 16M after 12 steps", nsample=512)
    assert o["n_rebuilds"] >= 2 and o["status_flags"] == 0
    s.close()
