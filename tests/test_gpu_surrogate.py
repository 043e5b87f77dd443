"""GPU parity of the learned surrogate against the FP64 oracle (through the C ABI).

Descriptors, network outputs, forces, energy, virial, the force-matching
loss and its parameter gradient, and one Adam update are compared with
``oracle.surrogate`` on the same inputs: FP32 network within 1e-5 (normwise;
forces also per particle against sum_j |f_ij|), the gradient within 1e-4
normwise (FP32 sums over ~10^5 per-pair terms), BF16 network within 3e-2.
Property checks at any size: Newton's third law, and an NVE run whose
total energy is conserved (the forces are the gradient of the energy).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import surrogate as S
from gpu_helpers import WCA, banner, rel
from kg_fixture import kg1k_state
from paper_2608_14911_amd import inputs
from paper_2608_14911_amd.system import System, lj_pair

pytestmark = pytest.mark.gpu

SKIN = 0.3


def theta32(seed=1004, scale=1.0):
    th = inputs.mlp_init(seed) * scale
    g = np.random.default_rng(seed)
    th[S.O_B1:S.O_W2] = g.uniform(-0.3, 0.3, 64)
    th[S.O_B2:S.O_W3] = g.uniform(-0.3, 0.3, 64)
    th[S.O_B3] = 0.1
    return th.astype(np.float32).astype(np.float64)


def norm32(pos, box):
    G = S.descriptors(pos, box)
    m = G.mean(0).astype(np.float32)
    istd = (1.0 / (G.std(0) + 1e-3)).astype(np.float32)
    return m.astype(np.float64), istd.astype(np.float64)


def melt(k_bend=0.0):
    w = kg1k_state(k_bend)
    return w, w["pos"], w["box"]


def sur_system(w, pos, precision="fp32", bonded=True, **kw):
    s = System(pos, w["box"], pair={(0, 0): lj_pair(rc=WCA)}, bonds=w["bonds"] if bonded else None,
               angles=w["angles"] if bonded and w.get("k_bend", 0) else None, k_bend=w.get("k_bend", 0.0),
               skin=SKIN, list_cutoff=S.RD, surrogate=True, **kw)
    return s


def test_descriptors_match_oracle():
    w, pos, box = melt()
    banner("surrogate descriptors KG 1k")
    s = sur_system(w, pos)
    G = s.descriptors().cpu().numpy().astype(np.float64)
    Go = S.descriptors(pos, box)
    err = np.linalg.norm(G - Go) / np.linalg.norm(Go)
    print("descriptor rel err %.3g" % err)
    assert err < 1e-5
    assert np.abs(G - Go).max() < 1e-5 * np.abs(Go).max()
    s.close()


def test_standardisation_matches_oracle():
    """md_sur_desc_stats against the oracle's constants over three frames;
    the bounds follow from the descriptors' own tolerance (1e-5 of max |G|
    per entry): |dm| <= that, and |d var| <= 4 max|G| of it, which moves
    istd = (var + 1e-6)^(-1/2) by at most half its relative size."""
    w, pos, box = melt()
    banner("surrogate standardisation KG 1k, 3 frames")
    g = np.random.default_rng(11)
    frames = [pos] + [np.mod(pos + g.normal(scale=0.05, size=pos.shape), box) for _ in range(2)]
    s = sur_system(w, pos)
    m, istd = s.desc_stats(np.stack(frames))
    m, istd = m.cpu().numpy().astype(np.float64), istd.cpu().numpy().astype(np.float64)
    mo, io = S.standardisation(frames, box)
    Gmax = max(np.abs(S.descriptors(f, box)).max() for f in frames)
    dG = 1e-5 * Gmax
    var_o = 1.0 / io ** 2 - 1e-6
    em = np.abs(m - mo).max()
    ei = (np.abs(istd - io) / io / (0.5 * 4.0 * Gmax * dG / (var_o + 1e-6) + 1e-6)).max()
    print("standardisation: max |dm| %.3g (bound %.3g), istd error / bound %.3g" % (em, dG, ei))
    assert em <= dG
    assert ei <= 1.0
    # the state is the last frame's
    st = s.get_state()
    d = st["pos"] - frames[-1]
    assert np.abs(d - box * np.round(d / box)).max() < 1e-12
    with pytest.raises(Exception):
        s.desc_stats(np.zeros((0, pos.shape[0], 3)))
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-2)])
def test_mlp_eval_matches_oracle(prec, tol):
    w, pos, box = melt()
    banner("surrogate MLP %s" % prec)
    s = sur_system(w, pos)
    m, istd = norm32(pos, box)
    th = theta32()
    s.sur_set(th, m, istd, prec)
    g = np.random.default_rng(7)
    # 1,000 rows: 15 full tiles of 64 and a ragged tail of 40
    G = (S.descriptors(pos, box) + g.normal(scale=0.1, size=(1000, 32))).astype(np.float32).astype(np.float64)
    e, a = s.mlp_eval(G)
    e, a = e.cpu().numpy(), a.cpu().numpy()
    eo, gx = S.mlp(th, (G - m) * istd)
    ao = gx * istd
    ee = np.linalg.norm(e - eo) / np.linalg.norm(eo)
    ea = np.linalg.norm(a - ao) / np.linalg.norm(ao)
    print("%s: energy rel err %.3g, dE/dG rel err %.3g" % (prec, ee, ea))
    assert ee < tol and ea < tol
    # round-trip of the master weights
    assert np.array_equal(s.sur_get(), th.astype(np.float32))
    s.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16", 3e-2)])
def test_surrogate_forces_energy_virial(prec, tol):
    w, pos, box = melt()
    banner("surrogate forces %s KG 1k with FENE" % prec)
    s = sur_system(w, pos)
    m, istd = norm32(pos, box)
    th = theta32()
    s.sur_set(th, m, istd, prec)
    s.set_pair_mode("surrogate")
    Fg = s.forces()
    o = s.observables()
    E, Ei, Fs, a, W, fs = S.energy_forces(th, m, istd, pos, box, want_fscale=True)
    Fb, ob = oracle.forces(pos, box, oracle.pair_params(eps=0.0, rc=WCA), bonds=w["bonds"], want_fscale=True)
    Fo = Fs + Fb
    scale = fs + ob["fscale"]
    d = np.linalg.norm(Fg - Fo, axis=1)
    nerr = np.linalg.norm(Fg - Fo) / np.linalg.norm(Fo)
    print("%s: force rel err %.3g, worst per-particle ratio %.3g, E rel %.3g, W rel %.3g" % (
        prec, nerr, (d / (scale + 1e-300)).max(), rel(o["e_pair"], E), rel(o["virial"], W + ob["virial"])))
    assert nerr < tol
    assert (d <= tol * scale + 1e-12).all()
    assert rel(o["e_pair"], E) < tol
    assert rel(o["virial"], W + ob["virial"]) < tol * 10
    assert rel(o["e_bond"], ob["e_bond"]) < 1e-5
    # Newton's third law (FP32 sums)
    assert np.abs(Fg.sum(0)).max() < 1e-5 * np.abs(Fg).sum(1).max() * math.sqrt(len(Fg))
    # switching back to the plain pair table gives the plain forces
    s.set_pair_mode("plain")
    Fp = s.forces()
    Fw = oracle.forces(pos, box, oracle.pair_params(rc=WCA), bonds=w["bonds"])[0]
    assert np.linalg.norm(Fp - Fw) / np.linalg.norm(Fw) < 1e-5
    s.close()


def training_frames(nf=2, seed=3):
    w, pos, box = melt()
    g = np.random.default_rng(seed)
    frames = [pos] + [(pos + g.normal(scale=0.03, size=pos.shape)) % box for _ in range(nf - 1)]
    f_ref = [oracle.forces(p, box, oracle.pair_params(rc=WCA))[0] for p in frames]
    return w, box, np.array(frames), np.array(f_ref)


@pytest.mark.parametrize("prec,tol_l,tol_g", [("fp32", 1e-5, 1e-4), ("bf16", 2e-2, 5e-2)])
def test_loss_gradient_matches_oracle(prec, tol_l, tol_g):
    w, box, frames, f_ref = training_frames()
    banner("surrogate loss/gradient %s, 2 frames of 1000" % prec)
    s = sur_system(w, frames[0], bonded=False)
    m, istd = norm32(frames[0], box)
    th = theta32(scale=0.5)
    s.sur_set(th, m, istd, prec)
    loss, grad = s.loss_grad(frames, f_ref)
    grad = grad.cpu().numpy()
    lo, go = S.loss_grad(th, m, istd, list(frames), list(f_ref), box)
    gerr = np.linalg.norm(grad - go) / np.linalg.norm(go)
    print("%s: loss %.6g vs %.6g (rel %.3g), gradient rel err %.3g" % (prec, loss, lo, rel(loss, lo), gerr))
    assert rel(loss, lo) < tol_l
    assert gerr < tol_g
    assert grad[S.O_B3] == 0.0
    if prec == "fp32":
        # per-block gradients: each parameter group on its own
        for a, b in ((S.O_W1, S.O_B1), (S.O_B1, S.O_W2), (S.O_W2, S.O_B2), (S.O_B2, S.O_W3), (S.O_W3, S.O_B3)):
            assert np.linalg.norm(grad[a:b] - go[a:b]) <= 1e-4 * np.linalg.norm(go[a:b]) + 1e-12
        # one Adam step on the master weights
        s.adam(1, 1e-3)
        th1 = s.sur_get().astype(np.float64)
        to, _, _ = S.adam_step(th, np.zeros_like(th), np.zeros_like(th), grad.astype(np.float64), 1, 1e-3)
        assert np.abs(th1 - to).max() < 1e-6
    s.close()


def test_training_lowers_the_loss():
    w, box, frames, f_ref = training_frames(nf=2, seed=5)
    banner("surrogate 30 Adam steps fp32")
    s = sur_system(w, frames[0], bonded=False)
    m, istd = norm32(frames[0], box)
    s.sur_set(theta32(scale=0.3), m, istd, "fp32")
    l0 = None
    for t in range(1, 31):
        loss, _ = s.loss_grad(frames, f_ref, want_grad=False)
        l0 = loss if l0 is None else l0
        s.adam(t, 3e-3)
    l1, _ = s.loss_grad(frames, f_ref, want_grad=False)
    print("loss %.4g -> %.4g" % (l0, l1))
    assert l1 < 0.5 * l0
    s.close()


def test_surrogate_nve_conserves_its_energy():
    """NVE with surrogate forces: the total energy drifts far less than the
    kinetic energy fluctuates, which holds only if F = -grad E."""
    w, pos, box = melt()
    banner("surrogate NVE energy conservation")
    vel = inputs.maxwell_boltzmann(pos.shape[0], 0.5, seed=11)
    s = System(pos, box, vel, pair={(0, 0): lj_pair(rc=WCA)}, bonds=w["bonds"], skin=SKIN, list_cutoff=S.RD,
               surrogate=True, dt=0.002, integrator="nve")
    m, istd = norm32(pos, box)
    s.sur_set(theta32(scale=0.3), m, istd, "fp32")
    s.set_pair_mode("surrogate")
    s.step(400)
    h = s.history()
    et = np.array([r["e_total"] for r in h])
    ek = np.array([r["e_kin"] for r in h])
    print("E_total std %.3g drift %.3g; E_kin std %.3g" % (et.std(), et[-1] - et[0], ek.std()))
    assert s.status() == 0
    assert abs(et[-1] - et[0]) < 0.02 * ek.std() * 10 and et.std() < 0.05 * ek.std()
    s.close()


def test_pair_forces_of_a_linear_readout():
    """A constant input gradient c (a linear readout of G) gives pair-potential
    forces linear in c; compared with the oracle's pair forces."""
    w, pos, box = melt()
    banner("surrogate pair forces, constant input gradient")
    s = sur_system(w, pos, bonded=False)
    c = np.random.default_rng(2).normal(size=32)
    a = np.tile(c, (pos.shape[0], 1)).astype(np.float32)
    F = s.sur_pair_forces(a).cpu().numpy()
    Fo, W, fs = S.pair_forces(a.astype(np.float64), pos, box, want_fscale=True)
    err = np.linalg.norm(F - Fo) / np.linalg.norm(Fo)
    print("linear readout forces rel err %.3g" % err)
    assert err < 1e-5
    assert (np.linalg.norm(F - Fo, axis=1) <= 1e-5 * fs + 1e-12).all()
    # linearity in c
    F2 = s.sur_pair_forces(2.0 * a).cpu().numpy()
    assert np.abs(F2 - 2.0 * F).max() <= 1e-6 * np.abs(F).max()
    s.close()


def test_trained_network_gains_over_the_untrained_one():
    """Force matching on frames of a plain-method run: the trained network's
    held-out force RMSE is well below the untrained one's.  The linear
    readout of the descriptors (a pair potential) is reported beside it:
    the target, WCA, is itself a pair potential."""
    from paper_2608_14911_amd import surrogate_experiment as X
    banner("surrogate gain: 10,000 beads, 24 frames")
    w, frames, fref = X.make_dataset(10, 1000, 24, 50, seed=77)
    ftr, rtr, fva, rva = frames[:20], fref[:20], frames[20:], fref[20:]
    s = System(frames[0].cpu().numpy(), w["box"], pair={(0, 0): lj_pair(rc=WCA)}, skin=0.4, list_cutoff=S.RD,
               surrogate=True)
    mean, istd = X.descriptor_stats(s, ftr)
    th0 = inputs.mlp_init(77)
    s.sur_set(th0, mean, istd, "fp32")
    r0 = X.rmse(s, fva, rva)
    X.train(s, th0, mean, istd, "bf16", ftr, rtr, epochs=12, lr0=3e-3, seed=77)
    r1 = X.rmse(s, fva, rva)
    c = X.linear_readout(s, ftr, rtr, 8)
    rl = X.linear_rmse(s, c, fva, rva)
    rms = float((rva * rva).mean().sqrt())
    print("held-out force RMSE / RMS F_ref: untrained %.3f, trained (BF16) %.3f, linear readout %.4f" % (
        r0 / rms, r1 / rms, rl / rms))
    assert r1 < 0.6 * r0
    assert rl < r0
    s.close()
