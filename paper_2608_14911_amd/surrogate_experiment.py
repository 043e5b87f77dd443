"""Train the learned non-bonded surrogate on a plain-method Kremer-Grest melt
and compare it with the plain WCA pair force.

    python -m paper_2608_14911_amd.surrogate_experiment [--quick] [--out report.json]

1. Data: an N_train-bead melt (random walks at density 0.85, WCA + FENE +
   bending 1.5, Langevin T = 1, gamma = 0.5, dt = 0.01) pushed off and
   equilibrated on the GPU; frames every 50 steps.  Labels are the plain WCA
   forces in FP64 from the plain kernel (pair part only).
2. Training: force matching with Adam (cosine decay from lr0), minibatches of
   4 frames in a Philox-stream-5 order, in FP32 and in BF16 (matrix-core
   operands, FP32 accumulation, FP32 master weights).
3. Baselines on the held-out frames: the untrained network, and a linear
   readout of the descriptors (a pair potential u(r) = 2 c . g(r), fitted by
   least squares on the training forces).
4. Inference on an N_inf-bead melt: plain WCA vs the surrogate (FP32, BF16)
   from the same state and seed: force RMSE at the shared start, radial
   distribution function against the plain-vs-plain noise floor (two noise
   seeds), mean pressure with its standard error, bead-steps per second.

Every force, descriptor, network and training step runs in libmdgpu.so;
torch holds the device arrays, and the analysis (least-squares solve of the
32 x 32 normal equations, histograms, averages) is plain torch / numpy.
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs, md
from .system import System, lj_pair, push_off

WCA = 2.0 ** (1.0 / 6.0)


def log(msg):
    print("[surrogate] " + msg, file=sys.stderr, flush=True)


def kg_melt(n_chains, chain_len, seed, equil, k_bend=1.5):
    """Pushed-off, equilibrated KG melt: (state dict, workload dict)."""
    w = inputs.workload_kg(n_chains, chain_len, seed=seed)
    w["k_bend"] = k_bend
    s = System(w["pos"], w["box"], np.zeros_like(w["pos"]), pair={(0, 0): lj_pair(rc=WCA, caprad=1.0)},
               bonds=w["bonds"], angles=w["angles"], k_bend=k_bend, dt=0.002, skin=0.4, integrator="langevin",
               temperature=1.0, gamma=1.0, seed=seed, nl_capacity=256)
    push_off(s, WCA, log=log)
    s.set_params(dt=0.01, gamma=0.5)
    s.step(equil)
    st = s.get_state()
    if s.status() != 0:
        raise RuntimeError("melt preparation failed")
    s.close()
    return st, w


def melt_system(st, w, surrogate):
    """The melt at state st (WCA + FENE + bending, Langevin T = 1, gamma =
    0.5, dt = 0.01, skin 0.4).  With surrogate, the list also reaches the
    descriptor cutoff, so the handle runs plain and surrogate forces."""
    s = System(st["pos"], w["box"], st["vel"], pair={(0, 0): lj_pair(rc=WCA)}, bonds=w["bonds"],
               angles=w["angles"], k_bend=w["k_bend"], dt=0.01, skin=0.4, integrator="langevin", temperature=1.0,
               gamma=0.5, seed=w["seed"], list_cutoff=md.MD_SUR_RCUT if surrogate else 0.0, surrogate=surrogate)
    s.set_state(st)
    return s


def device_positions(s):
    t = s.torch
    pos = t.zeros((s.n, 3), dtype=t.float64, device=s.device)
    md.md_get_state(s.h, pos.data_ptr(), None, None, None)
    return pos


def plain_pair_forces(label, frame):
    """FP64 plain WCA forces (no bonded terms) at one frame, on the device."""
    t = label.torch
    label.set_state({"pos": frame, "vel": t.zeros_like(frame)}, with_build=False)
    f = t.zeros((label.n, 3), dtype=t.float64, device=label.device)
    md.md_forces(label.h, f.data_ptr())
    return f


def set_positions(s, frame):
    t = s.torch
    s.set_state({"pos": frame, "vel": t.zeros_like(frame)}, with_build=False)


def make_dataset(n_chains, chain_len, nframes, every, seed):
    st, w = kg_melt(n_chains, chain_len, seed, equil=1000)
    s = melt_system(st, w, surrogate=False)
    t = s.torch
    frames = t.zeros((nframes, s.n, 3), dtype=t.float64, device=s.device)
    for f in range(nframes):
        s.step(every)
        frames[f] = device_positions(s)
    assert s.status() == 0
    s.close()
    label = System(frames[0].cpu().numpy(), w["box"], pair={(0, 0): lj_pair(rc=WCA)}, skin=0.4, precision="fp64")
    fref = t.zeros_like(frames)
    for f in range(nframes):
        fref[f] = plain_pair_forces(label, frames[f])
    label.close()
    return w, frames, fref


def descriptor_stats(s, frames):
    """The network's fixed standardisation constants (mean, 1/sqrt(var + 1e-6))
    over every bead of the training frames, from the library's own kernels."""
    return s.desc_stats(frames)


def rmse(s, frames, fref):
    loss, _ = s.loss_grad(frames, fref, want_grad=False)
    return math.sqrt(loss)


def train(s, theta0, mean, istd, precision, frames, fref, epochs, lr0, seed, batch=4, val=None):
    t = s.torch
    s.sur_set(theta0, mean, istd, precision)
    nf = frames.shape[0]
    nb = nf // batch
    total = epochs * nb
    order = inputs.rng(seed, 5)
    step = 0
    hist = []
    for ep in range(epochs):
        perm = t.as_tensor(order.permutation(nf)[:nb * batch], device=s.device)
        ep_loss = 0.0
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            loss, _ = s.loss_grad(frames.index_select(0, idx), fref.index_select(0, idx), want_grad=False)
            lr = lr0 * 0.5 * (1.0 + math.cos(math.pi * step / total))
            step += 1
            s.adam(step, lr)
            ep_loss += loss
        rec = {"epoch": ep + 1, "train_rmse": math.sqrt(ep_loss / nb)}
        if val is not None and (ep + 1 == epochs or (ep + 1) % max(1, epochs // 5) == 0):
            rec["val_rmse"] = rmse(s, *val)
        hist.append(rec)
        log("%s epoch %d: %s" % (precision, ep + 1, rec))
    return s.sur_get(), hist


def linear_readout(s, frames, fref, nfit):
    """Least-squares c for F = sum_k c_k F(e_k) over nfit training frames."""
    t = s.torch
    ata = t.zeros((32, 32), dtype=t.float64, device=s.device)
    atb = t.zeros(32, dtype=t.float64, device=s.device)
    eye = t.eye(32, dtype=t.float32, device=s.device)
    for f in range(nfit):
        set_positions(s, frames[f])
        cols = [s.sur_pair_forces(eye[k].expand(s.n, 32)).reshape(-1) for k in range(32)]
        A = t.stack(cols, 1)
        ata += A.T @ A
        atb += A.T @ fref[f].reshape(-1)
    return t.linalg.solve(ata, atb)


def linear_rmse(s, c, frames, fref):
    t = s.torch
    a = c.float().expand(s.n, 32)
    se = 0.0
    for f in range(frames.shape[0]):
        set_positions(s, frames[f])
        d = s.sur_pair_forces(a) - fref[f]
        se += float((d * d).sum())
    return math.sqrt(se / (3.0 * s.n * frames.shape[0]))


def rdf(pos, box, nq=4000, rmax=3.0, dr=0.02, seed=0):
    from scipy.spatial import cKDTree
    pos = np.mod(pos, box)
    tree = cKDTree(pos, boxsize=box)
    q = pos[np.random.default_rng(seed).choice(pos.shape[0], size=nq, replace=False)]
    d, _ = tree.query(q, k=256, distance_upper_bound=rmax)
    d = d[np.isfinite(d) & (d > 0)]
    edges = np.arange(0.0, rmax + 1e-9, dr)
    h, _ = np.histogram(d, bins=edges)
    rho = pos.shape[0] / float(np.prod(box))
    shell = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    return 0.5 * (edges[1:] + edges[:-1]), h / (nq * rho * shell)


def block_mean(x, nblocks=10):
    x = np.asarray(x)
    b = np.array_split(x, nblocks)
    m = np.array([v.mean() for v in b])
    return float(x.mean()), float(m.std(ddof=1) / math.sqrt(nblocks))


def run_leg(s, st, mode, seed, steps, theta=None, mean=None, istd=None, precision="fp32"):
    """steps of Langevin dynamics from state st; returns pressures, final
    positions and bead-steps/s."""
    s.set_state(st)
    s.set_params(seed=seed)
    if mode == "surrogate":
        s.sur_set(theta, mean, istd, precision)
        s.set_pair_mode("surrogate")
    else:
        s.set_pair_mode("plain")
    s.history()
    s.step(2)
    s.stream.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.stream.synchronize()
    el = time.perf_counter() - t0
    h = s.history()
    if s.status() != 0:
        raise RuntimeError("%s run failed with status %d" % (mode, s.status()))
    p = [r["pressure"] for r in h[2:]]
    pos = s.get_state()["pos"]
    return p, pos, s.n * steps / el


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="small sizes (CI scale)")
    ap.add_argument("--out", default="")
    ap.add_argument("--epochs", type=int, default=0)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--save", default="", help="write the trained models (npz: theta_fp32, theta_bf16, "
                                               "g_mean, g_istd) to this path")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    if a.quick:
        tr_chains, tr_len, nframes, every, ntrain, inf_chains, epochs, steps = 20, 1000, 40, 50, 32, 50, 10, 200
    else:
        tr_chains, tr_len, nframes, every, ntrain, inf_chains, epochs, steps = 100, 1000, 200, 50, 180, 1000, 60, 500
    epochs = a.epochs or epochs
    rep = {"config": {"train_beads": tr_chains * tr_len, "frames": nframes, "every": every, "train_frames": ntrain,
                      "val_frames": nframes - ntrain, "epochs": epochs, "batch": 4, "lr0": a.lr,
                      "inference_beads": inf_chains * 1000, "inference_steps": steps}}
    t0 = time.time()
    w, frames, fref = make_dataset(tr_chains, tr_len, nframes, every, seed=1004)
    log("dataset: %d frames of %d beads in %.1f s" % (nframes, frames.shape[1], time.time() - t0))
    ftr, rtr = frames[:ntrain], fref[:ntrain]
    fva, rva = frames[ntrain:], fref[ntrain:]
    rms_ref = float(torch.sqrt((rva * rva).mean()))
    s = System(frames[0].cpu().numpy(), w["box"], pair={(0, 0): lj_pair(rc=WCA)}, skin=0.4,
               list_cutoff=md.MD_SUR_RCUT, surrogate=True)
    mean, istd = descriptor_stats(s, ftr)
    theta0 = inputs.mlp_init(1004)
    s.sur_set(theta0, mean, istd, "fp32")
    untrained = rmse(s, fva, rva)
    c = linear_readout(s, ftr, rtr, min(ntrain, 40))
    lin = linear_rmse(s, c, fva, rva)
    res = {"rms_f_ref": rms_ref, "untrained": untrained, "linear_readout": lin}
    models = {}
    for prec in ("fp32", "bf16"):
        t1 = time.time()
        th, hist = train(s, theta0, mean, istd, prec, ftr, rtr, epochs, a.lr, seed=1004, val=(fva, rva))
        models[prec] = th
        s.sur_set(th, mean, istd, prec)
        res["trained_" + prec] = rmse(s, fva, rva)
        res["train_seconds_" + prec] = time.time() - t1
        res["history_" + prec] = hist
    if a.save:
        np.savez(a.save, theta_fp32=models["fp32"], theta_bf16=models["bf16"],
                 g_mean=mean.cpu().numpy(), g_istd=istd.cpu().numpy())
    # the FP32-trained weights evaluated with BF16 operands
    s.sur_set(models["fp32"], mean, istd, "bf16")
    res["trained_fp32_eval_bf16"] = rmse(s, fva, rva)
    s.close()
    rep["validation_force_rmse"] = res
    rep["validation_force_rmse_relative"] = {k: v / rms_ref for k, v in res.items()
                                             if isinstance(v, float) and k not in ("rms_f_ref",)
                                             and not k.startswith("train_seconds")}
    log("validation RMSE: %s" % {k: v for k, v in res.items() if not k.startswith("history")})

    # inference on the large melt
    t2 = time.time()
    st, wb = kg_melt(inf_chains, 1000, seed=1014, equil=1000)
    box = wb["box"]
    legs = {}
    # plain legs on a handle whose list is the plain one (rc + skin)
    plain = melt_system(st, wb, surrogate=False)
    legs["plain_a"] = run_leg(plain, st, "plain", 11, steps)
    legs["plain_b"] = run_leg(plain, st, "plain", 12, steps)
    plain.close()
    big = melt_system(st, wb, surrogate=True)
    for prec in ("fp32", "bf16"):
        legs["sur_" + prec] = run_leg(big, st, "surrogate", 11, steps, models[prec], mean, istd, prec)
    # force RMSE at the shared start: surrogate minus plain (bonded terms cancel)
    big.set_state(st)
    big.set_pair_mode("plain")
    Fp = big.forces()
    pair_only = System(st["pos"], box, pair={(0, 0): lj_pair(rc=WCA)}, skin=0.4)
    Fw = pair_only.forces()
    pair_only.close()
    inf = {}
    for prec in ("fp32", "bf16"):
        big.set_state(st)
        big.sur_set(models[prec], mean, istd, prec)
        big.set_pair_mode("surrogate")
        Fs = big.forces()
        inf["force_rmse_" + prec] = float(np.sqrt(((Fs - Fp) ** 2).mean()))
    inf["rms_plain_pair_force"] = float(np.sqrt((Fw ** 2).mean()))
    r, g_a = rdf(legs["plain_a"][1], box)
    _, g_b = rdf(legs["plain_b"][1], box)
    inf["rdf_noise_floor_max"] = float(np.abs(g_b - g_a).max())
    inf["rdf_noise_floor_l2"] = float(np.sqrt(((g_b - g_a) ** 2).mean()))
    for k, (p, pos, rate) in legs.items():
        pm, pe = block_mean(p)
        inf["pressure_" + k] = [pm, pe]
        inf["bead_steps_per_s_" + k] = rate
        if k.startswith("sur"):
            _, g = rdf(pos, box)
            inf["rdf_max_diff_" + k] = float(np.abs(g - g_a).max())
            inf["rdf_l2_diff_" + k] = float(np.sqrt(((g - g_a) ** 2).mean()))
    big.close()
    inf["seconds"] = time.time() - t2
    rep["inference"] = inf
    log("inference: %s" % inf)
    txt = json.dumps(rep, indent=1)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(json.dumps({k: v for k, v in rep.items() if k != "validation_force_rmse"}))


if __name__ == "__main__":
    main()
