"""A simulation handle with torch-owned device memory.

``System`` mirrors the nouns of the paper's scripting interface (section
"Example usage": System, OrthorhombicBC box, VerletList(cutoff) + skin,
LennardJones / LennardJonesCapped, VelocityVerlet + LangevinThermostat,
addParticles, run(n), computeEnergy()).  It only marshals arguments: torch
allocates the workspace and the state buffers and supplies the stream; every
step of the computation runs in libmdgpu.so (see md.py).
"""
import math

import numpy as np

from . import md


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the MD library runs on gfx950 only")
    return torch


class System:
    def __init__(self, pos, box, vel=None, *, types=None, n_types=1, pair=None, masses=(1.0,),
                 bonds=None, angles=None, dt=0.005, skin=0.3, integrator="nve", precision="fp32",
                 temperature=1.0, gamma=0.0, seed=0, fene_K=30.0, fene_R0=1.5, k_bend=0.0,
                 nl_capacity=0, flags=0, cell_factor=0, list_cutoff=0.0, surrogate=False, shear_rate=0.0,
                 dpd_rc=0.0, table_points=0, angle_kind=0, angle_K=0.0, angle_phi0=0.0, adress=None,
                 block_size=0, device="cuda"):
        torch = _torch()
        self.torch = torch
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        n = pos.shape[0]
        self.n = n
        self.box = np.asarray(box, dtype=np.float64)
        vel = np.zeros_like(pos) if vel is None else np.ascontiguousarray(vel, dtype=np.float64)
        self.device = torch.device(device)
        integ = {"langevin": md.MD_LANGEVIN, "dpd": md.MD_DPD}.get(integrator, md.MD_NVE)
        prec = md.MD_FP64 if precision == "fp64" else md.MD_FP32
        nb = 0 if bonds is None else len(bonds)
        na = 0 if angles is None else len(angles)
        self.cfg = md.make_config(n, self.box, n_types=n_types, pair=pair, dt=dt, skin=skin, integrator=integ,
                                  force_precision=prec, temperature=temperature, gamma=gamma, seed=seed,
                                  n_bonds=nb, n_angles=na, fene_K=fene_K, fene_R0=fene_R0, k_bend=k_bend,
                                  nl_capacity=nl_capacity, flags=flags, cell_factor=cell_factor,
                                  list_cutoff=list_cutoff, surrogate=int(bool(surrogate)),
                                  shear_rate=shear_rate, dpd_rc=dpd_rc, table_points=table_points,
                                  angle_kind=angle_kind, angle_K=angle_K, angle_phi0=angle_phi0, adress=adress,
                                  block_size=block_size)
        self.ws_bytes = md.md_workspace_bytes(self.cfg)
        self._ws_raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws_raw.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.stream = torch.cuda.current_stream(self.device)
        dpos = torch.as_tensor(pos, device=self.device)
        dvel = torch.as_tensor(vel, device=self.device)
        dtype_ = None if types is None else torch.as_tensor(np.asarray(types, dtype=np.int32), device=self.device)
        self.masses = np.asarray(masses, dtype=np.float64)
        self.h = md.md_init(self.cfg, dpos.data_ptr(), dvel.data_ptr(),
                            None if dtype_ is None else dtype_.data_ptr(), self.masses,
                            bonds, angles, self.ws_ptr, self.ws_bytes, self.stream.cuda_stream)
        self._closed = False

    # -------------------------------------------------------------- control
    def set_params(self, **kw):
        c = self.cfg
        if "pair" in kw:
            for (a, b), row in kw.pop("pair").items():
                for (x, y) in ((a, b), (b, a)):
                    pp = c.pair[x * md.MD_MAX_TYPES + y]
                    pp.eps, pp.sigma, pp.rc, pp.shift, pp.caprad = (float(v) for v in row)
        for k, v in kw.items():
            if k == "integrator":
                v = {"langevin": md.MD_LANGEVIN, "dpd": md.MD_DPD}.get(v, md.MD_NVE)
            if k == "precision":
                k, v = "force_precision", (md.MD_FP64 if v == "fp64" else md.MD_FP32)
            setattr(c, k, v)
        md.md_set_params(self.h, c)

    def set_pair_table(self, ti, tj, u, f, rmin):
        """Tabulated pair potential of types (ti, tj): energies u and radial
        forces f on the uniform grid from rmin to the pair's cutoff."""
        md.md_set_pair_table(self.h, ti, tj, u, f, rmin)

    def set_cg_table(self, ti, tj, u, f, rmin, rc_cg):
        """AdResS: the coarse-grained pair potential of types (ti, tj)."""
        md.md_set_cg_table(self.h, ti, tj, u, f, rmin, rc_cg)

    def set_angle_table(self, u, dudphi):
        md.md_set_angle_table(self.h, u, dudphi)

    def set_angle_subens(self, u_tables, g_tables, weights):
        md.md_set_angle_subens(self.h, u_tables, g_tables, weights)

    def step(self, n):
        md.md_step(self.h, n)

    def build_neighbors(self):
        md.md_build_neighbors(self.h)

    def observables(self, check=True):
        return md.md_observables(self.h, check=check)

    def history(self):
        return md.md_history(self.h)

    def forces(self):
        f = self.torch.zeros((self.n, 3), dtype=self.torch.float64, device=self.device)
        md.md_forces(self.h, f.data_ptr())
        self.stream.synchronize()
        return f.cpu().numpy()

    def get_state(self):
        t = self.torch
        z = lambda dt_: t.zeros((self.n, 3), dtype=dt_, device=self.device)
        pos, vel, pb, img = z(t.float64), z(t.float64), z(t.float64), z(t.int32)
        step, vh = md.md_get_state(self.h, pos.data_ptr(), vel.data_ptr(), img.data_ptr(), pb.data_ptr())
        self.stream.synchronize()
        return {"pos": pos.cpu().numpy(), "vel": vel.cpu().numpy(), "image": img.cpu().numpy(),
                "pos_build": pb.cpu().numpy(), "step": step, "vel_half": vh}

    def set_state(self, state, with_build=True):
        """Replace the state; arrays may be numpy or torch tensors."""
        t = self.torch
        pos = self._dev(state["pos"], t.float64)
        vel = self._dev(state["vel"], t.float64)
        img = None
        if state.get("image") is not None:
            img = self._dev(state["image"], t.int32)
        pb = None
        if with_build and state.get("pos_build") is not None:
            pb = self._dev(state["pos_build"], t.float64)
        md.md_set_state(self.h, pos.data_ptr(), vel.data_ptr(), None if img is None else img.data_ptr(),
                        None if pb is None else pb.data_ptr(), state.get("step", 0), state.get("vel_half", 0))
        self.stream.synchronize()

    def neighbors(self, cap=None, sort=True):
        """Neighbour tags of every particle (by tag), sorted, or in row order
        with sort=False."""
        t = self.torch
        cap = cap or int(self.cfg.nl_capacity or 512)
        cnt = t.zeros(self.n, dtype=t.int32, device=self.device)
        idx = t.full((self.n, cap), -1, dtype=t.int32, device=self.device)
        md.md_get_neighbors(self.h, cnt.data_ptr(), idx.data_ptr(), cap)
        c = cnt.cpu().numpy()
        m = idx.cpu().numpy()
        if not sort:
            return [m[i, :c[i]].copy() for i in range(self.n)]
        return [np.sort(m[i, :c[i]]) for i in range(self.n)]

    def timing(self, enable=None):
        if enable is not None:
            md.md_timing_enable(self.h, enable)
            return None
        return md.md_timing_read(self.h)

    def status(self):
        return md.md_status_check(self.h)

    # ------------------------------------------------------------ surrogate
    def _dev(self, x, dtype):
        t = self.torch
        if isinstance(x, t.Tensor):
            return x.to(device=self.device, dtype=dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(x), device=self.device, dtype=dtype)

    def sur_set(self, theta, g_mean, g_istd, precision="fp32"):
        """Load network parameters (6,337 values) and the descriptor
        standardisation (mean, 1/std per basis function)."""
        t = self.torch
        self._sur = [self._dev(theta, t.float32), self._dev(g_mean, t.float32), self._dev(g_istd, t.float32)]
        prec = md.MD_SUR_BF16 if precision == "bf16" else md.MD_SUR_FP32
        md.md_sur_set(self.h, self._sur[0].data_ptr(), self._sur[1].data_ptr(), self._sur[2].data_ptr(), prec)
        self.stream.synchronize()

    def sur_get(self):
        t = self.torch
        th = t.zeros(md.MD_SUR_NPARAM, dtype=t.float32, device=self.device)
        md.md_sur_get(self.h, th.data_ptr())
        self.stream.synchronize()
        return th.cpu().numpy()

    def set_pair_mode(self, mode):
        md.md_set_pair_mode(self.h, md.MD_PAIR_SURROGATE if mode == "surrogate" else md.MD_PAIR_PLAIN)

    def descriptors(self):
        t = self.torch
        G = t.zeros((self.n, md.MD_SUR_NBASIS), dtype=t.float32, device=self.device)
        md.md_sur_descriptors(self.h, G.data_ptr())
        self.stream.synchronize()
        return G

    def desc_stats(self, frames):
        """Standardisation constants (mean, 1/std per basis function) of the
        descriptors over device frames [nf, N, 3] (FP64); replaces the state
        with the last frame, like loss_grad."""
        t = self.torch
        frames = self._dev(frames, t.float64)
        m = t.zeros(md.MD_SUR_NBASIS, dtype=t.float32, device=self.device)
        istd = t.zeros(md.MD_SUR_NBASIS, dtype=t.float32, device=self.device)
        md.md_sur_desc_stats(self.h, frames.data_ptr(), frames.shape[0], m.data_ptr(), istd.data_ptr())
        self.stream.synchronize()
        return m, istd

    def mlp_eval(self, G):
        """Per-row energies and dE/dG for descriptor rows G [P, 32]."""
        t = self.torch
        G = self._dev(G, t.float32)
        P = G.shape[0]
        e = t.zeros(P, dtype=t.float32, device=self.device)
        a = t.zeros((P, md.MD_SUR_NBASIS), dtype=t.float32, device=self.device)
        md.md_sur_mlp_eval(self.h, G.data_ptr(), P, e.data_ptr(), a.data_ptr())
        self.stream.synchronize()
        return e, a

    def sur_pair_forces(self, dedg):
        """Surrogate pair forces at the current positions for given
        per-particle input gradients dedg [N, 32] (device FP64 [N, 3])."""
        t = self.torch
        a = self._dev(dedg, t.float32)
        f = t.zeros((self.n, 3), dtype=t.float64, device=self.device)
        md.md_sur_pair_forces(self.h, a.data_ptr(), f.data_ptr())
        return f

    def loss_grad(self, frames, f_ref, want_grad=True):
        """Force-matching loss over device frames [nf, N, 3] (FP64) and
        reference forces [nf, N, 3] (FP64); returns (loss, grad or None)."""
        t = self.torch
        frames = self._dev(frames, t.float64)
        f_ref = self._dev(f_ref, t.float64)
        g = t.zeros(md.MD_SUR_NPARAM, dtype=t.float32, device=self.device) if want_grad else None
        loss = md.md_sur_loss_grad(self.h, frames.data_ptr(), f_ref.data_ptr(), frames.shape[0],
                                   None if g is None else g.data_ptr())
        return loss, g

    def adam(self, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        md.md_sur_adam(self.h, t, lr, beta1, beta2, eps)

    def close(self):
        if not self._closed:
            md.md_destroy(self.h)
            self._closed = True

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prepare_replica(m, log=None):
    """Push off a raw Kremer-Grest replica on the GPU (capped WCA ladder, then
    200 steps at its own run parameters); returns the member dict with the
    new positions and velocities.  LJ replicas are returned unchanged."""
    if m.get("kind") != "kg":
        return m
    rc = m["pair"][(0, 0)][2]
    s = System(m["pos"], m["box"], np.zeros_like(m["pos"]), pair={(0, 0): lj_pair(rc=rc, caprad=1.0)},
               bonds=m["bonds"], angles=m["angles"], k_bend=m["k_bend"], dt=0.002, skin=m["skin"],
               integrator="langevin", temperature=m["temperature"], gamma=1.0, seed=m["seed"], nl_capacity=256)
    push_off(s, rc, chunk=1000, log=log)
    s.set_params(dt=m["dt"], gamma=m["gamma"])
    s.step(200)
    st = s.get_state()
    code = s.status()
    s.close()
    if code != 0:
        raise RuntimeError("replica push-off failed: %s" % md.status_string(code))
    out = dict(m)
    out["pos"], out["vel"] = st["pos"], st["vel"]
    return out


def nl_build_flags(name):
    """md_config.flags bits for a list-build choice."""
    return {"auto": 0, "tiles": md.MD_CFG_NL_TILES, "per_particle": md.MD_CFG_NL_PER_PARTICLE}[name]


class Batch:
    """Many independent systems advanced together (md_batch_*).

    ``members``: list of dicts with the keys of ``System`` (pos, box, vel,
    pair, bonds, angles, dt, skin, integrator, temperature, gamma, seed,
    k_bend, cell_factor, nl_capacity, masses) and ``nl_build`` ("auto",
    "tiles" or "per_particle": the Verlet-list build)."""

    def __init__(self, members, device="cuda"):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.cfgs, self._keep, pos_p, vel_p, masses, bonds, angles = [], [], [], [], [], [], []
        self.n = []
        for m in members:
            pos = np.ascontiguousarray(m["pos"], dtype=np.float64)
            n = pos.shape[0]
            vel = m.get("vel")
            vel = np.zeros_like(pos) if vel is None else np.ascontiguousarray(vel, dtype=np.float64)
            b, a = m.get("bonds"), m.get("angles")
            integ = md.MD_LANGEVIN if m.get("integrator", "nve") == "langevin" else md.MD_NVE
            cfg = md.make_config(n, m["box"], pair=m.get("pair"), dt=m.get("dt", 0.005), skin=m.get("skin", 0.3),
                                 integrator=integ, force_precision=md.MD_FP32,
                                 temperature=m.get("temperature", 1.0), gamma=m.get("gamma", 0.0),
                                 seed=m.get("seed", 0), n_bonds=0 if b is None else len(b),
                                 n_angles=0 if a is None else len(a), fene_K=m.get("fene_K", 30.0),
                                 fene_R0=m.get("fene_R0", 1.5), k_bend=m.get("k_bend", 0.0),
                                 nl_capacity=m.get("nl_capacity", 0), cell_factor=m.get("cell_factor", 0),
                                 flags=nl_build_flags(m.get("nl_build", "auto")))
            dp = torch.as_tensor(pos, device=self.device)
            dv = torch.as_tensor(vel, device=self.device)
            self._keep += [dp, dv]
            self.cfgs.append(cfg)
            pos_p.append(dp.data_ptr())
            vel_p.append(dv.data_ptr())
            masses.append(np.asarray(m.get("masses", (1.0,)), dtype=np.float64))
            bonds.append(b)
            angles.append(a)
            self.n.append(n)
        self.nsys = len(members)
        self.ws_bytes = md.md_batch_workspace_bytes(self.cfgs)
        self._ws_raw = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        self.ws_ptr = (self._ws_raw.data_ptr() + 255) & ~255
        self.stream = torch.cuda.current_stream(self.device)
        self.h = md.md_batch_init(self.cfgs, pos_p, vel_p, masses, bonds, angles, self.ws_ptr, self.ws_bytes,
                                  self.stream.cuda_stream)
        self._keep = []
        self._closed = False

    def step(self, n):
        md.md_batch_step(self.h, n)

    def observables(self, check=True):
        return md.md_batch_observables(self.h, self.nsys, check)

    def timing(self, enable=None):
        if enable is not None:
            md.md_batch_timing_enable(self.h, enable)
            return None
        return md.md_batch_timing_read(self.h)

    def get_state(self, s):
        t = self.torch
        n = self.n[s]
        z = lambda dt_: t.zeros((n, 3), dtype=dt_, device=self.device)
        pos, vel, pb, img = z(t.float64), z(t.float64), z(t.float64), z(t.int32)
        step, vh = md.md_batch_get_state(self.h, s, pos.data_ptr(), vel.data_ptr(), img.data_ptr(), pb.data_ptr())
        self.stream.synchronize()
        return {"pos": pos.cpu().numpy(), "vel": vel.cpu().numpy(), "image": img.cpu().numpy(),
                "pos_build": pb.cpu().numpy(), "step": step, "vel_half": vh}

    def close(self):
        if not self._closed:
            md.md_batch_destroy(self.h)
            self._closed = True

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lj_pair(eps=1.0, sigma=1.0, rc=2.5, shift=math.nan, caprad=0.0):
    return (eps, sigma, rc, shift, caprad)


def from_workload(w, precision="fp32", **kw):
    """System for a workload dict from inputs.py."""
    pair = {(0, 0): lj_pair(w["eps"], w["sigma"], w["rc"], w["shift"], w["caprad"])}
    return System(w["pos"], w["box"], w["vel"], pair=pair, bonds=w.get("bonds"), angles=w.get("angles"),
                  dt=w["dt"], skin=w["skin"], integrator=w["integrator"], precision=precision,
                  temperature=w["temperature"], gamma=w["gamma"], seed=w["seed"],
                  fene_K=w.get("fene_K", 30.0), fene_R0=w.get("fene_R0", 1.5), k_bend=w.get("k_bend", 0.0),
                  **kw)


# Capped-WCA push-off of overlapping random-walk chains, modelled on the
# paper's example (section "Example usage": a capped warm-up at a small time
# step, then the uncapped potential).  Rows: (capping radius, dt, steps).
PUSHOFF = ((1.0, 0.002, 500), (0.95, 0.002, 500), (0.9, 0.002, 1000), (0.85, 0.002, 1000),
           (0.8, 0.002, 1000), (0.0, 0.005, 1000))


def push_off(s, rc, schedule=PUSHOFF, chunk=250, max_halvings=4, log=None):
    """Run the push-off ladder on the GPU system ``s`` (pair type (0, 0)).

    Each stage runs in chunks from a host checkpoint; when a chunk latches a
    device error (a FENE bond at R0, a non-finite coordinate) the state is
    restored and the chunk is repeated at half the time step, down to
    dt / 2**max_halvings.  Large melts hold rare clusters of overlapping
    beads that a fixed time step tears apart.  Raises RuntimeError when a
    chunk still fails at the smallest step."""
    for caprad, dt, nsteps in schedule:
        s.set_params(pair={(0, 0): lj_pair(1.0, 1.0, rc, math.nan, caprad)})
        done = 0
        while done < nsteps:
            ns = min(chunk, nsteps - done)
            ck = s.get_state()
            for k in range(max_halvings + 1):
                sub = 2 ** k
                s.set_params(dt=dt / sub)
                s.step(ns * sub)
                code = s.status()
                if code == 0:
                    break
                if log:
                    log("push-off cap %.3g: chunk at dt %.3g failed (%s), halving" % (caprad, dt / sub,
                                                                                     md.status_string(code)))
                s.set_state(ck)
            else:
                raise RuntimeError("push-off failed at capping radius %g" % caprad)
            done += ns
