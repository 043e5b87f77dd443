"""FP64 CPU oracle for the short-range MD step (ESPResSo++, arXiv 2608.14911).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library in ``paper_2608_14911_amd`` and never imports it.

The arithmetic lives in ``md_oracle.c`` (plain C, FP64, no fused multiply-add);
this module only marshals numpy arrays through ctypes.  Functions and the
passages of the paper they follow:

* ``pair_eval``    -- LennardJones / LennardJonesCapped with shift='auto'
                      (section "Example usage").
* ``fene_eval``, ``bend_eval`` -- bonded interactions (section
                      "Functionality"); FENE and cosine bending of the
                      Kremer-Grest melt.
* ``forces``       -- F_i = -grad_i U summed over pairs inside the cutoff, by
                      brute force or the oracle's own linked cells (CellGrid,
                      section "Software design"), with the energies, the
                      virial W = sum r_ij . f_ij (computeEnergy(), pressure)
                      and the sum of its terms' magnitudes, W's scale.
* ``neighbors``    -- Verlet-list sets { j != i : r_ij^2 < (rc+skin)^2 }
                      (VerletList + system.skin, section "Example usage").
* ``run``          -- VelocityVerlet with the LangevinThermostat extension
                      (section "Example usage").
* ``philox``, ``gauss3`` -- the counter-based noise source (Philox4x64-10,
                      Salmon et al. 2011) that both sides implement
                      independently; ``philox32`` its 32-bit-word form
                      (Philox4x32-10, same paper), the DPD pair noise.
* ``forces_ext``, ``neighbors_le``, ``run_ext``, ``dpd_theta`` -- Lees-Edwards
                      sheared boundaries (section "New Features") and the
                      dissipative-particle-dynamics thermostat (section
                      "Functionality"), by brute force over pairs.
* ``tables(adress=..., cg=...)``, ``adress_weight`` -- AdResS force
                      interpolation (sections "Statement of need" and
                      "Functionality") on single-site molecules.
* ``tables``, ``angle_tables_combine`` -- tabulated pair and angle
                      potentials (section "Functionality") and
                      AngularCosineSquared / TabulatedSubEnsAngular (section
                      "New Features") for forces_ext / run_ext.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_md_oracle.so")
_lib = None

NOBS = 11   # e_pair, e_bond, e_angle, W, Wxx, Wyy, Wzz, Wxy, Wxz, Wyz, sum |r.f|
NHIST = 11  # e_pair, e_bond, e_angle, e_kin, W, tensor[6]

OK = 0
ERR_ARG = -1
ERR_NL_OVERFLOW = -4
ERR_BOND_BROKEN = -5
ERR_NONFINITE = -6


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with status %d" % (what, code))
        self.code = code


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, f64, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64
    lib.orc_philox4x64_10.argtypes = [P, P, P]
    lib.orc_philox4x64_10.restype = None
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_philox4x32_10.restype = None
    lib.orc_gauss3.argtypes = [u64, u64, u64, u64, P]
    lib.orc_gauss3.restype = None
    lib.orc_pair_eval.argtypes = [P, f64, P, P]
    lib.orc_pair_eval.restype = ctypes.c_int
    lib.orc_fene_eval.argtypes = [f64, f64, f64, P, P]
    lib.orc_fene_eval.restype = ctypes.c_int
    lib.orc_bend_eval.argtypes = [f64, P, P, P, P, P, P, P]
    lib.orc_bend_eval.restype = ctypes.c_int
    lib.orc_forces.argtypes = [i64, P, P, i32, P, P, i64, P, f64, f64, i64, P, f64, i32, i32, P, P, P]
    lib.orc_forces.restype = ctypes.c_int
    lib.orc_neighbors.argtypes = [i64, P, P, f64, i64, P, i32, P, P, i32]
    lib.orc_neighbors.restype = ctypes.c_int
    lib.orc_neighbors_cells.argtypes = [i64, P, P, f64, i32, P, P, i32]
    lib.orc_neighbors_cells.restype = ctypes.c_int
    lib.orc_run.argtypes = [i64, P, P, P, P, P, i32, P, P, i64, P, f64, f64, i64, P, f64,
                            f64, i32, f64, f64, u64, P, P, i64, i32, i32, P]
    lib.orc_run.restype = ctypes.c_int
    lib.orc_dpd_theta.argtypes = [u64, u64, u64, u64]
    lib.orc_dpd_theta.restype = f64
    lib.orc_forces_ext.argtypes = [i64, P, P, P, i32, P, P, i64, P, f64, f64, i64, P, f64, f64, f64, f64, f64, f64,
                                   u64, i64, P, P, P, P, P]
    lib.orc_forces_ext.restype = ctypes.c_int
    lib.orc_neighbors_le.argtypes = [i64, P, P, f64, f64, f64, i64, i32, P, P]
    lib.orc_neighbors_le.restype = ctypes.c_int
    lib.orc_run_ext.argtypes = [i64, P, P, P, P, P, i32, P, P, i64, P, f64, f64, i64, P, f64,
                                f64, i32, f64, f64, u64, f64, f64, P, P, P, i64, P]
    lib.orc_angle_tables_combine.argtypes = [i32, i32, P, P, P, P, P]
    lib.orc_adress_weight.argtypes = [f64, f64, f64, f64, f64]
    lib.orc_adress_weight.restype = f64
    lib.orc_angle_tables_combine.restype = None
    lib.orc_run_ext.restype = ctypes.c_int
    lib.orc_nthreads_default.argtypes = []
    lib.orc_nthreads_default.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def nthreads_default():
    return _load().orc_nthreads_default()


# ---------------------------------------------------------------- RNG
def philox32(counter, key):
    """One Philox4x32-10 block: counter (4 x u32), key (2 x u32) -> 4 x u32."""
    c = np.asarray(counter, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox(counter, key):
    """One Philox4x64-10 block: counter (4 x u64), key (2 x u64) -> 4 x u64."""
    c = np.asarray(counter, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gauss3(seed, stream, step, tag):
    """Three N(0,1) draws for (seed, stream, step, tag) by Box-Muller."""
    out = np.zeros(3, dtype=np.float64)
    _load().orc_gauss3(seed, stream, step, tag, _ptr(out))
    return out


# ---------------------------------------------------------------- potentials
def pair_params(eps=1.0, sigma=1.0, rc=2.5, shift=float("nan"), caprad=0.0):
    """One type-pair row: eps, sigma, rc, shift (NaN = auto), caprad (0 = none)."""
    return np.array([eps, sigma, rc, shift, caprad], dtype=np.float64)


def pair_eval(pp, r):
    """LJ energy u(r) and radial force magnitude f(r) (positive = repulsive)."""
    pp = _c(pp, np.float64)
    u = ctypes.c_double()
    f = ctypes.c_double()
    _load().orc_pair_eval(_ptr(pp), float(r), ctypes.byref(u), ctypes.byref(f))
    return u.value, f.value


def fene_eval(K, R0, r):
    u = ctypes.c_double()
    f = ctypes.c_double()
    st = _load().orc_fene_eval(K, R0, float(r), ctypes.byref(u), ctypes.byref(f))
    if st != OK:
        raise OracleError(st, "fene_eval")
    return u.value, f.value


def bend_eval(k, ra, rb, rc):
    """Cosine bending energy and forces on (a, centre b, c)."""
    ra, rb, rc = (_c(x, np.float64) for x in (ra, rb, rc))
    u = ctypes.c_double()
    Fa, Fb, Fc = (np.zeros(3) for _ in range(3))
    _load().orc_bend_eval(k, _ptr(ra), _ptr(rb), _ptr(rc), ctypes.byref(u), _ptr(Fa), _ptr(Fb), _ptr(Fc))
    return u.value, Fa, Fb, Fc


# ---------------------------------------------------------------- system-level
def pair_table(ntypes, rows):
    """rows: dict (ti, tj) -> pair_params row, symmetric; returns flat table."""
    t = np.zeros((ntypes, ntypes, 5), dtype=np.float64)
    for (a, b), row in rows.items():
        t[a, b] = row
        t[b, a] = row
    return t.reshape(-1)


def forces(pos, box, pp, ntypes=1, type=None, bonds=None, angles=None, fene_K=30.0,
           fene_R0=1.5, k_bend=0.0, use_cells=True, nthreads=0, want_fscale=False):
    """Forces F [N,3] and obs dict at positions pos [N,3] (FP64)."""
    pos = _c(pos, np.float64)
    n = pos.shape[0]
    box = _c(box, np.float64)
    pp = _c(pp, np.float64)
    type = _c(type, np.int32)
    bonds = _c(bonds, np.int32)
    angles = _c(angles, np.int32)
    nb = 0 if bonds is None else bonds.shape[0]
    na = 0 if angles is None else angles.shape[0]
    F = np.zeros((n, 3))
    obs = np.zeros(NOBS)
    fscale = np.zeros(n) if want_fscale else None
    st = _load().orc_forces(n, _ptr(pos), _ptr(type), ntypes, _ptr(pp), _ptr(box), nb, _ptr(bonds),
                            fene_K, fene_R0, na, _ptr(angles), k_bend, int(bool(use_cells)), nthreads,
                            _ptr(F), _ptr(obs), _ptr(fscale))
    if st != OK:
        raise OracleError(st, "forces")
    out = {"e_pair": obs[0], "e_bond": obs[1], "e_angle": obs[2], "virial": obs[3],
           "virial_tensor": obs[4:10].copy(), "virial_abs": obs[10]}
    if want_fscale:
        out["fscale"] = fscale
    return F, out


def neighbors(pos, box, rv, query=None, cap=512, nthreads=0):
    """Full Verlet-list sets by brute force: list of sorted int arrays."""
    pos = _c(pos, np.float64)
    box = _c(box, np.float64)
    n = pos.shape[0]
    q = None if query is None else _c(query, np.int64)
    nq = n if q is None else q.shape[0]
    count = np.zeros(nq, dtype=np.int32)
    idx = np.zeros((nq, cap), dtype=np.int32)
    st = _load().orc_neighbors(n, _ptr(pos), _ptr(box), float(rv), nq, _ptr(q), cap, _ptr(count),
                               _ptr(idx), nthreads)
    if st != OK:
        raise OracleError(st, "neighbors")
    return [np.sort(idx[k, :count[k]]) for k in range(nq)]


def neighbors_cells(pos, box, rv, cap=512, nthreads=0):
    """The same sets through the oracle's own linked cells (all particles)."""
    pos = _c(pos, np.float64)
    box = _c(box, np.float64)
    n = pos.shape[0]
    count = np.zeros(n, dtype=np.int32)
    idx = np.zeros((n, cap), dtype=np.int32)
    st = _load().orc_neighbors_cells(n, _ptr(pos), _ptr(box), float(rv), cap, _ptr(count), _ptr(idx),
                                     nthreads)
    if st != OK:
        raise OracleError(st, "neighbors_cells")
    return [np.sort(idx[k, :count[k]]) for k in range(n)]


NVE = 0
LANGEVIN = 1


def run(state, params, nsteps, use_cells=True, nthreads=0):
    """Advance ``state`` in place by nsteps of velocity Verlet (+ Langevin).

    state: dict with pos [N,3], vel [N,3], image [N,3] int32, step (int),
           vel_half (0/1), type [N] int32 or None.
    params: dict with box, pp, ntypes, mass_by_type, dt, integrator,
           temperature, gamma, seed, bonds, angles, fene_K, fene_R0, k_bend.
    Returns the per-step history [nsteps, NHIST].
    """
    pos = state["pos"]
    vel = state["vel"]
    img = state["image"]
    assert pos.dtype == np.float64 and pos.flags.c_contiguous
    assert vel.dtype == np.float64 and vel.flags.c_contiguous
    assert img.dtype == np.int32 and img.flags.c_contiguous
    n = pos.shape[0]
    type = _c(state.get("type"), np.int32)
    box = _c(params["box"], np.float64)
    pp = _c(params["pp"], np.float64)
    mass = _c(params["mass_by_type"], np.float64)
    bonds = _c(params.get("bonds"), np.int32)
    angles = _c(params.get("angles"), np.int32)
    nb = 0 if bonds is None else bonds.shape[0]
    na = 0 if angles is None else angles.shape[0]
    step = ctypes.c_int64(int(state["step"]))
    vh = ctypes.c_int32(int(state["vel_half"]))
    hist = np.zeros((nsteps, NHIST))
    st = _load().orc_run(n, _ptr(pos), _ptr(vel), _ptr(img), _ptr(type), _ptr(mass),
                         int(params.get("ntypes", 1)), _ptr(pp), _ptr(box), nb, _ptr(bonds),
                         float(params.get("fene_K", 30.0)), float(params.get("fene_R0", 1.5)), na,
                         _ptr(angles), float(params.get("k_bend", 0.0)), float(params["dt"]),
                         int(params["integrator"]), float(params.get("temperature", 0.0)),
                         float(params.get("gamma", 0.0)), int(params.get("seed", 0)),
                         ctypes.byref(step), ctypes.byref(vh), nsteps, int(bool(use_cells)),
                         nthreads, _ptr(hist))
    state["step"] = step.value
    state["vel_half"] = vh.value
    if st != OK:
        raise OracleError(st, "run")
    return hist


# ---------------------------------------------------------------- Lees-Edwards + DPD
DPD = 2


def dpd_theta(seed, step, ti, tj):
    """The symmetric pair noise theta_ij of the DPD thermostat."""
    return _load().orc_dpd_theta(seed, step, ti, tj)


class _Tabs(ctypes.Structure):
    _fields_ = [("npair", ctypes.c_int32), ("pair_rmin", ctypes.c_void_p), ("pair_u", ctypes.c_void_p),
                ("pair_f", ctypes.c_void_p), ("angle_kind", ctypes.c_int32), ("angle_K", ctypes.c_double),
                ("angle_phi0", ctypes.c_double), ("nang", ctypes.c_int32), ("angle_u", ctypes.c_void_p),
                ("angle_g", ctypes.c_void_p), ("adress", ctypes.c_int32), ("ad_x0", ctypes.c_double),
                ("ad_dat", ctypes.c_double), ("ad_dhy", ctypes.c_double), ("cg_rmin", ctypes.c_void_p),
                ("cg_rc", ctypes.c_void_p), ("cg_u", ctypes.c_void_p), ("cg_f", ctypes.c_void_p)]


ANGLE_COSINE = 0
ANGLE_COSINE_SQUARED = 1
ANGLE_TABULATED = 2


def tables(ntypes=1, pair=None, angle_kind=ANGLE_COSINE, angle_K=0.0, angle_phi0=0.0, angle_u=None, angle_g=None,
           adress=None, cg=None):
    """Tabulated interactions for forces_ext / run_ext.  pair: dict
    (ti, tj) -> (rmin, u[n], f[n]) on r_k = rmin + k (rc - rmin)/(n-1)
    (symmetric; every table the same n).  Angle kinds: ANGLE_COSINE (k_bend),
    ANGLE_COSINE_SQUARED (angle_K, angle_phi0), ANGLE_TABULATED (angle_u,
    angle_g = du/dphi on phi_k = k pi/(n-1)).  AdResS: adress = (x0, d_at,
    d_hy) and cg: dict (ti, tj) -> (rmin, rc, u[n], f[n]), the coarse-grained
    tables (the same n as the pair tables).  Returns an opaque object."""
    keep = []
    t = _Tabs()
    pair = pair or {}
    cg = cg or {}
    n = len(next(iter(pair.values()))[1]) if pair else (len(next(iter(cg.values()))[2]) if cg else 0)
    rmin = np.full(ntypes * ntypes, np.nan)
    U = np.zeros((ntypes * ntypes, max(n, 1)))
    Fv = np.zeros((ntypes * ntypes, max(n, 1)))
    for (a, b), (r0, u, f) in pair.items():
        for (x, y) in ((a, b), (b, a)):
            rmin[x * ntypes + y] = r0
            U[x * ntypes + y, :] = u
            Fv[x * ntypes + y, :] = f
    keep += [rmin, U, Fv]
    t.npair, t.pair_rmin, t.pair_u, t.pair_f = n, rmin.ctypes.data, U.ctypes.data, Fv.ctypes.data
    t.angle_kind, t.angle_K, t.angle_phi0 = angle_kind, float(angle_K), float(angle_phi0)
    if angle_u is not None:
        au, ag = np.ascontiguousarray(angle_u, dtype=np.float64), np.ascontiguousarray(angle_g, dtype=np.float64)
        keep += [au, ag]
        t.nang, t.angle_u, t.angle_g = au.size, au.ctypes.data, ag.ctypes.data
    cmin = np.full(ntypes * ntypes, np.nan)
    crc = np.zeros(ntypes * ntypes)
    CU = np.zeros((ntypes * ntypes, max(n, 1)))
    CF = np.zeros((ntypes * ntypes, max(n, 1)))
    for (a, b), (r0, rc, u, f) in cg.items():
        for (x, y) in ((a, b), (b, a)):
            cmin[x * ntypes + y], crc[x * ntypes + y] = r0, rc
            CU[x * ntypes + y, :] = u
            CF[x * ntypes + y, :] = f
    keep += [cmin, crc, CU, CF]
    t.cg_rmin, t.cg_rc, t.cg_u, t.cg_f = cmin.ctypes.data, crc.ctypes.data, CU.ctypes.data, CF.ctypes.data
    if adress is not None:
        t.adress = 1
        t.ad_x0, t.ad_dat, t.ad_dhy = (float(v) for v in adress)
    t._keep = keep
    return t


def adress_weight(x, Lx, x0, d_at, d_hy):
    """The AdResS weight w(x) of the oracle."""
    return _load().orc_adress_weight(float(x), float(Lx), float(x0), float(d_at), float(d_hy))


def angle_tables_combine(u_tables, g_tables, weights):
    """TabulatedSubEnsAngular: the table of the weighted sums of angle tables."""
    u = np.ascontiguousarray(u_tables, dtype=np.float64)
    g = np.ascontiguousarray(g_tables, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    uo, go = np.zeros(u.shape[1]), np.zeros(u.shape[1])
    _load().orc_angle_tables_combine(u.shape[0], u.shape[1], _ptr(u), _ptr(g), _ptr(w), _ptr(uo), _ptr(go))
    return uo, go


def forces_ext(pos, box, pp, vel=None, ntypes=1, type=None, bonds=None, angles=None, fene_K=30.0, fene_R0=1.5,
               k_bend=0.0, shear_rate=0.0, dpd_rc=0.0, dpd_gamma=0.0, kT=1.0, dt=0.005, seed=0, step=0,
               want_fscale=False, tabs=None):
    """Conservative forces F under the sheared boundaries at time step * dt
    and, when dpd_rc > 0, the DPD thermostat forces Fd at velocities vel.
    Returns (F, Fd or None, obs)."""
    pos = _c(pos, np.float64)
    n = pos.shape[0]
    vel = _c(vel, np.float64)
    box, pp = _c(box, np.float64), _c(pp, np.float64)
    type, bonds, angles = _c(type, np.int32), _c(bonds, np.int32), _c(angles, np.int32)
    nb = 0 if bonds is None else bonds.shape[0]
    na = 0 if angles is None else angles.shape[0]
    F = np.zeros((n, 3))
    Fd = np.zeros((n, 3)) if dpd_rc > 0 else None
    obs = np.zeros(NOBS)
    fscale = np.zeros(n) if want_fscale else None
    st = _load().orc_forces_ext(n, _ptr(pos), _ptr(vel), _ptr(type), ntypes, _ptr(pp), _ptr(box), nb, _ptr(bonds),
                                fene_K, fene_R0, na, _ptr(angles), k_bend, float(shear_rate), float(dpd_rc),
                                float(dpd_gamma), float(kT), float(dt), int(seed), int(step),
                                None if tabs is None else ctypes.byref(tabs), _ptr(F), _ptr(Fd), _ptr(obs),
                                _ptr(fscale))
    if st != OK:
        raise OracleError(st, "forces_ext")
    out = {"e_pair": obs[0], "e_bond": obs[1], "e_angle": obs[2], "virial": obs[3],
           "virial_tensor": obs[4:10].copy(), "virial_abs": obs[10]}
    if want_fscale:
        out["fscale"] = fscale
    return F, Fd, out


def neighbors_le(pos, box, rv, shear_rate=0.0, dt=1.0, step=0, cap=512):
    """Verlet-list sets under the sheared minimum image at time step * dt
    (brute force): list of sorted int arrays."""
    pos = _c(pos, np.float64)
    box = _c(box, np.float64)
    n = pos.shape[0]
    count = np.zeros(n, dtype=np.int32)
    idx = np.zeros((n, cap), dtype=np.int32)
    st = _load().orc_neighbors_le(n, _ptr(pos), _ptr(box), float(rv), float(shear_rate), float(dt), int(step), cap,
                                  _ptr(count), _ptr(idx))
    if st != OK:
        raise OracleError(st, "neighbors_le")
    return [np.sort(idx[k, :count[k]]) for k in range(n)]


def run_ext(state, params, nsteps):
    """``run`` with integrator DPD (2) and Lees-Edwards shear: params may hold
    shear_rate and dpd_rc (DPD takes gamma and temperature as its friction and
    kT).  Brute force over pairs."""
    pos, vel, img = state["pos"], state["vel"], state["image"]
    assert pos.dtype == np.float64 and pos.flags.c_contiguous
    assert vel.dtype == np.float64 and vel.flags.c_contiguous
    assert img.dtype == np.int32 and img.flags.c_contiguous
    n = pos.shape[0]
    type = _c(state.get("type"), np.int32)
    box = _c(params["box"], np.float64)
    pp = _c(params["pp"], np.float64)
    mass = _c(params["mass_by_type"], np.float64)
    bonds = _c(params.get("bonds"), np.int32)
    angles = _c(params.get("angles"), np.int32)
    nb = 0 if bonds is None else bonds.shape[0]
    na = 0 if angles is None else angles.shape[0]
    step = ctypes.c_int64(int(state["step"]))
    vh = ctypes.c_int32(int(state["vel_half"]))
    hist = np.zeros((nsteps, NHIST))
    st = _load().orc_run_ext(n, _ptr(pos), _ptr(vel), _ptr(img), _ptr(type), _ptr(mass),
                             int(params.get("ntypes", 1)), _ptr(pp), _ptr(box), nb, _ptr(bonds),
                             float(params.get("fene_K", 30.0)), float(params.get("fene_R0", 1.5)), na,
                             _ptr(angles), float(params.get("k_bend", 0.0)), float(params["dt"]),
                             int(params["integrator"]), float(params.get("temperature", 0.0)),
                             float(params.get("gamma", 0.0)), int(params.get("seed", 0)),
                             float(params.get("shear_rate", 0.0)), float(params.get("dpd_rc", 0.0)),
                             None if params.get("tabs") is None else ctypes.byref(params["tabs"]),
                             ctypes.byref(step), ctypes.byref(vh), nsteps, _ptr(hist))
    state["step"] = step.value
    state["vel_half"] = vh.value
    if st != OK:
        raise OracleError(st, "run_ext")
    return hist
