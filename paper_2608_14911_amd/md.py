"""ctypes binding of the C ABI in include/md.h (argument marshalling only).

Every function here has the name of the C entry point it calls and passes
plain pointers and sizes through; all arithmetic of the MD step runs in the
gfx950 kernels of libmdgpu.so.  Device pointers are given as integers (for
example ``tensor.data_ptr()``), host arrays as numpy arrays.  The library is
required: importing this module on a machine without the built library
raises at the first call instead of falling back to anything else.
"""
import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdgpu.so")

MD_OK = 0
MD_ERR_ARG = -1
MD_ERR_HIP = -2
MD_ERR_BOX_TOO_SMALL = -3
MD_ERR_NL_OVERFLOW = -4
MD_ERR_BOND_BROKEN = -5
MD_ERR_NONFINITE = -6
MD_ERR_STATE = -7
MD_ERR_WORKSPACE = -8
MD_ERR_TOPOLOGY = -9

MD_FLAG_NL_OVERFLOW = 0x1
MD_FLAG_BOND_BROKEN = 0x2
MD_FLAG_NONFINITE = 0x4

MD_NVE = 0
MD_LANGEVIN = 1
MD_DPD = 2
MD_ANGLE_COSINE = 0
MD_ANGLE_COSINE_SQUARED = 1
MD_ANGLE_TABULATED = 2
MD_FP64 = 0
MD_FP32 = 1
MD_MAX_TYPES = 4
MD_HISTORY_CAPACITY = 8192
MD_CFG_VIRIAL_TENSOR = 0x1
MD_CFG_NO_GRAPH = 0x2
MD_CFG_NL_PER_PARTICLE = 0x4
MD_CFG_NL_TILES = 0x8
MD_SUR_NBASIS = 32
MD_SUR_HIDDEN = 64
MD_SUR_NPARAM = 6337
MD_SUR_RCUT = 2.5
MD_SUR_WIDTH = 0.1
MD_SUR_MU0 = 0.8
MD_SUR_MU1 = 2.5
MD_SUR_VAR_FLOOR = 1e-6
MD_SUR_FP32 = 0
MD_SUR_BF16 = 1
MD_PAIR_PLAIN = 0
MD_PAIR_SURROGATE = 1

EXPORTED = ["md_workspace_bytes", "md_plan_config", "md_init", "md_set_params", "md_build_neighbors", "md_forces",
            "md_step", "md_observables", "md_history", "md_get_state", "md_set_state",
            "md_get_neighbors", "md_status_check", "md_timing_enable", "md_timing_read",
            "md_destroy", "md_status_string", "md_last_error", "md_sur_set", "md_sur_get",
            "md_set_pair_mode", "md_sur_descriptors", "md_sur_desc_stats", "md_sur_mlp_eval", "md_sur_pair_forces", "md_sur_loss_grad",
            "md_sur_adam", "md_batch_workspace_bytes", "md_batch_init", "md_batch_step",
            "md_batch_observables", "md_batch_get_state", "md_batch_destroy", "md_batch_last_error",
            "md_batch_timing_enable", "md_batch_timing_read", "md_init_static", "md_set_pair_table",
            "md_set_angle_table", "md_set_angle_subens", "md_set_cg_table"]


class md_pair_params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("sigma", ctypes.c_double), ("rc", ctypes.c_double),
                ("shift", ctypes.c_double), ("caprad", ctypes.c_double)]


class md_config(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_types", ctypes.c_int32),
                ("n_particles", ctypes.c_int64), ("box", ctypes.c_double * 3), ("dt", ctypes.c_double),
                ("skin", ctypes.c_double), ("integrator", ctypes.c_int32),
                ("force_precision", ctypes.c_int32), ("temperature", ctypes.c_double),
                ("gamma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("pair", md_pair_params * (MD_MAX_TYPES * MD_MAX_TYPES)), ("n_bonds", ctypes.c_int64),
                ("n_angles", ctypes.c_int64), ("fene_K", ctypes.c_double), ("fene_R0", ctypes.c_double),
                ("k_bend", ctypes.c_double), ("cell_factor", ctypes.c_int32),
                ("nl_capacity", ctypes.c_int32), ("block_size", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("list_cutoff", ctypes.c_double), ("surrogate", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("shear_rate", ctypes.c_double), ("dpd_rc", ctypes.c_double), ("table_points", ctypes.c_int32),
                ("angle_kind", ctypes.c_int32), ("angle_K", ctypes.c_double), ("angle_phi0", ctypes.c_double),
                ("adress", ctypes.c_int32), ("pad2_", ctypes.c_int32), ("adress_x0", ctypes.c_double),
                ("adress_d_at", ctypes.c_double), ("adress_d_hy", ctypes.c_double)]


class md_obs(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("e_pair", ctypes.c_double), ("e_bond", ctypes.c_double),
                ("e_angle", ctypes.c_double), ("e_kin", ctypes.c_double), ("e_total", ctypes.c_double),
                ("virial", ctypes.c_double), ("virial_tensor", ctypes.c_double * 6),
                ("pressure", ctypes.c_double), ("temperature", ctypes.c_double),
                ("n_rebuilds", ctypes.c_int64), ("status_flags", ctypes.c_uint32),
                ("nl_max_count", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["virial_tensor"] = np.array(list(self.virial_tensor))
        return d


class md_timing(ctypes.Structure):
    _fields_ = [("n_step_kernels", ctypes.c_int64), ("ms_step_kernels", ctypes.c_double),
                ("n_rebuild", ctypes.c_int64), ("ms_rebuild", ctypes.c_double),
                ("n_finalize", ctypes.c_int64), ("ms_finalize", ctypes.c_double),
                ("ms_bin_sort", ctypes.c_double)]


class md_plan(ctypes.Structure):
    _fields_ = [("cells", ctypes.c_int32 * 3), ("cell_factor", ctypes.c_int32), ("nl_capacity", ctypes.c_int32),
                ("nl_build", ctypes.c_int32), ("list_radius", ctypes.c_double)]


MD_NL_BUILD_PER_PARTICLE = 0
MD_NL_BUILD_TILES = 1


class MDError(RuntimeError):
    def __init__(self, code, fn, msg):
        super().__init__("%s -> %s: %s" % (fn, status_string(code), msg))
        self.code = code


_lib = None


def lib():
    """Load libmdgpu.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is not built; run __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950)" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "md_workspace_bytes": [ctypes.POINTER(md_config), ctypes.POINTER(SZ)],
        "md_plan_config": [ctypes.POINTER(md_config), ctypes.POINTER(md_plan)],
        "md_init": [ctypes.POINTER(md_config), P, P, P, P, P, P, P, SZ, P, ctypes.POINTER(P)],
        "md_init_static": [ctypes.POINTER(md_config), P, P, P, P, P, P, P, ctypes.POINTER(P)],
        "md_set_params": [P, ctypes.POINTER(md_config)],
        "md_set_pair_table": [P, I32, I32, P, P, I32, ctypes.c_double],
        "md_set_angle_table": [P, P, P, I32],
        "md_set_angle_subens": [P, I32, P, P, P, I32],
        "md_set_cg_table": [P, I32, I32, P, P, I32, ctypes.c_double, ctypes.c_double],
        "md_build_neighbors": [P],
        "md_forces": [P, P],
        "md_step": [P, I64],
        "md_observables": [P, ctypes.POINTER(md_obs)],
        "md_history": [P, P, I64, ctypes.POINTER(I64)],
        "md_get_state": [P, P, P, P, P, ctypes.POINTER(I64), ctypes.POINTER(I32)],
        "md_set_state": [P, P, P, P, P, I64, I32],
        "md_get_neighbors": [P, P, P, I32],
        "md_status_check": [P],
        "md_timing_enable": [P, I32],
        "md_timing_read": [P, ctypes.POINTER(md_timing)],
        "md_destroy": [P],
        "md_sur_set": [P, P, P, P, I32],
        "md_sur_get": [P, P],
        "md_set_pair_mode": [P, I32],
        "md_sur_descriptors": [P, P],
        "md_sur_desc_stats": [P, P, I32, P, P],
        "md_sur_mlp_eval": [P, P, I64, P, P],
        "md_sur_pair_forces": [P, P, P],
        "md_sur_loss_grad": [P, P, P, I32, P, ctypes.POINTER(ctypes.c_double)],
        "md_sur_adam": [P, I64, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    for name, args in {
        "md_batch_workspace_bytes": [P, I32, ctypes.POINTER(SZ)],
        "md_batch_init": [P, I32, P, P, P, P, P, P, SZ, P, ctypes.POINTER(P)],
        "md_batch_step": [P, I64],
        "md_batch_observables": [P, P],
        "md_batch_get_state": [P, I32, P, P, P, P, ctypes.POINTER(I64), ctypes.POINTER(I32)],
        "md_batch_destroy": [P],
        "md_batch_timing_enable": [P, I32],
        "md_batch_timing_read": [P, ctypes.POINTER(md_timing)],
    }.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    L.md_batch_last_error.argtypes = [P]
    L.md_batch_last_error.restype = ctypes.c_char_p
    L.md_status_string.argtypes = [ctypes.c_int32]
    L.md_status_string.restype = ctypes.c_char_p
    L.md_last_error.argtypes = [P]
    L.md_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def status_string(code):
    return lib().md_status_string(code).decode()


def md_last_error(h=None):
    return lib().md_last_error(h).decode()


def _check(code, fn, h=None):
    if code != MD_OK:
        raise MDError(code, fn, md_last_error(h))


def _p(x):
    if x is None:
        return None
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(ctypes.c_void_p)
    return ctypes.c_void_p(x.data_ptr())


# ------------------------------------------------------------------ config helper
def make_config(n, box, *, n_types=1, pair=None, dt=0.005, skin=0.3, integrator=MD_NVE,
                force_precision=MD_FP32, temperature=1.0, gamma=0.0, seed=0, n_bonds=0, n_angles=0,
                fene_K=30.0, fene_R0=1.5, k_bend=0.0, nl_capacity=0, flags=0, cell_factor=0,
                list_cutoff=0.0, surrogate=0, shear_rate=0.0, dpd_rc=0.0, table_points=0, angle_kind=0,
                angle_K=0.0, angle_phi0=0.0, adress=None, block_size=0):
    """Fill an md_config.  pair: dict (ti, tj) -> (eps, sigma, rc, shift, caprad)."""
    c = md_config()
    c.struct_size = ctypes.sizeof(md_config)
    c.n_types = n_types
    c.n_particles = int(n)
    for d in range(3):
        c.box[d] = float(box[d])
    c.dt, c.skin = float(dt), float(skin)
    c.integrator, c.force_precision = int(integrator), int(force_precision)
    c.temperature, c.gamma, c.seed = float(temperature), float(gamma), int(seed)
    pair = pair or {(0, 0): (1.0, 1.0, 2.5, math.nan, 0.0)}
    for (a, b), row in pair.items():
        for (x, y) in ((a, b), (b, a)):
            pp = c.pair[x * MD_MAX_TYPES + y]
            pp.eps, pp.sigma, pp.rc, pp.shift, pp.caprad = (float(v) for v in row)
    c.n_bonds, c.n_angles = int(n_bonds), int(n_angles)
    c.fene_K, c.fene_R0, c.k_bend = float(fene_K), float(fene_R0), float(k_bend)
    c.nl_capacity = int(nl_capacity)
    c.block_size = int(block_size)
    c.cell_factor = int(cell_factor)
    c.flags = int(flags)
    c.list_cutoff = float(list_cutoff)
    c.surrogate = int(surrogate)
    c.shear_rate = float(shear_rate)
    c.dpd_rc = float(dpd_rc)
    c.table_points = int(table_points)
    c.angle_kind = int(angle_kind)
    c.angle_K = float(angle_K)
    c.angle_phi0 = float(angle_phi0)
    if adress is not None:
        c.adress = 1
        c.adress_x0, c.adress_d_at, c.adress_d_hy = (float(v) for v in adress)
    return c


# ------------------------------------------------------------------ entry points
def md_workspace_bytes(cfg):
    n = ctypes.c_size_t()
    _check(lib().md_workspace_bytes(ctypes.byref(cfg), ctypes.byref(n)), "md_workspace_bytes")
    return n.value


def md_plan_config(cfg):
    """Cell grid and list build the configuration resolves to (dict)."""
    p = md_plan()
    _check(lib().md_plan_config(ctypes.byref(cfg), ctypes.byref(p)), "md_plan_config")
    return {"cells": list(p.cells), "cell_factor": p.cell_factor, "nl_capacity": p.nl_capacity,
            "nl_build": "tiles" if p.nl_build == MD_NL_BUILD_TILES else "per_particle",
            "list_radius": p.list_radius}


def md_init(cfg, pos, vel, type, mass_by_type, bonds, angles, workspace, ws_bytes, stream):
    h = ctypes.c_void_p()
    mass = np.ascontiguousarray(mass_by_type, dtype=np.float64)
    b = None if bonds is None else np.ascontiguousarray(bonds, dtype=np.int32)
    a = None if angles is None else np.ascontiguousarray(angles, dtype=np.int32)
    code = lib().md_init(ctypes.byref(cfg), _p(pos), _p(vel), _p(type), _p(mass), _p(b), _p(a),
                         _p(workspace), ws_bytes, _p(stream), ctypes.byref(h))
    _check(code, "md_init")
    return h


MD_STATIC_WORKSPACE_BYTES = 64 << 20


def md_init_static(cfg, pos, vel, type, mass_by_type, bonds, angles, stream):
    h = ctypes.c_void_p()
    mass = np.ascontiguousarray(mass_by_type, dtype=np.float64)
    b = None if bonds is None else np.ascontiguousarray(bonds, dtype=np.int32)
    a = None if angles is None else np.ascontiguousarray(angles, dtype=np.int32)
    code = lib().md_init_static(ctypes.byref(cfg), _p(pos), _p(vel), _p(type), _p(mass), _p(b), _p(a),
                                _p(stream), ctypes.byref(h))
    _check(code, "md_init_static")
    return h


def md_set_params(h, cfg):
    _check(lib().md_set_params(h, ctypes.byref(cfg)), "md_set_params", h)


def md_set_pair_table(h, ti, tj, u, f, rmin):
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert u.shape == f.shape
    _check(lib().md_set_pair_table(h, int(ti), int(tj), _p(u), _p(f), u.size, float(rmin)), "md_set_pair_table", h)


def md_set_cg_table(h, ti, tj, u, f, rmin, rc_cg):
    u = np.ascontiguousarray(u, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    assert u.shape == f.shape
    _check(lib().md_set_cg_table(h, int(ti), int(tj), _p(u), _p(f), u.size, float(rmin), float(rc_cg)),
           "md_set_cg_table", h)


def md_set_angle_table(h, u, dudphi):
    u = np.ascontiguousarray(u, dtype=np.float64)
    g = np.ascontiguousarray(dudphi, dtype=np.float64)
    assert u.shape == g.shape
    _check(lib().md_set_angle_table(h, _p(u), _p(g), u.size), "md_set_angle_table", h)


def md_set_angle_subens(h, u_tables, g_tables, weights):
    u = np.ascontiguousarray(u_tables, dtype=np.float64)
    g = np.ascontiguousarray(g_tables, dtype=np.float64)
    w = np.ascontiguousarray(weights, dtype=np.float64)
    assert u.shape == g.shape and u.shape[0] == w.size
    _check(lib().md_set_angle_subens(h, u.shape[0], _p(u), _p(g), _p(w), u.shape[1]), "md_set_angle_subens", h)


def md_build_neighbors(h):
    _check(lib().md_build_neighbors(h), "md_build_neighbors", h)


def md_forces(h, f_out):
    _check(lib().md_forces(h, _p(f_out)), "md_forces", h)


def md_step(h, nsteps):
    _check(lib().md_step(h, int(nsteps)), "md_step", h)


def md_observables(h, check=True):
    o = md_obs()
    code = lib().md_observables(h, ctypes.byref(o))
    if check:
        _check(code, "md_observables", h)
    return o.as_dict() if check else (code, o.as_dict())


def md_history(h, max_records=MD_HISTORY_CAPACITY):
    arr = (md_obs * max_records)()
    n = ctypes.c_int64()
    _check(lib().md_history(h, ctypes.cast(arr, ctypes.c_void_p), max_records, ctypes.byref(n)), "md_history", h)
    return [arr[k].as_dict() for k in range(n.value)]


def md_get_state(h, pos, vel, image=None, pos_build=None):
    step = ctypes.c_int64()
    vh = ctypes.c_int32()
    _check(lib().md_get_state(h, _p(pos), _p(vel), _p(image), _p(pos_build), ctypes.byref(step),
                              ctypes.byref(vh)), "md_get_state", h)
    return step.value, vh.value


def md_set_state(h, pos, vel, image, pos_build, step, vel_half):
    _check(lib().md_set_state(h, _p(pos), _p(vel), _p(image), _p(pos_build), int(step), int(vel_half)),
           "md_set_state", h)


def md_get_neighbors(h, count, idx, cap):
    _check(lib().md_get_neighbors(h, _p(count), _p(idx), int(cap)), "md_get_neighbors", h)


def md_status_check(h):
    return lib().md_status_check(h)


def md_timing_enable(h, enable):
    _check(lib().md_timing_enable(h, int(bool(enable))), "md_timing_enable", h)


def md_timing_read(h):
    t = md_timing()
    _check(lib().md_timing_read(h, ctypes.byref(t)), "md_timing_read", h)
    return {k: getattr(t, k) for k, _ in t._fields_}


def md_destroy(h):
    _check(lib().md_destroy(h), "md_destroy")


def md_sur_set(h, theta, g_mean, g_istd, precision):
    _check(lib().md_sur_set(h, _p(theta), _p(g_mean), _p(g_istd), int(precision)), "md_sur_set", h)


def md_sur_get(h, theta):
    _check(lib().md_sur_get(h, _p(theta)), "md_sur_get", h)


def md_set_pair_mode(h, mode):
    _check(lib().md_set_pair_mode(h, int(mode)), "md_set_pair_mode", h)


def md_sur_descriptors(h, G):
    _check(lib().md_sur_descriptors(h, _p(G)), "md_sur_descriptors", h)


def md_sur_desc_stats(h, frames, nf, g_mean, g_istd):
    _check(lib().md_sur_desc_stats(h, _p(frames), int(nf), _p(g_mean), _p(g_istd)), "md_sur_desc_stats", h)


def md_sur_mlp_eval(h, G, P, e, dedg):
    _check(lib().md_sur_mlp_eval(h, _p(G), int(P), _p(e), _p(dedg)), "md_sur_mlp_eval", h)


def md_sur_loss_grad(h, frames, f_ref, nf, grad=None, want_loss=True):
    loss = ctypes.c_double()
    _check(lib().md_sur_loss_grad(h, _p(frames), _p(f_ref), int(nf), _p(grad),
                                  ctypes.byref(loss) if want_loss else None), "md_sur_loss_grad", h)
    return loss.value if want_loss else None


def md_sur_adam(h, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().md_sur_adam(h, int(t), float(lr), float(beta1), float(beta2), float(eps)), "md_sur_adam", h)


def md_sur_pair_forces(h, dedg, f_out):
    _check(lib().md_sur_pair_forces(h, _p(dedg), _p(f_out)), "md_sur_pair_forces", h)


# ------------------------------------------------------------------ batches
def _bcheck(code, fn, b=None):
    if code != MD_OK:
        raise MDError(code, fn, lib().md_batch_last_error(b).decode())


def _ptr_array(ptrs):
    return (ctypes.c_void_p * len(ptrs))(*[None if p is None else int(p) for p in ptrs])


def md_batch_workspace_bytes(cfgs):
    arr = (md_config * len(cfgs))(*cfgs)
    n = ctypes.c_size_t()
    _bcheck(lib().md_batch_workspace_bytes(ctypes.cast(arr, ctypes.c_void_p), len(cfgs), ctypes.byref(n)),
            "md_batch_workspace_bytes")
    return n.value


def md_batch_init(cfgs, pos_ptrs, vel_ptrs, masses, bonds, angles, workspace, ws_bytes, stream):
    """masses / bonds / angles: lists of host numpy arrays (bonds / angles
    entries may be None)."""
    nsys = len(cfgs)
    arr = (md_config * nsys)(*cfgs)
    keep = []

    def host_list(xs, dtype):
        if xs is None:
            return None
        out = []
        for x in xs:
            if x is None:
                out.append(None)
            else:
                a = np.ascontiguousarray(x, dtype=dtype)
                keep.append(a)
                out.append(a.ctypes.data)
        return _ptr_array(out)

    m = host_list(masses, np.float64)
    bp = host_list(bonds, np.int32)
    ap = host_list(angles, np.int32)
    h = ctypes.c_void_p()
    code = lib().md_batch_init(ctypes.cast(arr, ctypes.c_void_p), nsys, _ptr_array(pos_ptrs), _ptr_array(vel_ptrs),
                               m, bp, ap, _p(workspace), ws_bytes, _p(stream), ctypes.byref(h))
    _bcheck(code, "md_batch_init")
    return h


def md_batch_step(b, nsteps):
    _bcheck(lib().md_batch_step(b, int(nsteps)), "md_batch_step", b)


def md_batch_observables(b, nsys, check=True):
    arr = (md_obs * nsys)()
    code = lib().md_batch_observables(b, ctypes.cast(arr, ctypes.c_void_p))
    if check:
        _bcheck(code, "md_batch_observables", b)
    return [arr[k].as_dict() for k in range(nsys)]


def md_batch_get_state(b, sys, pos, vel, image=None, pos_build=None):
    step = ctypes.c_int64()
    vh = ctypes.c_int32()
    _bcheck(lib().md_batch_get_state(b, int(sys), _p(pos), _p(vel), _p(image), _p(pos_build), ctypes.byref(step),
                                     ctypes.byref(vh)), "md_batch_get_state", b)
    return step.value, vh.value


def md_batch_destroy(b):
    _bcheck(lib().md_batch_destroy(b), "md_batch_destroy")


def md_batch_timing_enable(b, enable):
    _bcheck(lib().md_batch_timing_enable(b, int(bool(enable))), "md_batch_timing_enable", b)


def md_batch_timing_read(b):
    t = md_timing()
    _bcheck(lib().md_batch_timing_read(b, ctypes.byref(t)), "md_batch_timing_read", b)
    return {k: getattr(t, k) for k, _ in t._fields_}
