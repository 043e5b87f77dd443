"""Host-side tests of the C ABI (no GPU needed): the library loads, exports
every entry point include/md.h declares, its structs have the layout ctypes
assumes, and argument / geometry validation and workspace sizing behave as
documented.  Nothing here launches a kernel."""
import ctypes
import math
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2608_14911_amd import inputs, md

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "md.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:md_status|const char\*)\s+(md_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = md.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(md.EXPORTED) == set(names)


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text('''
#include <stdio.h>
#include <stddef.h>
#include "md.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(md_config), sizeof(md_obs), sizeof(md_timing), sizeof(md_pair_params));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(md_config, n_particles), offsetof(md_config, pair),
         offsetof(md_config, n_bonds), offsetof(md_config, flags), offsetof(md_obs, status_flags));
  printf("%zu %zu %d %d\\n", offsetof(md_config, list_cutoff), offsetof(md_config, surrogate),
         MD_SUR_NPARAM, MD_SUR_NBASIS);
  printf("%zu %zu %d %d\\n", sizeof(md_plan), offsetof(md_plan, list_radius), MD_CFG_NL_PER_PARTICLE,
         MD_CFG_NL_TILES);
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    c_sizes = list(map(int, out))
    py = [ctypes.sizeof(md.md_config), ctypes.sizeof(md.md_obs), ctypes.sizeof(md.md_timing),
          ctypes.sizeof(md.md_pair_params), md.md_config.n_particles.offset, md.md_config.pair.offset,
          md.md_config.n_bonds.offset, md.md_config.flags.offset, md.md_obs.status_flags.offset,
          md.md_config.list_cutoff.offset, md.md_config.surrogate.offset, md.MD_SUR_NPARAM, md.MD_SUR_NBASIS,
          ctypes.sizeof(md.md_plan), md.md_plan.list_radius.offset, md.MD_CFG_NL_PER_PARTICLE, md.MD_CFG_NL_TILES]
    assert c_sizes == py


def lj_cfg(n=4000, L=20.0, **kw):
    return md.make_config(n, [L, L, L], **kw)


def test_workspace_bytes_grows_with_size_and_capacity():
    a = md.md_workspace_bytes(lj_cfg(4000))
    b = md.md_workspace_bytes(lj_cfg(8000))
    c = md.md_workspace_bytes(lj_cfg(4000, nl_capacity=256))
    assert 0 < a < b and a < c
    # the Verlet list dominates: the automatic capacity at density 0.5 and
    # rv = 2.8 is 1.5 * 46 + 32 -> 104 slots, so 256 slots add 152 int32
    assert c - a == pytest.approx(4032 * (256 - 104) * 4, rel=0.01)
    kg = md.make_config(1000, [10.5567] * 3, pair={(0, 0): (1.0, 1.0, 2 ** (1 / 6), math.nan, 0.0)},
                        n_bonds=980, n_angles=960, skin=0.3)
    assert md.md_workspace_bytes(kg) > md.md_workspace_bytes(
        md.make_config(1000, [10.5567] * 3, pair={(0, 0): (1.0, 1.0, 2 ** (1 / 6), math.nan, 0.0)}, skin=0.3))


@pytest.mark.parametrize("mutate,code", [
    (lambda c: setattr(c, "struct_size", 8), md.MD_ERR_ARG),
    (lambda c: setattr(c, "n_types", 0), md.MD_ERR_ARG),
    (lambda c: setattr(c, "n_types", 5), md.MD_ERR_ARG),
    (lambda c: setattr(c, "n_particles", 0), md.MD_ERR_ARG),
    (lambda c: setattr(c, "n_particles", 1 << 28), md.MD_ERR_ARG),     # 32-bit record offsets
    (lambda c: setattr(c, "dt", 0.0), md.MD_ERR_ARG),
    (lambda c: setattr(c, "skin", -0.1), md.MD_ERR_ARG),
    (lambda c: setattr(c, "integrator", 7), md.MD_ERR_ARG),
    (lambda c: setattr(c, "force_precision", 3), md.MD_ERR_ARG),
    (lambda c: c.box.__setitem__(1, float("nan")), md.MD_ERR_ARG),
    (lambda c: setattr(c.pair[0], "sigma", 0.0), md.MD_ERR_ARG),
    (lambda c: setattr(c, "cell_factor", 3), md.MD_ERR_ARG),
    (lambda c: c.box.__setitem__(0, 7.0), md.MD_ERR_BOX_TOO_SMALL),     # 2 cells of 2.8
])
def test_invalid_configs_are_rejected(mutate, code):
    c = lj_cfg()
    mutate(c)
    with pytest.raises(md.MDError) as e:
        md.md_workspace_bytes(c)
    assert e.value.code == code
    assert md.md_last_error()


def test_asymmetric_pair_table_rejected():
    c = md.make_config(4000, [20.0] * 3, n_types=2,
                       pair={(0, 0): (1, 1, 2.5, math.nan, 0), (1, 1): (1, 1, 2.5, math.nan, 0),
                             (0, 1): (1, 1, 2.5, math.nan, 0)})
    md.md_workspace_bytes(c)
    c.pair[1].eps = 0.5                      # (0,1) != (1,0)
    with pytest.raises(md.MDError) as e:
        md.md_workspace_bytes(c)
    assert e.value.code == md.MD_ERR_ARG


def test_cell_factor_two_needs_five_cells():
    c = lj_cfg(L=12.0, cell_factor=2)        # 12 / 1.4 = 8 half-cells: fine
    md.md_workspace_bytes(c)
    c = lj_cfg(L=6.5, cell_factor=2)         # 6.5 / 1.4 = 4 half-cells < 5
    with pytest.raises(md.MDError) as e:
        md.md_workspace_bytes(c)
    assert e.value.code == md.MD_ERR_BOX_TOO_SMALL


def test_init_argument_errors_before_any_device_call():
    c = lj_cfg()
    n = ctypes.c_size_t()
    h = ctypes.c_void_p()
    lib = md.lib()
    assert lib.md_init(ctypes.byref(c), None, None, None, None, None, None, None, 0, None,
                       ctypes.byref(h)) == md.MD_ERR_ARG
    assert lib.md_init(ctypes.byref(c), None, None, None, None, None, None, None, 0, None, None) == md.MD_ERR_ARG
    assert lib.md_workspace_bytes(ctypes.byref(c), None) == md.MD_ERR_ARG
    mass = (ctypes.c_double * 1)(1.0)
    # a workspace that is too small is rejected before it is touched
    assert lib.md_init(ctypes.byref(c), ctypes.c_void_p(256), ctypes.c_void_p(256), None,
                       ctypes.cast(mass, ctypes.c_void_p), None, None, ctypes.c_void_p(256), 16, None,
                       ctypes.byref(h)) == md.MD_ERR_WORKSPACE
    # bonds declared but not given
    c2 = lj_cfg(n_bonds=10)
    assert lib.md_init(ctypes.byref(c2), ctypes.c_void_p(256), ctypes.c_void_p(256), None,
                       ctypes.cast(mass, ctypes.c_void_p), None, None, ctypes.c_void_p(256), 1 << 40, None,
                       ctypes.byref(h)) == md.MD_ERR_ARG
    # null handles
    for f in ("md_build_neighbors", "md_status_check", "md_destroy"):
        assert getattr(lib, f)(None) in (md.MD_ERR_ARG, md.MD_OK)
    assert lib.md_step(None, 1) == md.MD_ERR_ARG


def test_status_strings():
    for code in (md.MD_OK, md.MD_ERR_ARG, md.MD_ERR_HIP, md.MD_ERR_BOX_TOO_SMALL, md.MD_ERR_NL_OVERFLOW,
                 md.MD_ERR_BOND_BROKEN, md.MD_ERR_NONFINITE, md.MD_ERR_STATE, md.MD_ERR_WORKSPACE,
                 md.MD_ERR_TOPOLOGY):
        assert md.status_string(code).startswith("MD_")
    assert md.status_string(-99) == "MD_ERR_UNKNOWN"


def test_list_cutoff_and_surrogate_workspace():
    base = lj_cfg(4000, pair={(0, 0): (1.0, 1.0, 2 ** (1 / 6), math.nan, 0.0)}, skin=0.4)
    a = md.md_workspace_bytes(base)
    wide = lj_cfg(4000, pair={(0, 0): (1.0, 1.0, 2 ** (1 / 6), math.nan, 0.0)}, skin=0.4, list_cutoff=2.5)
    b = md.md_workspace_bytes(wide)
    sur = lj_cfg(4000, pair={(0, 0): (1.0, 1.0, 2 ** (1 / 6), math.nan, 0.0)}, skin=0.4, list_cutoff=2.5,
                 surrogate=1)
    c = md.md_workspace_bytes(sur)
    assert a < b < c
    # descriptor, input-gradient and sensitivity rows (3 x 128 B), two float4
    # per particle, and the fixed network buffers (< 8 MB)
    assert 4000 * (3 * 128 + 32) <= c - b < 4000 * (3 * 128 + 32) + 8 * 2 ** 20
    for bad in (-1.0, float("nan")):
        with pytest.raises(md.MDError):
            md.md_workspace_bytes(lj_cfg(4000, list_cutoff=bad))
    with pytest.raises(md.MDError):
        md.md_workspace_bytes(lj_cfg(4000, surrogate=2))


def test_surrogate_calls_reject_null_handle():
    lib = md.lib()
    assert lib.md_sur_set(None, None, None, None, 0) == md.MD_ERR_ARG
    assert lib.md_set_pair_mode(None, 1) == md.MD_ERR_ARG
    assert lib.md_sur_adam(None, 1, 1e-3, 0.9, 0.999, 1e-8) == md.MD_ERR_ARG
    assert lib.md_sur_loss_grad(None, None, None, 1, None, None) == md.MD_ERR_ARG


def test_batch_workspace_and_member_validation():
    a = lj_cfg(4000)
    b = md.make_config(1000, [10.5567] * 3, pair={(0, 0): (1.0, 1.0, 2 ** (1 / 6), math.nan, 0.0)},
                       n_bonds=980, skin=0.4)
    both = md.md_batch_workspace_bytes([a, b])
    # each member's workspace without its own cell arrays, plus shared cells and tables
    assert both > md.md_batch_workspace_bytes([a]) > 0
    assert both > md.md_workspace_bytes(b)
    bad = [lj_cfg(4000, force_precision=md.MD_FP64),
           lj_cfg(4000, pair={(0, 0): (1.0, 1.0, 2.5, math.nan, 0.9)}),
           md.make_config(4000, [20.0, 20.0, 21.0]),
           md.make_config(4000, [20.0] * 3, n_types=2,
                          pair={(0, 0): (1, 1, 2.5, math.nan, 0), (0, 1): (1, 1, 2.5, math.nan, 0),
                                (1, 1): (1, 1, 2.5, math.nan, 0)}),
           lj_cfg(4000, integrator=md.MD_DPD, dpd_rc=1.0),
           lj_cfg(4000, shear_rate=0.1),
           lj_cfg(4000, table_points=64),
           lj_cfg(4000, table_points=64, adress=(10.0, 2.0, 2.0)),
           lj_cfg(4000, angle_kind=md.MD_ANGLE_COSINE_SQUARED, angle_K=1.0, angle_phi0=2.0)]
    for c in bad:
        with pytest.raises(md.MDError):
            md.md_batch_workspace_bytes([a, c])
    with pytest.raises(md.MDError):
        md.md_batch_workspace_bytes([])


def test_batch_replica_sampler_matches_its_definition():
    from paper_2608_14911_amd import inputs
    reps = inputs.batch_replicas(256, seed=1003)
    ns = np.array([r["pos"].shape[0] for r in reps])
    assert len(reps) == 256 and sum(r["kind"] == "kg" for r in reps) == 128
    assert ns.min() >= 2048 // 2 and ns.max() <= 65536 + 200
    assert 4.0e6 < ns.sum() < 5.5e6
    for r in reps:
        L = r["box"][0]
        rho = r["pos"].shape[0] / L ** 3
        assert abs(rho - r["density"]) < 1e-9 * rho
        assert 0.70 <= r["density"] <= 0.90 and 0.7 <= r["temperature"] <= 1.2
        assert (r["pos"] >= 0).all() and (r["pos"] < L).all()
        if r["kind"] == "kg":
            assert 10 <= r["chain_len"] <= 200 and r["pos"].shape[0] % r["chain_len"] == 0
    # log-uniform sizes: the median is near the geometric mean of the range
    assert 6000 < np.median(ns) < 17000


def test_lattice_melt_bonds_join_lattice_neighbours():
    """The lattice melt's path visits every site once and each bond joins
    lattice neighbours: bond lengths stay within the jitter of the spacing,
    no two beads come closer than the spacing minus the jitter, and the
    density is the requested one."""
    for nc, cl in [(4, 50), (13, 77), (7, 300)]:
        w = inputs.lattice_melt(nc, cl, 0.85, jitter=0.05, seed=3)
        pos, box, b = w["pos"], w["box"], w["bonds"]
        n = nc * cl
        assert pos.shape == (n, 3) and abs(n / np.prod(box) - 0.85) < 1e-12
        m = int(np.ceil(n ** (1.0 / 3.0) - 1e-9))
        a = box[0] / m
        d = pos[b[:, 1]] - pos[b[:, 0]]
        d -= box * np.round(d / box)
        r = np.linalg.norm(d, axis=1)
        # each bead moves by at most 0.05 a per component
        assert r.min() >= a * (1 - 0.1) - 1e-12 and r.max() <= a * np.sqrt(1.1 ** 2 + 2 * 0.1 ** 2) + 1e-12
        # sites distinct: rounding back to the lattice gives n different sites
        sites = np.floor(pos / a).astype(np.int64) % m
        key = (sites[:, 2] * m + sites[:, 1]) * m + sites[:, 0]
        assert np.unique(key).size == n
        assert w["angles"].shape == (nc * (cl - 2), 3)


def test_plan_chooses_cells_and_list_build():
    """The automatic choices: dense fluids (>= 8 particles per cell of side
    rc+skin) take the tile list build, melts the per-particle build, both on
    cells of side rc+skin; half-cutoff cells only when fewer than 3 full
    cells fit per side; the flags force either build; a box of 3 list radii
    gets 3 cells."""
    lj = dict(pair={(0, 0): (1.0, 1.0, 2.5, float("nan"), 0.0)}, skin=0.3)
    wca = dict(pair={(0, 0): (1.0, 1.0, 2.0 ** (1 / 6), float("nan"), 0.0)}, skin=0.4)
    L = (1048576 / 0.8442) ** (1 / 3)
    p = md.md_plan_config(md.make_config(1048576, [L] * 3, **lj))
    assert p["nl_build"] == "tiles" and p["cell_factor"] == 1 and p["cells"] == [int(L / 2.8)] * 3
    assert abs(p["list_radius"] - 2.8) < 1e-12
    # the automatic capacity: 1.5 x the expected neighbours + 32, a multiple of 8
    expect = 0.8442 * 4.0 / 3.0 * math.pi * 2.8 ** 3
    assert p["nl_capacity"] == (math.ceil(1.5 * expect + 32) + 7) // 8 * 8
    L2 = (2000000 / 0.85) ** (1 / 3)
    p = md.md_plan_config(md.make_config(2000000, [L2] * 3, **wca))
    rv = 2.0 ** (1 / 6) + 0.4
    assert p["nl_build"] == "per_particle" and p["cell_factor"] == 1
    assert p["cells"] == [int(L2 / (rv * (1 + 1e-12)))] * 3
    p = md.md_plan_config(md.make_config(2000000, [L2] * 3, flags=md.MD_CFG_NL_TILES, **wca))
    assert p["nl_build"] == "tiles" and p["cell_factor"] == 1
    p = md.md_plan_config(md.make_config(2000000, [L2] * 3, cell_factor=2, **wca))
    assert p["nl_build"] == "per_particle" and p["cell_factor"] == 2
    assert p["cells"] == [int(L2 * 2 / (rv * (1 + 1e-12)))] * 3
    p = md.md_plan_config(md.make_config(1048576, [L] * 3, flags=md.MD_CFG_NL_PER_PARTICLE, **lj))
    assert p["nl_build"] == "per_particle" and p["cell_factor"] == 1
    p = md.md_plan_config(md.make_config(1048576, [L] * 3, cell_factor=2, **lj))
    assert p["nl_build"] == "per_particle"
    # a dense box of 3 list radii: 3 full cells per side and tiles
    p = md.md_plan_config(md.make_config(1000, [8.4 * 1.0000001] * 3, **lj))
    assert p["cells"] == [3, 3, 3] and p["cell_factor"] == 1 and p["nl_build"] == "tiles"
    # a sparse box of 4.3 list radii: 4 full cells per side, per particle
    p = md.md_plan_config(md.make_config(100, [12.0] * 3, **lj))
    assert p["cell_factor"] == 1 and p["nl_build"] == "per_particle" and p["cells"] == [4, 4, 4]
    # a box of 2.7 list radii holds 2 full cells but 5 half cells per side
    p = md.md_plan_config(md.make_config(20, [7.6] * 3, **lj))
    assert p["cell_factor"] == 2 and p["nl_build"] == "per_particle" and p["cells"] == [5, 5, 5]


def test_nl_capacity_rounds_up_to_a_multiple_of_8():
    """The step kernels stream a row in batches of 8 slots, up to the row
    length rounded up to 8.  A capacity that is not a multiple of 8 would let
    a long row read the first slots of another particle's row: the list
    layout puts slot k of particle i at (i // 64) * cap * 64 + k * 64 + i % 64,
    so slot cap of particle i is slot 0 of particle i + 64.  The library
    therefore rounds the capacity up."""
    lj = dict(pair={(0, 0): (1.0, 1.0, 2.5, float("nan"), 0.0)}, skin=0.3)
    for asked, got in ((78, 80), (80, 80), (1, 8), (81, 88), (4095, 4096), (4096, 4096)):
        p = md.md_plan_config(md.make_config(4000, [20.0] * 3, nl_capacity=asked, **lj))
        assert p["nl_capacity"] == got, (asked, p["nl_capacity"])

    def base(i, cap):
        return (i // 64) * cap * 64 + (i % 64)

    # the aliasing the rounding prevents, and that it is gone once rounded
    assert base(5, 78) + 78 * 64 == base(5 + 64, 78)
    for asked in range(1, 200):
        cap = (asked + 7) // 8 * 8
        for cnt in range(cap + 1):
            nslots = min((cnt + 7) // 8 * 8, cap)
            assert nslots <= cap
    # a workspace sized for the rounded capacity
    assert md.md_workspace_bytes(lj_cfg(4000, nl_capacity=78)) == md.md_workspace_bytes(lj_cfg(4000, nl_capacity=80))
