"""md_init_static, the allocation-free variant of md_init, through the C ABI.

Its handle takes the workspace from the library's static per-GPU array
instead of a caller buffer.  Everything after init runs the same kernels on
the same workspace layout, so trajectories must equal md_init's bit for bit.
Two handles are created in a row on the same array, the second for a smaller
system (a bonded melt after an LJ fluid), so the second run starts from the
first one's leftover contents.
"""
import numpy as np
import pytest

from gpu_helpers import banner
from kg_fixture import kg1k_state
from paper_2608_14911_amd import inputs, md
from paper_2608_14911_amd.system import from_workload

pytestmark = pytest.mark.gpu


def _run_static(w, nsteps, precision):
    import torch
    ref = from_workload(w, precision=precision)   # md_init with a torch workspace: the configuration
    cfg = ref.cfg
    ref.close()
    dev = torch.device("cuda")
    pos = torch.as_tensor(np.ascontiguousarray(w["pos"]), device=dev)
    vel = torch.as_tensor(np.ascontiguousarray(w["vel"]), device=dev)
    stream = torch.cuda.current_stream()
    h = md.md_init_static(cfg, pos.data_ptr(), vel.data_ptr(), None, np.array([1.0]), w.get("bonds"),
                          w.get("angles"), stream.cuda_stream)
    try:
        # a second handle on the same device's array is refused while h lives
        with pytest.raises(md.MDError) as e:
            md.md_init_static(cfg, pos.data_ptr(), vel.data_ptr(), None, np.array([1.0]), w.get("bonds"),
                              w.get("angles"), stream.cuda_stream)
        assert e.value.code == md.MD_ERR_STATE
        md.md_step(h, nsteps)
        out = {k: torch.zeros((pos.shape[0], 3), dtype=t, device=dev)
               for k, t in (("pos", torch.float64), ("vel", torch.float64), ("image", torch.int32))}
        step, _ = md.md_get_state(h, out["pos"].data_ptr(), out["vel"].data_ptr(), out["image"].data_ptr())
        obs = md.md_observables(h)
        stream.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}, step, obs
    finally:
        md.md_destroy(h)


def _run_plain(w, nsteps, precision):
    s = from_workload(w, precision=precision)
    s.step(nsteps)
    st = s.get_state()
    obs = s.observables()
    s.close()
    return st, obs


@pytest.mark.parametrize("order", ["lj_then_kg"])
def test_init_static_matches_init_twice(order):
    cases = [("LJ fluid 4000, FP32", inputs.workload_lj(ncell=10, seed=41), 60, "fp32"),
             ("KG melt 1000 (bending), FP64", kg1k_state(1.5), 60, "fp64")]
    assert cases[1][1]["pos"].shape[0] < cases[0][1]["pos"].shape[0]
    for name, w, nsteps, prec in cases:
        banner("md_init_static vs md_init: %s, %d steps" % (name, nsteps))
        got, step, obs = _run_static(w, nsteps, prec)
        ref, obs_ref = _run_plain(w, nsteps, prec)
        assert step == nsteps == ref["step"]
        for k in ("pos", "vel", "image"):
            assert np.array_equal(got[k], ref[k]), (name, k)
        for k in ("e_pair", "e_bond", "e_angle", "e_kin", "virial", "n_rebuilds"):
            assert obs[k] == obs_ref[k], (name, k)
        assert obs["n_rebuilds"] >= 2


def test_init_static_rejects_a_system_beyond_the_array():
    banner("md_init_static size limit")
    import torch
    L = (1048576 / 0.8442) ** (1 / 3)
    cfg = md.make_config(1048576, [L] * 3)
    assert md.md_workspace_bytes(cfg) > md.MD_STATIC_WORKSPACE_BYTES
    d = torch.zeros((8, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(md.MDError) as e:
        md.md_init_static(cfg, d.data_ptr(), d.data_ptr(), None, np.array([1.0]), None, None,
                          torch.cuda.current_stream().cuda_stream)
    assert e.value.code == md.MD_ERR_WORKSPACE and "static workspace" in str(e.value)
