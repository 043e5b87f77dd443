"""Autotuner of a batch's performance parameters.

The parameters change only the cost of a step, never its result (the list
holds every pair inside the cutoff whatever the skin, cell size and build):
the Verlet skin (longer lists against fewer rebuilds), the cell size and the
list build, tried as the three forms that make sense: one wavefront per
64-particle tile on cells of side rc+skin, one particle per lane on the same
cells, and one particle per lane on half-cutoff cells (fewer candidate pairs,
more cells to walk).  Members are grouped by kind (LJ fluid, polymer melt);
one group at a time, every candidate is timed on the whole batch with the
graph-replayed step and the fastest is kept (coordinate descent).  The force
kernels' tile is 256 particles (one block), fixed by the kernels.
"""
import time

SKINS = {"lj": (0.3, 0.4, 0.5), "kg": (0.3, 0.4, 0.5)}
# (cell factor, list build)
BUILDS = ((1, "tiles"), (1, "per_particle"), (2, "per_particle"))


def _apply(members, choice):
    out = []
    for m in members:
        k = m.get("kind", "lj")
        m = dict(m)
        if k in choice:
            m["skin"], m["cell_factor"], m["nl_build"] = choice[k]
        out.append(m)
    return out


def time_batch(members, steps, warmup=6):
    """Mean wall time per step (ms) of the batch, graph-replayed, and the
    batch itself is closed afterwards."""
    from .system import Batch
    b = Batch(members)
    b.step(warmup)
    b.stream.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.stream.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    b.close()
    return ms


def tune(members, steps=40, log=None):
    """Returns (choice {kind: (skin, cell_factor, nl_build)}, table of trials)."""
    kinds = sorted({m.get("kind", "lj") for m in members})
    # start from each group's own skin and the library's automatic choice
    choice = {k: (next(m["skin"] for m in members if m.get("kind", "lj") == k), 0, "auto") for k in kinds}
    table = []
    for k in kinds:
        best = None
        for skin in SKINS.get(k, (0.3,)):
            for cf, build in BUILDS:
                trial = dict(choice)
                trial[k] = (skin, cf, build)
                try:
                    ms = time_batch(_apply(members, trial), steps)
                except Exception as e:   # e.g. a box too small for half-cutoff cells
                    if log:
                        log("autotune %s skin %.2f cf %d %s: skipped (%s)" % (k, skin, cf, build, e))
                    continue
                table.append({"kind": k, "skin": skin, "cell_factor": cf, "nl_build": build, "ms_per_step": ms})
                if log:
                    log("autotune %s skin %.2f cf %d %s: %.3f ms/step" % (k, skin, cf, build, ms))
                if best is None or ms < best[0]:
                    best = (ms, skin, cf, build)
        if best is not None:
            choice[k] = best[1:]
    return choice, table


def apply(members, choice):
    return _apply(members, choice)
