"""Autotuner of a batch's performance parameters.

The parameters change only the cost of a step, never its result (the list
holds every pair inside the cutoff whatever the skin and cell size): the
Verlet skin (longer lists against fewer rebuilds) and the cell factor (cells
of side rv or rv / 2: fewer candidate pairs per list build against more cells
to scan).  Members are grouped by kind (LJ fluid, polymer melt); one group at
a time, every candidate is timed on the whole batch with HIP events and the
fastest is kept (coordinate descent).  The tile of the batched kernels is 256
particles (one block), fixed by the kernels.
"""
import time

SKINS = {"lj": (0.3, 0.4, 0.5), "kg": (0.3, 0.4, 0.5)}
CELL_FACTORS = (1, 2)


def _apply(members, choice):
    out = []
    for m in members:
        k = m.get("kind", "lj")
        m = dict(m)
        if k in choice:
            m["skin"], m["cell_factor"] = choice[k]
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
    """Returns (choice {kind: (skin, cell_factor)}, table of trials)."""
    kinds = sorted({m.get("kind", "lj") for m in members})
    # start from each group's own skin and half-cutoff cells
    choice = {k: (next(m["skin"] for m in members if m.get("kind", "lj") == k), 2) for k in kinds}
    table = []
    for k in kinds:
        best = None
        for skin in SKINS.get(k, (0.3,)):
            for cf in CELL_FACTORS:
                trial = dict(choice)
                trial[k] = (skin, cf)
                try:
                    ms = time_batch(_apply(members, trial), steps)
                except Exception as e:   # e.g. a box too small for half-cutoff cells
                    if log:
                        log("autotune %s skin %.2f cf %d: skipped (%s)" % (k, skin, cf, e))
                    continue
                table.append({"kind": k, "skin": skin, "cell_factor": cf, "ms_per_step": ms})
                if log:
                    log("autotune %s skin %.2f cf %d: %.3f ms/step" % (k, skin, cf, ms))
                if best is None or ms < best[0]:
                    best = (ms, skin, cf)
        if best is not None:
            choice[k] = (best[1], best[2])
    return choice, table


def apply(members, choice):
    return _apply(members, choice)
