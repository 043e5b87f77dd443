"""Autotuner of the performance parameters of single systems and batches.

The parameters change only the cost of a step, never which pairs interact
(the list holds every pair inside the cutoff whatever the skin, cell size and
build; only the order of the FP32 sums follows the list order):

* the Verlet skin (longer lists against fewer rebuilds) -- batches only, since
  the single-system workloads fix their skin;
* the cell size and the list build, tried as the three forms that make sense:
  one wavefront per 64-particle tile on cells of side rc+skin, one particle
  per lane on the same cells, and one particle per lane on half-cutoff cells
  (fewer candidate pairs, more cells to walk);
* the tile of the force kernel: particles per block (64, 128, 256, 512) --
  single systems only; a batch packs its members in 256-particle tiles.

Results are cached in ``data/autotune_cache.json`` by

    (arch, kind, N bucket, density bucket, rc)

with N buckets of a factor 4 from 2,048 (2048-8191, 8192-32767, ...) and
density buckets 0.1 wide.  A batch is tuned group by group (members sharing a
key), each candidate timed on the whole batch with the graph-replayed step
(coordinate descent over the groups); a single system times each candidate on
itself.  Timing needs the GPU; looking up the cache does not.
"""
import json
import math
import os
import time

ARCH = "gfx950"
CACHE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "autotune_cache.json")
SKINS = (0.3, 0.4, 0.5)
# (cell factor, list build)
BUILDS = ((1, "tiles"), (1, "per_particle"), (2, "per_particle"))
BLOCKS = (64, 128, 256, 512)


# ---------------------------------------------------------------- keys
def n_bucket(n):
    """Lower edge of n's bucket: 2048 * 4^k (smaller systems share the first)."""
    k = max(0, int(math.floor(math.log(max(n, 1) / 2048.0, 4.0) + 1e-12)))
    return 2048 * 4 ** k


def rho_bucket(rho):
    return "%.1f" % (math.floor(rho * 10.0 + 1e-9) / 10.0)


def key_of(kind, n, rho, rc):
    return "%s|%s|n%d|rho%s|rc%.4f" % (ARCH, kind, n_bucket(n), rho_bucket(rho), rc)


def member_key(m):
    n = m["pos"].shape[0]
    box = m["box"]
    rho = n / float(box[0] * box[1] * box[2])
    return key_of(m.get("kind", "lj"), n, rho, m["pair"][(0, 0)][2])


# ---------------------------------------------------------------- cache
def load_cache(path=CACHE_PATH):
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def save_cache(cache, path=CACHE_PATH):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached_choice(members, path=CACHE_PATH):
    """Per-member parameters {member key: (skin, cell_factor, nl_build)} from
    the cache; keys without an entry keep the member's own skin and the
    library's automatic cells and build.  Returns (choice, description)."""
    cache = load_cache(path)
    choice, hit, miss = {}, 0, 0
    for m in members:
        k = member_key(m)
        if k in choice:
            continue
        e = cache.get(k)
        if e is None:
            choice[k] = (m["skin"], 0, "auto")
            miss += 1
        else:
            choice[k] = (e["skin"], e["cell_factor"], e["nl_build"])
            hit += 1
    return choice, "%d keys from the cache, %d without an entry (library defaults)" % (hit, miss)


def apply(members, choice):
    """Members with the parameters of their key (choice from tune() or
    cached_choice())."""
    out = []
    for m in members:
        k = member_key(m)
        m = dict(m)
        if k in choice:
            m["skin"], m["cell_factor"], m["nl_build"] = choice[k]
        out.append(m)
    return out


# ---------------------------------------------------------------- timing
def time_batch(members, steps, warmup=6):
    """Mean wall time per step (ms) of the batch, graph-replayed; the batch
    is closed afterwards."""
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


def tune(members, steps=40, skins=SKINS, builds=BUILDS, log=None, path=CACHE_PATH, write=True):
    """Tune a batch group by group.  Returns (choice {key: (skin, cell_factor,
    nl_build)}, table of trials); with write=True the winners go to the
    cache."""
    keys = sorted({member_key(m) for m in members})
    choice = {k: (next(m["skin"] for m in members if member_key(m) == k), 0, "auto") for k in keys}
    table = []
    for k in keys:
        best = None
        for skin in skins:
            for cf, build in builds:
                trial = dict(choice)
                trial[k] = (skin, cf, build)
                try:
                    ms = time_batch(apply(members, trial), steps)
                except Exception as e:   # e.g. a box too small for half-cutoff cells
                    if log:
                        log("autotune %s skin %.2f cf %d %s: skipped (%s)" % (k, skin, cf, build, e))
                    continue
                table.append({"key": k, "skin": skin, "cell_factor": cf, "nl_build": build, "ms_per_step": ms})
                if log:
                    log("autotune %s skin %.2f cf %d %s: %.3f ms/step" % (k, skin, cf, build, ms))
                if best is None or ms < best[0]:
                    best = (ms, skin, cf, build)
        if best is not None:
            choice[k] = best[1:]
    if write:
        cache = load_cache(path)
        for k, (skin, cf, build) in choice.items():
            if build != "auto":
                cache[k] = {"skin": skin, "cell_factor": cf, "nl_build": build, "source": "batch"}
        save_cache(cache, path)
    return choice, table


def _time_system(s, steps):
    s.step(6)
    s.stream.synchronize()
    t0 = time.perf_counter()
    s.step(steps)
    s.stream.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps


def tune_system(make, n, rho, rc, kind, steps=40, builds=BUILDS, blocks=BLOCKS, skins=None, log=None,
                path=CACHE_PATH, write=True):
    """Tune the cells, list build and force-kernel tile of one system, and
    its skin when ``skins`` is given (workloads whose skin is a performance
    choice, such as the surrogate's descriptor list).  ``make(cell_factor,
    flags)`` -- or ``make(cell_factor, flags, skin)`` with ``skins`` --
    returns a fresh System.  Skins, cells and builds are tried first at 256
    particles per block, then the block sizes on the winner (switched in
    place with md_set_params, which changes cost only).  Returns
    ((cell_factor, nl_build, block_size, skin), table)."""
    from .system import nl_build_flags
    table, best = [], None
    for skin_try in (skins or (None,)):
        for cf, build in builds:
            try:
                s = make(cf, nl_build_flags(build)) if skin_try is None else make(cf, nl_build_flags(build), skin_try)
            except Exception as e:
                if log:
                    log("autotune %s cf %d %s: skipped (%s)" % (kind, cf, build, e))
                continue
            ms = _time_system(s, steps)
            skin = s.cfg.skin
            s.close()
            table.append({"skin": skin, "cell_factor": cf, "nl_build": build, "block_size": 256, "ms_per_step": ms})
            if log:
                log("autotune %s skin %.2f cf %d %s block 256: %.3f ms/step" % (kind, skin, cf, build, ms))
            if best is None or ms < best[0]:
                best = (ms, cf, build, 256, skin)
    if best is None:
        raise RuntimeError("no candidate configuration ran")
    s = make(best[1], nl_build_flags(best[2])) if skins is None else make(best[1], nl_build_flags(best[2]), best[4])
    for bs in blocks:
        s.set_params(block_size=bs)
        ms = _time_system(s, steps)
        table.append({"skin": best[4], "cell_factor": best[1], "nl_build": best[2], "block_size": bs,
                      "ms_per_step": ms})
        if log:
            log("autotune %s cf %d %s block %d: %.3f ms/step" % (kind, best[1], best[2], bs, ms))
        if ms < best[0]:
            best = (ms, best[1], best[2], bs, best[4])
    s.close()
    if write:
        cache = load_cache(path)
        cache[key_of(kind, n, rho, rc)] = {"skin": best[4], "cell_factor": best[1], "nl_build": best[2],
                                           "block_size": best[3], "source": "single"}
        save_cache(cache, path)
    return best[1:], table


def cached_system_choice(kind, n, rho, rc, path=CACHE_PATH):
    """(cell_factor, nl_build, block_size, skin) of a single system from the
    cache, or None."""
    e = load_cache(path).get(key_of(kind, n, rho, rc))
    if e is None or e.get("source") != "single":
        return None
    return e["cell_factor"], e["nl_build"], e.get("block_size", 256), e["skin"]
