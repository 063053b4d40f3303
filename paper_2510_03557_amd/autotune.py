"""Launch-shape tuner of the short-range step.

Times the whole captured step on the workload itself and keeps the fastest
shape.  The search runs one dimension at a time from a starting shape
(coordinate descent), each dimension's best value kept for the next:

* leaf_max (k-d leaf size bound): 32, 48, 64;
* sub_sweep (wavefronts per leaf): 2 = one wavefront per sub-leaf, each
  staging its own candidates; 3 = four wavefronts per leaf sharing one
  staging of the leaf's candidates;
* tile (j-tile width of the split form): the candidate buffer of 64 x
  {pass default, 2, 8} records;
* grid_mult (persistent cost-ordered queue): 0 = one workgroup per item,
  or 32 x the CU count workgroups popping items.

Every shape gives the same results up to floating-point rounding order
(tested), so the tuner can only change speed.  Results are cached per
(workload signature, GPU architecture) in ~/.cache/crk_mi355x/tuning.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

START = dict(leaf_max=64, sub_sweep=2, tile=0, grid_mult=0, xcd_remap=1)
DIMENSIONS = (("leaf_max", (32, 48, 64)), ("sub_sweep", (2, 3)),
              ("tile", (0, 2, 8)), ("grid_mult", (0, 32)))
CACHE = os.path.join(os.path.expanduser("~"), ".cache", "crk_mi355x",
                     "tuning.json")


def signature(wl, precision: str) -> str:
    h = hashlib.sha256()
    h.update(precision.encode())
    for a in (wl.gas_off, wl.dm_off, wl.r_c, wl.eps):
        h.update(a.tobytes())
    h.update(wl.gas.x[:4096].tobytes())
    h.update(wl.gas.h[:4096].tobytes())
    return h.hexdigest()[:20]


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name)


def _load_cache() -> dict:
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(d: dict):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _name(c) -> str:
    return (f"L{c['leaf_max']}_s{c.get('sub_sweep', 2)}_t{c.get('tile', 0)}"
            f"_g{c.get('grid_mult', 0)}_x{c.get('xcd_remap', 1)}")


def _time(step, cand, reps):
    """Milliseconds per replay of the captured step at one shape."""
    import torch
    step.ctx.set_tuning(**cand)
    step.capture(integrate=False)
    step.replay()
    step.ctx.stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        step.replay()
    step.ctx.stream.synchronize()
    ms = (time.perf_counter() - t0) / reps * 1e3
    step.sync()
    return ms


def tune(step, candidates=None, reps: int = 5, use_cache: bool = True,
         log=None) -> dict:
    """Picks the fastest tuning for an existing ShortRangeStep (which is
    left set to it, eager, with no graph captured).  With ``candidates``
    (a list of tuning dicts) those are timed; otherwise the coordinate
    search over DIMENSIONS from START.  Returns
    {"tuning": {...}, "ms": {name: ms}, "cached": bool}."""
    key = signature(step.wl, step.ctx.precision) + "@" + _arch()
    cache = _load_cache() if use_cache else {}
    if key in cache:
        best = cache[key]["tuning"]
        if step.graph:
            step.drop_graph()
        step.ctx.set_tuning(**best)
        return {"tuning": best, "ms": cache[key]["ms"], "cached": True}
    results = {}

    def measure(cand):
        name = _name(cand)
        if name not in results:
            results[name] = _time(step, cand, reps)
            if log:
                log(f"[tune] {name}: {results[name]:.3f} ms")
        return results[name]

    if candidates:
        for cand in candidates:
            measure(cand)
        best_name = min(results, key=results.get)
        best = next(c for c in candidates if _name(c) == best_name)
    else:
        best = dict(START)
        for dim, values in DIMENSIONS:
            timed = []
            for v in values:
                cand = dict(best, **{dim: v})
                timed.append((measure(cand), v))
            best[dim] = min(timed)[1]
    # the last candidate's graph holds that candidate's launch shape: drop
    # it, so that the step is left eager at the chosen tuning
    step.drop_graph()
    step.ctx.set_tuning(**best)
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tuning": best, "ms": results}
        _store_cache(cache)
    return {"tuning": best, "ms": results, "cached": False}
