"""Launch-shape tuner of the short-range step.

Times the whole captured step for a small grid of (leaf_max, sweep form,
launch shape) choices on the workload itself and keeps the fastest.  Every choice gives
the same results up to floating-point rounding order (tested), so the tuner
can only change speed.  Results are cached per (workload signature, GPU
architecture) in ~/.cache/crk_mi355x/tuning.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

CANDIDATES = ([dict(leaf_max=L, sub_sweep=s) for L in (32, 48, 64)
               for s in (0, 2)]
              + [dict(leaf_max=64, sub_sweep=2, xcd_remap=0),
                 dict(leaf_max=128, sub_sweep=0),
                 dict(leaf_max=64, sub_sweep=0, grid_mult=16)])
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
    return (f"L{c['leaf_max']}_g{c.get('grid_mult', 0)}_x{c.get('xcd_remap', 0)}"
            f"_s{c.get('sub_sweep', 2)}")


def tune(step, candidates=None, reps: int = 5, use_cache: bool = True,
         log=None) -> dict:
    """Picks the fastest tuning for an existing ShortRangeStep (which is
    left set to it, with no graph captured).  Returns
    {"tuning": {...}, "ms": {...}, "cached": bool}."""
    import torch
    key = signature(step.wl, step.ctx.precision) + "@" + _arch()
    cache = _load_cache() if use_cache else {}
    if key in cache:
        best = cache[key]["tuning"]
        if step.graph:
            step.drop_graph()
        step.ctx.set_tuning(**best)
        return {"tuning": best, "ms": cache[key]["ms"], "cached": True}
    results = {}
    for cand in candidates or CANDIDATES:
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
        name = _name(cand)
        results[name] = ms
        if log:
            log(f"[tune] {name}: {ms:.3f} ms")
    best_name = min(results, key=results.get)
    best = next(c for c in (candidates or CANDIDATES) if _name(c) == best_name)
    # the last candidate's graph holds that candidate's launch shape: drop
    # it, so that the step is left eager at the chosen tuning
    step.drop_graph()
    step.ctx.set_tuning(**best)
    if use_cache:
        cache = _load_cache()
        cache[key] = {"tuning": best, "ms": results}
        _store_cache(cache)
    return {"tuning": best, "ms": results, "cached": False}
