#!/usr/bin/env python
"""Throughput of one full short-range step (build_tree, lists, density,
coefficients, hydro forces, gravity, integrate) on one MI355X.

Workload (default): the one-GPU share at its real shape, 448^3 dm + 448^3
gas particles (179,830,784), Zel'dovich displacements of a Gaussian random
field with P(k) ~ k^-1.5 (rms 1.0 grid spacing), ~64 hydro neighbours,
r_c = 3/448; synthetic, seeded.

value = particles / s of the float32 path (pair sums in float32 with
compensated accumulation, double moment solve and integration), replayed as
one HIP graph per step.  The plain float64 path (same kernels in double,
launched eagerly) is timed beside it and reported as fp64_plain; the
speedup is their ratio.  The roofline entry covers the pass kernel with
the largest average duration, timed with HIP events on the library's stream.
The CPU baseline is the FP64 oracle (C, OpenMP) on a bounded sample of the
same workload (a central cube with the halo its outputs depend on); the
float32 outputs at the cube's inner particles are compared with it, per
output (parity_vs_oracle).  A secondary workload (128^3 + 128^3, P(k) ~
k^-2) is measured after the headline together with the next rows: the
reconstructed viscosity, the hierarchical substep cycle, the long-range
mesh gravity and friends-of-friends groups.
Progress goes to stderr; stdout carries one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FLOP per in-range ordered pair of each pass kernel, counted from its
# arithmetic (FMA = 2, rsqrt/rcp = 1, compares and selects not counted).
# gravity: 33 for r < r_c/2, 39 beyond; 38 is the uniform-density mean.
FLOP_PER_PAIR = {"density": 20, "coefficients": 89, "hydro": 178,
                 "gravity": 38}
# with the reconstructed viscosity: the gradient pass (the corrected-kernel
# gradient and nine products per pair) and the hydro pass with the limiter
RECON_FLOP_PER_PAIR = {"velocity_gradient": 86, "hydro": 220}
PEAK_FP32_TFLOPS = 157.3          # MI355X FP32 vector, published (packed)
PASS_TYPES = {"density": "DensityPass", "coefficients": "CoeffPass",
              "hydro": "HydroPass", "gravity": "GravityPass"}


def kernel_name(p: str, tuning: dict) -> str:
    """The float32 kernel a pass launches under a tuning (as rocprofv3 names
    it, namespaces dropped)."""
    t = PASS_TYPES[p]
    # (the hydro pass is a template on the reconstruction and the
    # compatible-energy form; the step's plain form is <false, false>)
    t = t + "<float, false, false>" if p == "hydro" else t + "<float>"
    L = tuning.get("leaf_max", 64)
    if tuning.get("grid_mult", 0) > 0:
        b = 64 if L <= 64 else (128 if L <= 128 else 256)
        return f"pair_kernel_queue<float, {t}, {b}>"
    if L <= 64 and (tuning.get("walk_mask", 0) >> list(PASS_TYPES).index(p)) & 1:
        return f"pair_kernel<float, {t}, 64, 1>"
    if L <= 64 and tuning.get("sub_sweep", 2) == 2:
        return f"pair_kernel_split<float, {t} >"
    if L <= 64 and tuning.get("sub_sweep", 2) == 3:
        return f"pair_kernel_leaf<float, {t} >"
    if L <= 64 and tuning.get("sub_sweep", 2) == 1:
        return f"pair_kernel<float, {t}, 64, 2>"
    b = 64 if L <= 64 else (128 if L <= 128 else 256)
    return f"pair_kernel<float, {t}, {b}, 0>"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("passes.hip", "crk_internal.h"):
        with open(os.path.join(ROOT, "paper_2510_03557_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(pass_name: str, kname: str, workload: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the same workload, kernel and kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"{pass_name}_pmc_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    def bare(name):  # the trace may or may not print the return type
        name = (name or "").strip()
        return name[5:] if name.startswith("void ") else name

    if (d.get("source_hash") != source_hash()
            or bare(d.get("kernel_name")) != bare(kname)
            or d.get("workload") != workload):
        return None
    return d.get("hbm_bytes_per_launch")


def time_steps(fn, sync, steps, warmup):
    for _ in range(warmup):
        fn()
    sync()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    sync()
    return (time.perf_counter() - t0) / steps


def measure_cycle(wl, tuning, max_levels, cycles, ms_per_step, log):
    """Hierarchical time steps on the same workload.  Per particle, the step
    its criteria allow, tau_i = min(c_cfl h / cs (gas), sqrt(2 eta eps /
    |a|)), from the step's own accelerations; the interval dt is about four
    median steps (at most the time in which the fastest particle crosses
    r_c / 4), cut into 2^L substeps with L the smallest level count
    (at most max_levels) whose deepest step resolves the smallest tau_i;
    bins from crk_timestep_bins.  Then timed block kick-drift-kick cycles
    (tree built once per cycle, refitted every substep, passes over the
    active leaves only), each from the same starting state; the same cycle
    with the other grouping of the active particles and with the
    compatible energy update are timed after it."""
    import numpy as np
    import torch
    from paper_2510_03557_amd import binding
    from paper_2510_03557_amd.step import ShortRangeStep
    c_cfl, eta = 0.25, 0.025
    st = ShortRangeStep(wl, precision="fp32", tuning=tuning)
    st.run()
    out = st.outputs()
    eps = float(wl.eps[0])
    ag = np.linalg.norm(out["a_grav_gas"] + out["a_hydro"], axis=0)
    ad = np.linalg.norm(out["a_grav_dm"], axis=0)
    tau_g = np.minimum(c_cfl * np.asarray(wl.gas.h, np.float64)
                       / np.maximum(out["cs"], 1e-30),
                       np.sqrt(2 * eta * eps / np.maximum(ag, 1e-30)))
    tau_d = np.sqrt(2 * eta * eps / np.maximum(ad, 1e-30))
    tau = np.concatenate([tau_g, tau_d])
    tmed, tmin = float(np.median(tau)), float(np.min(tau))
    # the tree serves the whole interval: the fastest particle moves at most
    # r_c / 4 (well inside the chaining-mesh margin, so no rebuild is due)
    vmax = max(float(np.max(np.sqrt(wl.gas.vx.astype(np.float64) ** 2
                                    + wl.gas.vy.astype(np.float64) ** 2
                                    + wl.gas.vz.astype(np.float64) ** 2))),
               float(np.max(np.sqrt(wl.dm.vx.astype(np.float64) ** 2
                                    + wl.dm.vy.astype(np.float64) ** 2
                                    + wl.dm.vz.astype(np.float64) ** 2))))
    dt = min(4.0 * tmed, 0.25 * float(wl.r_c[0]) / max(vmax, 1e-30))
    def timed_cycles(s):
        """Every timed cycle starts from the state the step was made with
        (restored outside the timed region), so each one does the same work
        and none drifts further than the first."""
        snap = s.snapshot()
        s.substep_cycle(dt, levels)  # warm-up (sizes)
        s.sync()
        s.ctx.timing(True)
        sec = 0.0
        for _ in range(cycles):
            s.restore(snap)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.substep_cycle(dt, levels)
            torch.cuda.synchronize()
            s.ctx.stream.synchronize()
            sec += time.perf_counter() - t0
        pm, _, _ = s.ctx.pass_times()
        s.ctx.timing(False)
        s.sync()
        return sec / cycles, pm

    # where the chaining-mesh bins leave less margin than that, the refit
    # reports CRK_ESTALE: the interval is then halved (fresh state)
    for attempt in range(4):
        levels = int(min(max(np.ceil(np.log2(dt / tmin)), 1), max_levels))
        bg, bd = st.timestep_bins(dt, levels, c_cfl=c_cfl, eta=eta)
        log(f"[bench] substep cycle: {levels} levels, dt {dt:.3g} (median "
            f"tau {tmed:.3g}, min {tmin:.3g}), bins gas "
            f"{np.bincount(bg, minlength=levels + 1).tolist()} dm "
            f"{np.bincount(bd, minlength=levels + 1).tolist()}")
        try:
            sec, pass_ms = timed_cycles(st)
            break
        except binding.CrkError as e:
            if e.status != binding.CRK_ESTALE or attempt == 3:
                raise
            log("[bench] the tree went stale inside the interval: halving dt")
            st.close()
            st = ShortRangeStep(wl, precision="fp32", tuning=tuning)
            st.run()
            dt *= 0.5
    steps = int(np.sum(2 ** bg.astype(np.int64)) + np.sum(2 ** bd.astype(np.int64)))
    n = wl.n_total
    subsets = list(st.cycle_subsets)
    st.close()

    def variant(label, tuning_change=None, **kw):
        """The same cycle (same bins and dt) with one option changed."""
        log(f"[bench] substep cycle, {label}")
        v = ShortRangeStep(wl, precision="fp32",
                           tuning=dict(tuning, **(tuning_change or {})), **kw)
        v.run()
        v.set_bins(bg, bd)
        s2, pm = timed_cycles(v)
        v.close()
        return {"ms_per_cycle": s2 * 1e3,
                "pass_ms_per_cycle": {k: round(x / cycles, 3)
                                      for k, x in pm.items()}}

    groups = int(tuning.get("act_groups", 1))
    # the two fixed choices beside the default threshold
    others = {}
    for k, label in ((1, "active groups at every substep"),
                     (0, "active particles on the tree's sub-leaves")):
        if k != groups:
            others[f"act_groups_{k}"] = variant(label, {"act_groups": k})
    per_leaf = [p / max(lv, 1) for lv, p, _ in subsets]
    comp = variant("compatible energy update in every kick", compatible=True)
    flat = (2 ** levels) * ms_per_step if ms_per_step else None
    return {"levels": levels, "substeps": 2 ** levels, "dt": dt,
            "tau_median": tmed, "tau_min": tmin, "v_max": vmax,
            "bins_gas": np.bincount(bg, minlength=levels + 1).tolist(),
            "bins_dm": np.bincount(bd, minlength=levels + 1).tolist(),
            "cycles": cycles, "ms_per_cycle": sec * 1e3,
            "particle_steps": steps,
            "particle_steps_per_s": steps / sec,
            "evaluations_per_s": (n + steps) / sec,
            "pass_ms_per_cycle": {k: round(v / cycles, 3)
                                  for k, v in pass_ms.items()},
            "flat_deepest_ms": flat,
            "speedup_vs_flat": (flat / (sec * 1e3)) if flat else None,
            "act_groups": groups,
            "grouped_substeps": int(sum(g for _, _, g in subsets)),
            "active_per_leaf": ([round(float(q), 2) for q in
                                 np.percentile(per_leaf, [0, 50, 100])]
                                if per_leaf else None),
            **others,
            "compatible_energy": comp,
            "launch": "eager"}


def measure_recon(wl, tuning, steps, warmup, gather_pairs, hydro_pairs,
                  log):
    """The whole step with the viscosity on the limited midpoint
    reconstruction: the velocity-gradient pass added before the hydro
    forces, which then read the gradients of both sides.  Per-kernel HIP
    event times over eager steps, then graph replays of the step."""
    import torch
    from paper_2510_03557_amd.step import ShortRangeStep
    n = wl.n_total
    log("[bench] step with the reconstructed viscosity")
    st = ShortRangeStep(wl, precision="fp32", tuning=tuning, dt=1e-5,
                        recon=True)
    try:
        st.run(integrate=True)
        st.sync()
        st.ctx.timing(True)
        n_eager = max(steps // 4, 3)
        for _ in range(n_eager):
            st.run(integrate=True)
        pass_ms, kern_ms, launches = st.ctx.pass_times()
        st.ctx.timing(False)
        st.sync()
        st.capture(integrate=True)
        sec = time_steps(st.replay, lambda: (torch.cuda.synchronize(),
                                             st.ctx.stream.synchronize()),
                         steps, warmup)
        st.sync()
    finally:
        st.close()
    # the same step with the compatible energy update before the kick
    log("[bench] step with the reconstructed viscosity and the compatible "
        "energy update")
    st = ShortRangeStep(wl, precision="fp32", tuning=tuning, dt=1e-5,
                        recon=True, compatible=True)
    try:
        st.run(integrate=True)
        st.sync()
        st.ctx.timing(True)
        for _ in range(n_eager):
            st.run(integrate=True)
        cpass_ms, ckern_ms, claunch = st.ctx.pass_times()
        st.ctx.timing(False)
        st.sync()
        st.capture(integrate=True)
        csec = time_steps(st.replay, lambda: (torch.cuda.synchronize(),
                                              st.ctx.stream.synchronize()),
                          steps, warmup)
        st.sync()
    finally:
        st.close()
    kern = {}
    for p, pairs in (("velocity_gradient", gather_pairs),
                     ("hydro", hydro_pairs)):
        avg = kern_ms[p] / max(launches[p], 1)
        kern[p] = {"avg_ms": round(avg, 4), "pairs": pairs,
                   "flop_per_pair": RECON_FLOP_PER_PAIR[p],
                   "tflops": round(pairs * RECON_FLOP_PER_PAIR[p]
                                   / (avg * 1e-3) / 1e12, 3)}
    return {"value": n / sec, "ms_per_step": sec * 1e3, "launch": "hip_graph",
            "eta_crit": 0.8, "eta_fold": 0.2,
            "pass_ms": {k: round(v / n_eager, 4) for k, v in pass_ms.items()},
            "kernels": kern,
            "compatible_energy": {
                "value": n / csec, "ms_per_step": csec * 1e3,
                "launch": "hip_graph",
                "energy_pass_ms": round(cpass_ms["energy"] / n_eager, 4),
                "energy_kernel_ms": round(ckern_ms["energy"]
                                          / max(claunch["energy"], 1), 4),
                "energy_tflops": round(
                    hydro_pairs * RECON_FLOP_PER_PAIR["hydro"]
                    / (ckern_ms["energy"] / max(claunch["energy"], 1) * 1e-3)
                    / 1e12, 3)}}


def measure_pm(wl, reps, log):
    """Long-range mesh gravity of the whole box (crk_pm_gravity) on the mesh
    with r_c = 6 cells, float32; HIP-event time of one call on the
    library's stream, averaged over reps calls after a warm-up."""
    import numpy as np
    import torch
    from paper_2510_03557_amd.step import ShortRangeStep
    if wl.n_boxes != 1:
        return None
    st = ShortRangeStep(wl, precision="fp32")
    n_mesh = int(2 * np.ceil(3.0 / float(wl.r_c[0])))
    st.pm_gravity(n_mesh)  # warm-up: workspace and FFT plans
    st.ctx.timing(True)
    sec = time_steps(lambda: st.ctx.pm_gravity(
        n_mesh, float(wl.r_c[0]), st.ng, st.gx, st.gy, st.gz, st.gm, st.nd,
        st.dx, st.dy, st.dz, st.dm, st.pm_gas, st.pm_dm),
        lambda: (torch.cuda.synchronize(), st.ctx.stream.synchronize()),
        reps, 0)
    pass_ms, _, launches = st.ctx.pass_times()
    st.ctx.timing(False)
    st.close()
    n = wl.n_total
    log(f"[bench] mesh gravity: {n_mesh}^3 mesh, {sec * 1e3:.3f} ms")
    return {"n_mesh": n_mesh, "ms_per_call": sec * 1e3,
            "ms_per_call_events": pass_ms["gravity"] / max(reps, 1),
            "particles_per_s": n / sec, "reps": reps, "dtype": "f32",
            "deposit": "cic, double atomics", "fft": "hipfft r2c/c2r"}


def measure_fof(wl, tuning, reps, log):
    """Friends-of-friends groups of the whole workload (crk_fof) with the
    linking length 0.2 of the mean inter-particle spacing, over the step's
    tree and gravity lists (built once, outside the timed calls)."""
    import numpy as np
    import torch
    from paper_2510_03557_amd.step import ShortRangeStep
    st = ShortRangeStep(wl, precision="fp32", tuning=tuning)
    st.run()
    b = 0.2 * wl.n_total ** (-1.0 / 3.0)
    lg, ld = st.fof(b)  # warm-up
    with torch.cuda.stream(st.ctx.stream):
        tg = torch.zeros(max(st.ng, 1), dtype=torch.int32, device="cuda")
        td = torch.zeros(max(st.nd, 1), dtype=torch.int32, device="cuda")
    sec = time_steps(lambda: st.ctx.fof(st.tree, b, tg if st.ng else None,
                                        td if st.nd else None),
                     lambda: (torch.cuda.synchronize(),
                              st.ctx.stream.synchronize()), reps, 0)
    # group properties (count, mass, centre of mass) from those labels
    n = wl.n_total
    with torch.cuda.stream(st.ctx.stream):
        cnt = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
        mass = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
        cen = torch.zeros(3 * max(n, 1), dtype=torch.float64, device="cuda")

    def props():
        st.ctx.fof_properties(
            st.ng, st.nd, tg if st.ng else None, td if st.nd else None,
            (st.gx, st.gy, st.gz) if st.ng else None, st.gm if st.ng else None,
            (st.dx, st.dy, st.dz) if st.nd else None, st.dm if st.nd else None,
            cnt, mass, cen)
    psec = time_steps(props, lambda: (torch.cuda.synchronize(),
                                      st.ctx.stream.synchronize()), reps, 1)
    st.sync()
    st.close()
    lab = np.concatenate([lg, ld])
    sizes = np.bincount(lab)
    sizes = sizes[sizes > 0]
    log(f"[bench] fof: b {b:.4g}, {len(sizes)} groups, {sec * 1e3:.3f} ms")
    return {"linking_length": b, "ms_per_call": sec * 1e3,
            "particles_per_s": wl.n_total / sec,
            "properties_ms_per_call": psec * 1e3, "groups": int(len(sizes)),
            "groups_20_or_more": int(np.sum(sizes >= 20)),
            "largest_group": int(sizes.max()), "reps": reps}


def host_info() -> dict:
    """CPU model, logical CPUs and RAM of the host (Linux /proc)."""
    model, ram = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    ram = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "ram_gib": ram}


def measure_step(wl, workload, tuning, args, log, sample=None, tune=False):
    """The whole step on one workload: float32 kernel times (HIP events over
    eager steps), eager steps, graph replays (the value), the plain float64
    path, and the roofline of the dominant pass kernel.  With a sample
    (gas and dm indices), also the float32 outputs of the first step at
    those particles (before any integration)."""
    import torch
    from paper_2510_03557_amd.step import ShortRangeStep
    n = wl.n_total
    st = ShortRangeStep(wl, precision="fp32", tuning=tuning, dt=args.dt)
    tuned = None
    if tune:
        from paper_2510_03557_amd import autotune
        log(f"[bench] {workload}: tuning the launch shape")
        tuned = autotune.tune(st, log=log)
        tuning = dict(tuning, **tuned["tuning"])
    log(f"[bench] {workload}: fp32 path with {tuning}: first step, kernel timing")
    st.run(integrate=False)
    st.sync()
    got = st.outputs_at(*sample) if sample is not None else None
    pairs = st.ctx.count_pairs(st.tree)
    info = st.tree.info()
    st.run(integrate=True)
    st.sync()
    # per-kernel HIP-event timing over eager steps on the library stream
    st.ctx.timing(True)
    n_eager = max(args.steps // 4, 3)
    for _ in range(n_eager):
        st.run(integrate=True)
    pass_ms, kern_ms, launches = st.ctx.pass_times()
    st.ctx.timing(False)
    st.sync()
    # the same float32 step launched eagerly (no graph): separates the gain
    # of graph replay from that of the precision
    sec_eager = time_steps(lambda: st.run(integrate=True),
                           lambda: st.ctx.stream.synchronize(),
                           max(args.steps // 2, 3), 1)
    st.sync()
    log(f"[bench] {workload}: fp32 path: graph capture and timed replays")
    st.capture(integrate=True)
    sec = time_steps(st.replay, lambda: (torch.cuda.synchronize(),
                                         st.ctx.stream.synchronize()),
                     args.steps, args.warmup)
    st.sync()
    st.close()
    value = n / sec

    fp64 = None
    if not args.no_fp64:
        log(f"[bench] {workload}: fp64 plain path")
        st64 = ShortRangeStep(wl, precision="fp64", tuning=dict(leaf_max=64),
                              dt=args.dt)
        sec64 = time_steps(lambda: st64.run(integrate=True),
                           lambda: st64.ctx.stream.synchronize(),
                           args.fp64_steps, 1)
        st64.sync()
        fp64 = {"value": n / sec64, "ms_per_step": sec64 * 1e3,
                "dtype": "f64", "launch": "eager", "leaf_max": 64}
        st64.close()

    pair_of = {"density": pairs[0], "coefficients": pairs[0],
               "hydro": pairs[1], "gravity": pairs[2]}
    kern = {}
    for p in ("density", "coefficients", "hydro", "gravity"):
        if launches[p]:
            avg = kern_ms[p] / launches[p]
            flop = pair_of[p] * FLOP_PER_PAIR[p]
            kern[p] = {"avg_ms": avg, "pairs": pair_of[p],
                       "flop_per_pair": FLOP_PER_PAIR[p],
                       "tflops": flop / (avg * 1e-3) / 1e12}
    dom = max(kern, key=lambda k: kern[k]["avg_ms"])
    ach = kern[dom]["tflops"]
    traffic = measured_traffic(dom, kernel_name(dom, tuning), workload)
    roofline = {"bound": "alu", "achieved": round(ach, 3),
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": round(ach / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic, "kernel": kernel_name(dom, tuning),
                "avg_launch_ms": round(kern[dom]["avg_ms"], 4),
                "flop_per_unit": FLOP_PER_PAIR[dom],
                "units_per_launch": pair_of[dom],
                "unit_of_work": "in-range ordered pair",
                }
    res = {
        "value": value, "ms_per_step": sec * 1e3,
        "config": {"workload": workload, "description": wl.name,
                   "n_particles": n, "boxes": wl.n_boxes,
                   "leaf_max": tuning["leaf_max"],
                   "grid_mult": tuning.get("grid_mult", 0),
                   "xcd_remap": tuning.get("xcd_remap", 1),
                   "walk_mask": tuning.get("walk_mask", 0),
                   "sub_sweep": tuning.get("sub_sweep", 2),
                   "tree_lds": tuning.get("tree_lds", 1),
                   "tile": tuning.get("tile", 0), "launch": "hip_graph",
                   "leaves": info["n_leaves"],
                   "list_entries": {"gravity": info["grav_entries"],
                                    "hydro": info["hydro_entries"]}},
        "fp32_eager": {"value": n / sec_eager, "ms_per_step": sec_eager * 1e3,
                       "launch": "eager"},
        "fp64_plain": fp64,
        "speedup_vs_fp64": (value / fp64["value"]) if fp64 else None,
        "pairs": {"gather": pairs[0], "hydro": pairs[1], "gravity": pairs[2]},
        "swept_pairs": {"gather": pairs[3], "hydro": pairs[4],
                        "gravity": pairs[5]},
        "tuning": tuned,
        "pass_ms": {k: round(v / n_eager, 4) for k, v in pass_ms.items()},
        "kernels": kern,
        "roofline": roofline,
    }
    return res, got


# oracle sample: the particles of a central cube plus the halo their outputs
# depend on (hydro force neighbours, their gather neighbours, theirs: three
# hydro ranges, 6 h_max; gravity: r_c), sized for about 10-30 s of oracle
# time on the host's cores
CPU_SAMPLE_PARTICLES = 6.0e6
PARITY_KEYS = ("V", "rho_tilde", "rho", "A", "B", "gradA", "gradB", "P", "cs",
               "a_hydro", "dudt", "a_grav_gas", "a_grav_dm")


def oracle_sample(wl):
    """(sub, gas_idx, dm_idx, inner_gas, inner_dm, side, halo) of the
    oracle's sample of a single-box workload (workloads.sub_cube)."""
    import numpy as np
    from paper_2510_03557_amd import workloads
    h_max = float(np.max(wl.gas.h)) if wl.gas.n else 0.0
    halo = 1.001 * max(float(wl.r_c[0]), 6.0 * h_max)
    side = max((CPU_SAMPLE_PARTICLES / wl.n_total) ** (1.0 / 3.0) - 2 * halo,
               2 * halo)
    side = min(side, 0.49 - 2 * halo)
    return workloads.sub_cube(wl, side, halo) + (side, halo)


def parity_errors(got, ref, keys=PARITY_KEYS):
    """Per output: relative RMS (vectors and tensors by their Euclidean /
    Frobenius norms) and the worst particle's error |y_i - y_ref_i| /
    (|y_ref_i| + RMS_i |y_ref_i|) of the float32 GPU step against the FP64
    oracle."""
    import numpy as np
    out = {}
    for k in keys:
        g = np.asarray(got[k], np.float64)
        r = np.asarray(ref[k], np.float64)
        if k.startswith("a_"):
            g, r = np.moveaxis(g, -1, 0), np.moveaxis(r, -1, 0)
        g = g.reshape(g.shape[0], -1)
        r = r.reshape(r.shape[0], -1)
        if g.shape[0] == 0:
            continue
        d = np.sqrt(np.sum((g - r) ** 2, axis=1))
        rn = np.sqrt(np.sum(r * r, axis=1))
        scale = float(np.sqrt(np.mean(rn * rn)))
        out[k] = {"rel_rms": float(np.sqrt(np.sum(d * d)) / scale
                                   / np.sqrt(rn.shape[0])) if scale > 0
                  else float(np.sqrt(np.mean(d * d))),
                  "worst_particle": float(np.max(d / (rn + scale)))
                  if scale > 0 else float(np.max(d))}
    return out


def cpu_baseline_and_parity(sample, workload, got, log):
    """The FP64 oracle timed on a bounded sample of the benchmarked
    workload (a central cube with its dependency halo, every particle of it
    computed), and the per-output errors of the float32 GPU step (got: its
    outputs at the cube's inner particles) against the oracle there, where
    the sample holds every neighbourhood in full."""
    import numpy as np
    import oracle
    sub, gi, di, ig, idm, side, halo = sample
    oracle.build(force=False)
    log(f"[bench] cpu baseline: FP64 oracle on a cube of side {side:.4f} with "
        f"halo {halo:.4f} ({sub.n_total} particles)")
    t0 = time.perf_counter()
    ref = oracle.step(sub)
    tc = time.perf_counter() - t0
    cpu = {"value": sub.n_total / tc, "unit": "particles/s",
           "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"central cube of side {side:.4f} of {workload} with a "
                     f"{halo:.4f} halo (max(r_c, 6 h_max)): {sub.n_total} "
                     f"particles, every one computed (one step of the four "
                     f"passes, FP64 C oracle with OpenMP); rate = sample "
                     f"particles / oracle seconds",
           "seconds": round(tc, 2), "host": host_info()}
    gsel, dsel = np.nonzero(ig)[0], np.nonzero(idm)[0]
    inner = {}
    for k in PARITY_KEYS:
        if k == "a_grav_dm":
            inner[k] = ref[k][:, dsel]
        elif k.startswith("a_"):
            inner[k] = ref[k][:, gsel]
        else:
            inner[k] = ref[k][gsel]
    par = {"particles": {"gas": int(gsel.size), "dm": int(dsel.size)},
           "region": "inner cube of the oracle sample",
           "bound_rel_rms": 1e-5,
           "outputs": parity_errors(got, inner)}
    par["max_rel_rms"] = max(v["rel_rms"] for v in par["outputs"].values())
    return cpu, par


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="zeldovich448")
    ap.add_argument("--secondary", default="zeldovich128",
                    help="second workload, measured after the headline with "
                         "the next rows (reconstructed viscosity, substep "
                         "cycle, mesh gravity, friends-of-friends); 'none' "
                         "skips it")
    # defaults: the fastest shape the tuner found for these workloads on
    # MI355X (--tune re-runs the search)
    ap.add_argument("--leaf-max", type=int, default=64)
    ap.add_argument("--grid-mult", type=int, default=0)
    ap.add_argument("--xcd-remap", type=int, default=1)
    ap.add_argument("--walk-mask", type=int, default=0)
    ap.add_argument("--sub-sweep", type=int, default=2)
    ap.add_argument("--tree-lds", type=int, default=1)
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--act-groups", type=int, default=1)
    ap.add_argument("--tune", action="store_true",
                    help="tune the launch shape of the headline workload")
    ap.add_argument("--tuned-workload", default="uneven_boxes512",
                    help="workload measured after the others with the shape "
                         "the tuner picks for it ('none' skips it)")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--dt", type=float, default=1e-5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--substep-levels", type=int, default=8,
                    help="most levels of the hierarchical time-step cycle "
                         "timed on the secondary workload (0: none)")
    ap.add_argument("--cycles", type=int, default=3)
    ap.add_argument("--cycle-only", action="store_true",
                    help="time only the hierarchical time-step cycle and "
                         "print its JSON object")
    ap.add_argument("--pm-only", action="store_true",
                    help="time only the long-range mesh gravity and print "
                         "its JSON object")
    ap.add_argument("--no-pm", action="store_true")
    ap.add_argument("--no-fof", action="store_true")
    ap.add_argument("--fof-only", action="store_true",
                    help="time only the friends-of-friends groups and print "
                         "their JSON object")
    ap.add_argument("--no-recon", action="store_true",
                    help="skip the step with the reconstructed viscosity")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB three times "
                         "(reference kernel for scaling HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the short-range step runs on "
              "a single MI355X; spreading boxes or subdomains over several "
              "GPUs is described as a design, not implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        torch.cuda.set_device(0)
        src = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 2 ** 30, "copy_bytes_written":
                          2 ** 30, "launches": 3}), flush=True)
        return

    from paper_2510_03557_amd import workloads

    torch.cuda.set_device(0)
    tuning = dict(leaf_max=args.leaf_max, grid_mult=args.grid_mult,
                  xcd_remap=args.xcd_remap, walk_mask=args.walk_mask,
                  sub_sweep=args.sub_sweep, tree_lds=args.tree_lds,
                  tile=args.tile, act_groups=args.act_groups)

    if args.fof_only or args.pm_only or args.cycle_only:
        log(f"[bench] generating {args.workload}")
        wl = workloads.make(args.workload)
        n = wl.n_total
        if args.fof_only:
            out = measure_fof(wl, tuning, 5, log)
            half = n // 2
            out["clustered"] = measure_fof(
                workloads.random_uniform(half, n - half, 77, clustered=True,
                                         h_rule="global"), tuning, 5, log)
        elif args.pm_only:
            out = measure_pm(wl, 10, log)
        else:
            out = measure_cycle(wl, tuning, max(args.substep_levels, 1),
                                args.cycles, None, log)
        print(json.dumps(out), flush=True)
        return

    # ---------------- headline: the step on the benchmarked workload ---------
    log(f"[bench] generating {args.workload}")
    t0 = time.perf_counter()
    wl = workloads.make(args.workload)
    log(f"[bench] {wl.n_total} particles in {time.perf_counter() - t0:.1f} s")
    n = wl.n_total
    cpu = par = sample = None
    if not args.no_cpu_baseline and wl.n_boxes == 1:
        # the oracle's sample is fixed before the GPU step, whose outputs at
        # the sample's inner particles are kept for the parity entry
        sample = oracle_sample(wl)
    res, got = measure_step(
        wl, args.workload, tuning, args, log, tune=args.tune,
        sample=None if sample is None else (sample[1][sample[3]],
                                            sample[2][sample[4]]))
    if sample is not None:
        cpu, par = cpu_baseline_and_parity(sample, args.workload, got, log)
        del sample
    elif not args.no_cpu_baseline:
        # batches of boxes: the oracle on the whole workload
        import oracle
        oracle.build(force=False)
        t0 = time.perf_counter()
        oracle.step(wl)
        tc = time.perf_counter() - t0
        cpu = {"value": n / tc, "unit": "particles/s",
               "cores": oracle.num_threads(), "kind": "oracle",
               "sample": f"the whole {args.workload} workload ({n} particles)"
                         ", one step of the four passes, FP64 C oracle with "
                         "OpenMP", "seconds": round(tc, 2), "host": host_info()}

    out = {
        "metric": "particles/s per full short-range step (grav+CRKSPH), "
                  "FP32-batched vs FP64 plain",
        "value": res["value"], "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
    }
    out.update({k: v for k, v in res.items()
                if k not in ("value", "ms_per_step")})
    out["cpu_baseline"] = cpu
    out["parity_vs_oracle"] = par

    # ---------------- secondary workload and the next rows ------------------
    wl2 = wl
    name2 = args.workload
    if args.secondary not in ("none", "", args.workload):
        del wl
        log(f"[bench] generating {args.secondary}")
        wl2 = workloads.make(args.secondary)
        name2 = args.secondary
        sec_res, _ = measure_step(wl2, name2, tuning, args, log)
        out[name2] = sec_res
    sec_pairs = (out[name2] if name2 in out else res)["pairs"]
    nxt = out[name2] if name2 in out else out
    if not args.no_recon:
        nxt["recon_viscosity"] = measure_recon(
            wl2, tuning, args.steps, args.warmup, sec_pairs["gather"],
            sec_pairs["hydro"], log)
    if args.substep_levels > 0:
        nxt["substep_cycle"] = measure_cycle(
            wl2, tuning, args.substep_levels, args.cycles,
            (out[name2] if name2 in out else res)["ms_per_step"], log)
    if not args.no_pm:
        nxt["pm_long_range"] = measure_pm(wl2, 10, log)
    if not args.no_fof:
        fof = measure_fof(wl2, tuning, 5, log)
        # the Zel'dovich box is nearly uniform at this linking length (no
        # friends at all): a clustered set of the same size exercises the
        # unions as well
        log("[bench] fof on a clustered set of the same size")
        half = wl2.n_total // 2
        fof["clustered"] = measure_fof(
            workloads.random_uniform(half, wl2.n_total - half, 77,
                                     clustered=True, h_rule="global"),
            tuning, 5, log)
        nxt["fof"] = fof
    # ---------------- the batch of uneven boxes at the tuned shape ---------
    if args.tuned_workload not in ("none", ""):
        del wl2
        log(f"[bench] generating {args.tuned_workload}")
        wl3 = workloads.make(args.tuned_workload)
        res3, _ = measure_step(wl3, args.tuned_workload, tuning, args, log,
                               tune=True)
        out[args.tuned_workload] = res3
    out["context"] = ("paper: 46.6e9 particles/s on 9,000 Frontier nodes for "
                      "the whole solver per PM step (not like-for-like)")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
