"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerance: relative RMS <= 1e-5 per output for the float32 path (the bound
the short-range step is specified to), 1e-10 for the float64 path (only
summation order differs).  rel_rms(y) = sqrt(sum |y - y_ref|^2 / sum
|y_ref|^2) with vectors and tensors compared by their Euclidean/Frobenius
norms.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_03557_amd import workloads as W  # noqa: E402

FP32_TOL = 1e-5
FP64_TOL = 1e-10
KEYS = ("V", "rho_tilde", "A", "B", "gradA", "gradB", "rho", "P", "cs",
        "a_hydro", "dudt", "a_grav_gas", "a_grav_dm")


from parity_util import (PER_PARTICLE_FP32, PER_PARTICLE_FP64,  # noqa: E402
                         degenerate_disagreements, rel_rms, worst_particle)


def compare(got, ref, tol, keys=KEYS, sel=None, per_particle=None):
    """Relative RMS per output within tol, the worst particle of every
    output within the per-particle bound (by default the one of the
    precision that tol belongs to), and no particle on a different
    coefficient branch than the oracle."""
    if per_particle is None:
        per_particle = PER_PARTICLE_FP64 if tol < 1e-8 else PER_PARTICLE_FP32
    errs, worst = {}, {}
    for k in keys:
        g, r = got[k], ref[k]
        if sel is not None:
            g = g[..., sel] if k.startswith("a_") else g[sel]
        errs[k] = rel_rms(g, r)
        worst[k] = worst_particle(k, g, r)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    badw = {k: v for k, v in worst.items() if not v[0] <= per_particle}
    flips = degenerate_disagreements(got, ref, sel) if "B" in keys else 0
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    print("worst particle:", {k: f"{v[0]:.2e}@{v[1]}" for k, v in worst.items()},
          "branch flips:", flips, flush=True)
    assert not bad, bad
    assert not badw, badw
    assert flips == 0, flips
    return errs


@pytest.fixture(scope="module")
def step_cls():
    from paper_2510_03557_amd.step import ShortRangeStep
    assert torch.cuda.is_available()
    return ShortRangeStep


def run(step_cls, wl, precision="fp32", tuning=None):
    st = step_cls(wl, precision=precision, tuning=tuning)
    st.run()
    out = st.outputs()
    return st, out


# ---------------------------------------------------------------------------
# small cases, whole chain
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,ng,nd", [(101, 3000, 2500), (102, 777, 1301),
                                        (103, 4096, 0)])
def test_small_fp64_matches_oracle(orc, step_cls, seed, ng, nd):
    print(f"case random_uniform({ng},{nd},{seed}) fp64", flush=True)
    wl = W.random_uniform(ng, nd, seed, n_ngb=48.0, h_spread=0.15)
    st, got = run(step_cls, wl, "fp64")
    ref = orc.step(wl)
    keys = KEYS if nd else KEYS[:-1]
    compare(got, ref, FP64_TOL, keys)
    st.close()


@pytest.mark.parametrize("seed,ng,nd,clustered", [
    (201, 3000, 2500, False), (202, 5000, 3000, True), (203, 1500, 4000, False)])
def test_small_fp32_matches_oracle(orc, step_cls, seed, ng, nd, clustered):
    print(f"case random_uniform({ng},{nd},{seed},clustered={clustered}) fp32",
          flush=True)
    wl = W.random_uniform(ng, nd, seed, n_ngb=48.0, h_spread=0.15,
                          clustered=clustered)
    st, got = run(step_cls, wl, "fp32")
    ref = orc.step(wl)
    compare(got, ref, FP32_TOL)
    st.close()


def test_dm_only_box(orc, step_cls):
    print("case dm only", flush=True)
    wl = W.random_uniform(0, 3000, 301)
    st, got = run(step_cls, wl, "fp32")
    ref = orc.step(wl)
    compare(got, ref, FP32_TOL, ("a_grav_dm",))
    st.close()


# ---------------------------------------------------------------------------
# each pass fed with the oracle's own inputs (isolates the pass)
# ---------------------------------------------------------------------------

def test_passes_with_oracle_inputs_fp32(orc, step_cls):
    print("case per-pass random_uniform(4000,3000,401) fp32", flush=True)
    wl = W.random_uniform(4000, 3000, 401, n_ngb=48.0, h_spread=0.15)
    ref = orc.step(wl)
    st = step_cls(wl, precision="fp32")
    ng = wl.gas.n
    # oracle intermediates rounded to float32 feed both sides
    V32 = ref["V"].astype(np.float32)
    g = wl.gas
    coef = orc.coefficients(g.x, g.y, g.z, g.h, g.m, V32.astype(np.float64),
                            g.u)
    st.set_inputs(V=V32)
    st.run(passes=("coefficients",))
    got = st.outputs()
    compare(got, coef, FP32_TOL, ("A", "B", "gradA", "gradB", "rho", "P", "cs"))
    c32 = {k: np.asarray(coef[k], np.float32) for k in
           ("A", "B", "gradA", "gradB", "rho", "P", "cs")}
    st.set_inputs(A=c32["A"], B=c32["B"].T.ravel(), gA=c32["gradA"].T.ravel(),
                  gB=c32["gradB"].transpose(1, 2, 0).ravel(), rho=c32["rho"],
                  P=c32["P"], cs=c32["cs"])
    st.run(passes=("hydro",))
    got = st.outputs()
    c64 = {k: v.astype(np.float64) for k, v in c32.items()}
    ax, ay, az, du = orc.hydro(g.x, g.y, g.z, g.vx, g.vy, g.vz, g.h, g.m,
                               V32, c64["rho"], c64["P"], c64["cs"], c64["A"],
                               c64["B"], c64["gradA"], c64["gradB"])
    compare(got, {"a_hydro": np.stack([ax, ay, az]), "dudt": du}, FP32_TOL,
            ("a_hydro", "dudt"))
    assert ng == got["V"].shape[0]
    st.close()


# ---------------------------------------------------------------------------
# the benchmark configurations
# ---------------------------------------------------------------------------

def test_lattice32_fp64_and_fp32(orc, step_cls):
    print("case lattice32 (65,536 particles)", flush=True)
    wl = W.make("lattice32")
    ref = orc.step(wl)
    st, got = run(step_cls, wl, "fp64")
    compare(got, ref, FP64_TOL)
    st.close()
    st, got = run(step_cls, wl, "fp32")
    compare(got, ref, FP32_TOL)
    st.close()


def test_zeldovich128_fp32_full(orc, step_cls):
    """The benchmark box in full, in the benchmark's launch shape (default
    tuning, graph replay of the whole step) and with leaves of 128 (the
    whole-leaf broadcast sweep), against one oracle step."""
    print("case zeldovich128 (4,194,304 particles) fp32, bench shape + leaf 128",
          flush=True)
    wl = W.make("zeldovich128")
    ref = orc.step(wl)
    st = step_cls(wl, precision="fp32")
    st.capture(integrate=False)
    st.replay()
    compare(st.outputs(), ref, FP32_TOL)
    st.close()
    st, got = run(step_cls, wl, "fp32", tuning=dict(leaf_max=128))
    compare(got, ref, FP32_TOL)
    st.close()


# ---------------------------------------------------------------------------
# invariances of the GPU path
# ---------------------------------------------------------------------------

def test_tree_structure(step_cls):
    print("case tree structure", flush=True)
    wl = W.random_uniform(5000, 4000, 501, n_ngb=48.0, h_spread=0.15,
                          clustered=True)
    st = step_cls(wl, precision="fp32", tuning=dict(leaf_max=32))
    st.run(passes=())
    info = st.tree.info()
    perm, start, count = st.tree.leaves()
    n = wl.n_total
    assert np.array_equal(np.sort(perm), np.arange(n))
    assert (count >= 1).all() and (count <= 32).all()
    assert start[0] == 0 and np.array_equal(start[1:], np.cumsum(count)[:-1])
    assert start[-1] + count[-1] == n
    # gas slots first, leaves never mix species
    assert (perm[:wl.gas.n] < wl.gas.n).all()
    ngl = info["n_gas_leaves"]
    assert start[ngl] == wl.gas.n if ngl < len(start) else True
    st.close()


def test_results_independent_of_leaf_size(orc, step_cls):
    print("case leaf-size independence", flush=True)
    wl = W.random_uniform(4000, 3000, 601, n_ngb=48.0, h_spread=0.15,
                          clustered=True)
    outs = []
    for L in (32, 64, 128, 256):
        st, got = run(step_cls, wl, "fp32", tuning=dict(leaf_max=L))
        outs.append(got)
        st.close()
    for o in outs[1:]:
        compare(o, outs[0], 2e-6)


def test_deterministic_and_graph_replay(step_cls):
    print("case determinism + graph replay", flush=True)
    wl = W.random_uniform(4000, 3000, 701, n_ngb=48.0, h_spread=0.15)
    st, a = run(step_cls, wl, "fp32")
    st.run()
    b = st.outputs()
    for k in KEYS:
        assert np.array_equal(a[k], b[k]), k
    st.capture(integrate=False)
    for rep in range(3):
        st.replay()
        c = st.outputs()
        for k in KEYS:
            assert np.array_equal(a[k], c[k]), (rep, k)
    st.close()


def test_batched_boxes(orc, step_cls):
    print("case 6 uneven boxes", flush=True)
    boxes = [W.random_uniform(n, m, 800 + k, n_ngb=48.0, h_spread=0.15)
             for k, (n, m) in enumerate([(2000, 1500), (500, 700), (3000, 0),
                                         (900, 2600), (1200, 1200),
                                         (4000, 3500)])]
    wl = W.concat_boxes("six", boxes)
    st, got = run(step_cls, wl, "fp32")
    ref = orc.step(wl)
    compare(got, ref, FP32_TOL)
    # box 3 alone gives bitwise the same results as inside the batch
    alone, got3 = run(step_cls, boxes[3], "fp32")
    gs = slice(int(wl.gas_off[3]), int(wl.gas_off[4]))
    ds = slice(int(wl.dm_off[3]), int(wl.dm_off[4]))
    for k in ("V", "A", "B", "gradB", "rho", "dudt"):
        assert np.array_equal(got[k][gs], got3[k]), k
    assert np.array_equal(got["a_hydro"][:, gs], got3["a_hydro"])
    assert np.array_equal(got["a_grav_dm"][:, ds], got3["a_grav_dm"])
    st.close()
    alone.close()


def test_integrate_matches_oracle(orc, step_cls):
    print("case integrate", flush=True)
    dt = 1e-3
    wl = W.random_uniform(3000, 2000, 901, n_ngb=48.0, h_spread=0.15)
    st = step_cls(wl, precision="fp32", dt=dt)
    st.run(integrate=True)
    st.sync()
    ref = orc.step(wl)
    g = wl.gas
    x0 = np.stack([g.x, g.y, g.z]).astype(np.float64)
    v0 = np.stack([g.vx, g.vy, g.vz]).astype(np.float64)
    o = orc.integrate(dt, x0, v0, g.u, ref["a_grav_gas"], ref["a_hydro"],
                      ref["dudt"])
    x64 = st.gx64.cpu().numpy().reshape(3, -1)
    v64 = st.gv64.cpu().numpy().reshape(3, -1)
    u64 = st.gu64.cpu().numpy()
    # increments carry the float32 accelerations: same bound as the passes
    assert rel_rms(v64 - v0, o["v"] - v0) < FP32_TOL
    assert rel_rms(u64 - g.u, o["u"] - g.u) < FP32_TOL
    # the drift uses the new velocity, then wraps into [1, 2)
    xd = x0 + dt * v64
    xd = np.where(xd >= 2.0, xd - 1.0, xd)
    xd = np.where(xd < 1.0, xd + 1.0, xd)
    assert np.abs(x64 - xd).max() < 1e-15
    # the float32 copies are the rounded doubles
    x32 = x64[0].astype(np.float32)
    x32[x32 >= 2.0] = 1.0
    assert np.array_equal(st.gx.cpu().numpy()[:g.n], x32)
    st.close()


# ---------------------------------------------------------------------------
# errors detected on the device and on the host
# ---------------------------------------------------------------------------

def test_device_input_errors(step_cls):
    from paper_2510_03557_amd.binding import CrkError, CRK_EINVAL
    print("case device-side input errors", flush=True)
    wl = W.random_uniform(1000, 500, 1001)
    st = step_cls(wl, precision="fp32")
    st.h_max = st.h_max * 0.5  # declared bound below the real h
    st.run(passes=())
    with pytest.raises(CrkError) as e:
        st.sync()
    assert e.value.status == CRK_EINVAL
    st.sync()  # the error is cleared
    st.close()


def test_host_argument_errors(step_cls):
    from paper_2510_03557_amd.binding import CrkError, CRK_EINVAL, CRK_ESTATE
    print("case host-side argument errors", flush=True)
    wl = W.random_uniform(1000, 500, 1002)
    st = step_cls(wl, precision="fp32")
    c, t = st.ctx, st.tree
    with pytest.raises(CrkError) as e:
        c.density(t, st.gm, st.V, st.rho_t)  # tree not built yet
    assert e.value.status in (CRK_EINVAL, CRK_ESTATE)
    for bad in (dict(r_c=[0.6]), dict(r_c=[0.0]), dict(h_max=[0.3]),
                dict(eps=[1.0])):
        args = dict(r_c=wl.r_c, eps=wl.eps, h_max=st.h_max)
        args.update({k: np.array(v) for k, v in bad.items()})
        with pytest.raises(CrkError) as e:
            c.build_tree(t, wl.gas_off, wl.dm_off, args["r_c"], args["eps"],
                         args["h_max"], st.gx, st.gy, st.gz, st.gh, st.dx,
                         st.dy, st.dz)
        assert e.value.status == CRK_EINVAL
    with pytest.raises(CrkError):
        c.set_tuning(leaf_max=8)
    with pytest.raises(CrkError):
        c.build_tree(t, wl.gas_off, wl.dm_off, wl.r_c, wl.eps, st.h_max,
                     None, st.gy, st.gz, st.gh, st.dx, st.dy, st.dz)
    st.close()


def test_capacity_overflow_in_graph_is_reported(step_cls):
    from paper_2510_03557_amd.binding import CrkError, CRK_ECAPACITY, CRK_ESTATE
    print("case graph capacity overflow", flush=True)
    wl = W.random_uniform(3000, 2000, 1101, n_ngb=48.0, h_spread=0.15)
    st = step_cls(wl, precision="fp32")
    try:
        st.capture(integrate=False)
        # gathering all gas into one tiny region after capture needs deeper
        # k-d trees and longer lists than the captured capacities
        g = wl.gas
        blob = (np.float32(1.5) + np.float32(1e-4) *
                np.arange(g.n, dtype=np.float32) / g.n).astype(np.float32)
        st.set_inputs(gx=blob, gy=blob[::-1].copy(), gz=blob)
        st.replay()
        with pytest.raises(CrkError) as e:
            st.sync()
        assert e.value.status == CRK_ECAPACITY
        # the documented recovery: an eager step at the new size, then a
        # new capture.  The old graph is never replayed past that step
        # unnoticed: if the eager step grew (moved) a buffer the graph
        # refuses to launch (CRK_ESTATE); if every buffer was large enough
        # it still carries the capacities of its capture and reports the
        # overflow again
        st.run(integrate=False)
        st.sync()
        try:
            st.replay()
        except CrkError as e:
            assert e.value.status == CRK_ESTATE
        else:
            with pytest.raises(CrkError) as e:
                st.sync()
            assert e.value.status == CRK_ECAPACITY
        st.capture(integrate=False)
        st.replay()
        st.sync()
    finally:
        st.close()


def test_graph_refuses_launch_after_buffers_are_freed(step_cls):
    """A captured graph is not launched once library buffers it may hold
    were freed (here: another context and its tree destroyed); a new
    capture launches again."""
    from paper_2510_03557_amd.binding import CrkError, CRK_ESTATE
    print("case graph invalidated by freed buffers", flush=True)
    wl = W.random_uniform(2000, 1500, 1111, n_ngb=48.0, h_spread=0.15)
    st = step_cls(wl, precision="fp32")
    try:
        st.capture(integrate=False)
        st.replay()
        st.sync()
        other = step_cls(W.random_uniform(500, 400, 1112, n_ngb=32.0),
                         precision="fp32")
        other.run()
        other.sync()
        other.close()
        with pytest.raises(CrkError) as e:
            st.replay()
        assert e.value.status == CRK_ESTATE
        st.drop_graph()
        with pytest.raises(RuntimeError):
            st.replay()
        st.capture(integrate=False)
        st.replay()
        st.sync()
    finally:
        st.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_sub_leaf_sweeps_match_whole_leaf_sweep(orc, step_cls, precision):
    """Sub-leaf sweeps (lane groups; one wavefront per sub-leaf with four
    lanes per particle; four wavefronts per leaf sharing one staging of the
    leaf's candidates) only drop candidates that are out of range of every
    particle of the sub-leaf.  The sub-leaf split reorders the slots inside
    each leaf and the split forms sum each particle's candidates in four
    interleaved streams (and, in float, far gravity candidates with the
    series form of the softening), so sums agree with the whole-leaf sweep
    up to rounding, and all agree with the oracle."""
    print(f"case sub-leaf sweeps vs whole-leaf sweep {precision}", flush=True)
    wl = W.random_uniform(6000, 5000, 1301, n_ngb=48.0, clustered=True)
    outs = []
    for ss in (0, 1, 2, 3):
        st, o = run(step_cls, wl, precision,
                    tuning=dict(leaf_max=64, sub_sweep=ss))
        outs.append(o)
        st.close()
    tol_same = 2e-6 if precision == "fp32" else 1e-12
    for k in (1, 2, 3):
        compare(outs[k], outs[0], tol_same)
    ref = orc.step(wl)
    for k in (2, 3):
        compare(outs[k], ref, FP32_TOL if precision == "fp32" else FP64_TOL)


@pytest.mark.parametrize("tuning", [dict(grid_mult=16), dict(xcd_remap=1),
                                    dict(walk_mask=15),
                                    dict(grid_mult=8, leaf_max=128)])
def test_launch_shapes_are_bitwise_identical(step_cls, tuning):
    """The persistent cost-ordered queue, the XCD remap and the per-lane hit
    walk change only which workgroup or lane order runs a leaf: each lane
    still meets its candidates in list order, so the sums are bitwise the
    same as one workgroup per leaf with the broadcast sweep."""
    print(f"case launch shape {tuning}", flush=True)
    wl = W.random_uniform(6000, 5000, 1501, n_ngb=48.0, clustered=True)
    L = tuning.get("leaf_max", 64)
    base = dict(leaf_max=L, sub_sweep=0, xcd_remap=0)
    st, ref = run(step_cls, wl, "fp32", tuning=base)
    st.close()
    st, got = run(step_cls, wl, "fp32", tuning=dict(base, **tuning))
    st.close()
    for k in KEYS:
        assert np.array_equal(ref[k], got[k]), k


@pytest.mark.parametrize("form", [dict(sub_sweep=2), dict(sub_sweep=3)])
def test_sub_leaf_queue_forms(orc, step_cls, form):
    """The persistent cost-ordered queue of each sub-leaf form (64-thread
    workgroups popping sub-leaves; four-wavefront workgroups popping
    leaves) runs every item exactly as the one-workgroup-per-item launch
    does, so the outputs are bitwise the same; and they match the oracle."""
    print(f"case queue form {form}", flush=True)
    wl = W.random_uniform(6000, 5000, 1511, n_ngb=48.0, clustered=True)
    base = dict(leaf_max=64, **form)
    st, ref = run(step_cls, wl, "fp32", tuning=base)
    st.close()
    for gm in (1, 16):
        st, got = run(step_cls, wl, "fp32", tuning=dict(base, grid_mult=gm))
        st.close()
        for k in KEYS:
            assert np.array_equal(ref[k], got[k]), (gm, k)
    compare(got, orc.step(wl), FP32_TOL)


@pytest.mark.parametrize("tile", [1, 2, 8])
def test_tile_widths_match_oracle(orc, step_cls, tile):
    """The j-tile width (candidate buffer of the split form) only moves the
    points where partial sums are folded: every width matches the oracle."""
    print(f"case tile {tile}", flush=True)
    wl = W.random_uniform(5000, 4000, 1521, n_ngb=48.0, clustered=True)
    st, got = run(step_cls, wl, "fp32",
                  tuning=dict(leaf_max=64, sub_sweep=2, tile=tile))
    st.close()
    compare(got, orc.step(wl), FP32_TOL)


@pytest.mark.parametrize("precision,L,cm", [("fp32", 64, 0.0), ("fp64", 32, 0.0),
                                            ("fp32", 64, 64.0)])
def test_lds_tree_matches_global_sorts(step_cls, precision, L, cm):
    """The per-bin LDS build gives the same tree as the per-axis global
    sorts (same leaves, same slot order), hence bitwise the same outputs.
    cm_factor 64 makes one bin per species per box, larger than the LDS
    segment bound, which takes the global path under either setting."""
    print(f"case lds tree vs global sorts {precision} L={L} cm={cm}",
          flush=True)
    wl = W.random_uniform(6000, 5000, 1401, n_ngb=48.0, clustered=True)
    trees, outs = [], []
    for lds in (0, 1):
        st, o = run(step_cls, wl, precision,
                    tuning=dict(leaf_max=L, cm_factor=cm, tree_lds=lds,
                                sub_sweep=0))
        trees.append(st.tree.leaves())
        outs.append(o)
        st.close()
    for a, b in zip(trees[0], trees[1]):
        assert np.array_equal(a, b)
    for k in KEYS:
        assert np.array_equal(outs[0][k], outs[1][k]), k
    # with sub-leaves the two paths split the leaves independently (the
    # per-bin build continues its levels at 16, the general path splits
    # each leaf in a wavefront): same leaves, sums equal up to rounding
    subs = []
    for lds in (0, 1):
        st, o = run(step_cls, wl, precision,
                    tuning=dict(leaf_max=L, cm_factor=cm, tree_lds=lds,
                                sub_sweep=2))
        _, start, count = st.tree.leaves()
        assert np.array_equal(start, trees[0][1])
        assert np.array_equal(count, trees[0][2])
        subs.append(o)
        st.close()
    compare(subs[1], subs[0], 2e-6 if precision == "fp32" else 1e-12)


def test_autotune_keeps_results(orc, step_cls):
    """The tuner only picks among launch shapes; after it the step still
    matches the oracle."""
    from paper_2510_03557_amd import autotune
    print("case autotune", flush=True)
    wl = W.random_uniform(3000, 2500, 1601, n_ngb=48.0, h_spread=0.15)
    st = step_cls(wl, precision="fp32")
    cands = [dict(leaf_max=32, sub_sweep=0), dict(leaf_max=64, sub_sweep=2)]
    res = autotune.tune(st, candidates=cands, reps=2, use_cache=False)
    assert res["tuning"] in cands and len(res["ms"]) == 2
    # the tuner leaves the step eager at the chosen shape: no stale graph
    # of the last candidate can be replayed
    assert not st.graph
    with pytest.raises(RuntimeError):
        st.replay()
    got = st.ctx.get_tuning()
    for k, v in res["tuning"].items():
        assert got[k] == v, k
    st.run()
    compare(st.outputs(), orc.step(wl), FP32_TOL)
    st.close()


# ---------------------------------------------------------------------------
# degenerate and edge inputs
# ---------------------------------------------------------------------------

def test_tiny_and_empty_boxes(orc, step_cls):
    """Boxes with one, two, three or no particles of a species, and an
    empty box, batched with ordinary ones: a lone gas particle has only
    itself in range, and two or three points span no volume (singular
    moments, the degenerate coefficient branch)."""
    print("case tiny and empty boxes", flush=True)
    sizes = [(1, 0), (0, 1), (0, 0), (2, 1), (3, 2), (40, 30), (2000, 1500)]
    boxes = [W.random_uniform(n, m, 1700 + k, n_ngb=20.0 if n < 100 else 48.0,
                              h_spread=0.15,
                              h_rule="knn" if n > 22 else "global")
             for k, (n, m) in enumerate(sizes)]
    wl = W.concat_boxes("tiny", boxes)
    for precision, tol in (("fp32", FP32_TOL), ("fp64", FP64_TOL)):
        st, got = run(step_cls, wl, precision)
        ref = orc.step(wl)
        compare(got, ref, tol)
        assert (ref["degenerate"][:6] == 1).all()
        st.close()


def test_empty_workload(step_cls):
    """No particles at all: build_tree refuses (CRK_EINVAL, nothing to
    build); the step driver skips the calls and returns empty outputs."""
    from paper_2510_03557_amd.binding import CrkError, CRK_EINVAL
    print("case empty workload", flush=True)
    wl = W.random_uniform(0, 0, 1801)
    st, got = run(step_cls, wl, "fp32")
    assert all(np.asarray(v).size == 0 for v in got.values())
    with pytest.raises(CrkError) as e:
        st.ctx.build_tree(st.tree, wl.gas_off, wl.dm_off, wl.r_c, wl.eps,
                          st.h_max, st.gx, st.gy, st.gz, st.gh, st.dx, st.dy,
                          st.dz)
    assert e.value.status == CRK_EINVAL
    st.close()


def test_coincident_particles(orc, step_cls):
    """Exactly coincident particles: r = 0 pairs add nothing to gravity, an
    isolated coincident group has exactly singular moments, and a group
    inside a random set stays regular."""
    print("case coincident particles", flush=True)
    a = W.random_uniform(8, 0, 1901, h_rule="global")
    for c in (a.gas.x, a.gas.y, a.gas.z):
        c[:] = np.float32(1.5)
    a.gas.h[:] = np.float32(0.05)
    b = W.random_uniform(2000, 1000, 1902, n_ngb=48.0)
    for c in (b.gas.x, b.gas.y, b.gas.z):
        c[:30] = np.float32(1.25)
    for c in (b.dm.x, b.dm.y, b.dm.z):
        c[:20] = np.float32(1.25)
    wl = W.concat_boxes("coincident", [a, b])
    st, got = run(step_cls, wl, "fp32")
    ref = orc.step(wl)
    assert (ref["degenerate"][:8] == 1).all()
    compare(got, ref, FP32_TOL)
    st.close()
