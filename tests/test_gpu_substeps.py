"""GPU parity of the hierarchical time steps (timestep bins, active leaves on
a refitted tree, block kick-drift-kick cycle) against the FP64 oracle,
through the C ABI.

Bins are integers decided in double on both sides from the same inputs:
bit-exact.  The cycle's changes of velocity, position and energy and the
last evaluation's outputs: relative RMS <= 1e-5 (float32 path) and 1e-9
(float64 path, rounding order only, accumulated over the substeps).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_03557_amd import workloads as W  # noqa: E402

FP32_TOL = 1e-5
FP64_TOL = 1e-9
KEYS = ("V", "rho_tilde", "A", "B", "gradA", "gradB", "rho", "P", "cs",
        "a_hydro", "dudt", "a_grav_gas", "a_grav_dm")


def rel_rms(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.sqrt(np.sum(b * b))
    num = np.sqrt(np.sum((a - b) ** 2))
    return num / den if den > 0 else num


@pytest.fixture()
def step_cls():
    """The step class; every step made in a test is closed at its end,
    also when the test fails."""
    from paper_2510_03557_amd.step import ShortRangeStep
    assert torch.cuda.is_available()
    made = []

    def make(*args, **kw):
        st = ShortRangeStep(*args, **kw)
        made.append(st)
        return st

    yield make
    for st in made:
        st.close()
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# bins
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_timestep_bins_match_oracle(orc, precision):
    from paper_2510_03557_amd.binding import Context
    print(f"case timestep bins {precision}", flush=True)
    rng = np.random.default_rng(7)
    n = 200_000
    dt, L, eps, c_cfl, eta = 0.01, 8, 1e-4, 0.25, 0.025
    npT = np.float32 if precision == "fp32" else np.float64
    # accelerations over five decades, some exactly zero
    mag = 10.0 ** rng.uniform(-1, 4, n)
    mag[::97] = 0.0
    ag = (rng.standard_normal((3, n)) * mag).astype(npT)
    ah = (0.3 * rng.standard_normal((3, n)) * mag).astype(npT)
    h = (0.01 * np.exp(0.5 * rng.standard_normal(n))).astype(npT)
    cs = (10.0 ** rng.uniform(-1, 2.5, n)).astype(npT)
    ctx = Context(precision)
    try:
        _bins_case(orc, ctx, n, dt, L, eps, c_cfl, eta, ag, ah, h, cs)
    finally:
        ctx.close()
        torch.cuda.synchronize()


def _bins_case(orc, ctx, n, dt, L, eps, c_cfl, eta, ag, ah, h, cs):
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
           for a in (*ag, *ah, h, cs)]
    bins = torch.zeros(n, dtype=torch.int32, device="cuda")
    # (the inputs and the zero fill are on torch's stream, the library works
    # on its own)
    torch.cuda.synchronize()
    ctx.timestep_bins(n, dt, L, eps, c_cfl, eta, dev[0:3], dev[3:6], dev[6],
                      dev[7], bins)
    ctx.stream.synchronize()
    a64 = ag.astype(np.float64) + ah.astype(np.float64)
    ref = orc.timestep_bins(dt, L, eps, a64[0], a64[1], a64[2],
                            h=h.astype(np.float64), cs=cs.astype(np.float64),
                            c_cfl=c_cfl, eta=eta)
    got = bins.cpu().numpy()
    print("gas bin counts", np.bincount(ref, minlength=L + 1), flush=True)
    assert np.array_equal(got, ref)
    assert len(np.unique(ref)) >= 6
    # dark matter: acceleration only
    ctx.timestep_bins(n, dt, L, eps, c_cfl, eta, dev[0:3], None, None, None,
                      bins)
    ctx.stream.synchronize()
    ref = orc.timestep_bins(dt, L, eps, *ag.astype(np.float64), eta=eta)
    assert np.array_equal(bins.cpu().numpy(), ref)


# ---------------------------------------------------------------------------
# one pass over active leaves writes exactly the active particles
# ---------------------------------------------------------------------------

def _agree(g, f, rel):
    """Per value: |g - f| <= rel (|f| + RMS of f)."""
    g = np.asarray(g, np.float64)
    f = np.asarray(f, np.float64)
    rms = np.sqrt(np.mean(f * f)) if f.size else 0.0
    return bool(np.all(np.abs(g - f) <= rel * (np.abs(f) + rms)))


@pytest.mark.parametrize("sub_sweep,act_groups", [(2, 0), (3, 0), (2, 1),
                                                  (3, 1), (2, 4096)])
def test_active_passes_write_active_particles_only(step_cls, sub_sweep,
                                                   act_groups):
    """After crk_tree_set_active, each pass writes, for the active particles,
    the values of the full pass and leaves every other output untouched; in
    both sub-leaf forms (one wavefront per sub-leaf, or four per leaf
    sharing the staging).  On the tree's sub-leaves (act_groups 0) the
    active particles' leaves are swept as in the full pass: bitwise.  On the
    dense active groups (act_groups 1) each active particle sweeps the same
    pairs with candidates culled against another box, so the compensated
    sums group differently: to 2e-6 of |value| + RMS per value.  A
    threshold above the active particles per active leaf (4096) keeps the
    tree's sub-leaves."""
    print(f"case active passes random_uniform(6000, 5000) sub_sweep "
          f"{sub_sweep} act_groups {act_groups}", flush=True)
    wl = W.random_uniform(6000, 5000, 401, n_ngb=48.0, h_spread=0.15)
    st = step_cls(wl, "fp32", tuning=dict(leaf_max=64, sub_sweep=sub_sweep,
                                          act_groups=act_groups))
    st.run()
    full = st.outputs()
    rng = np.random.default_rng(5)
    L = 3
    bg = rng.integers(0, L + 1, st.ng)
    bd = rng.integers(0, L + 1, st.nd)
    st.set_bins(bg, bd)
    c, t = st.ctx, st.tree
    s = 2  # ends a step: (s + 1) % 2^(L - b) == 0 -> bins 3 and 2
    act_g = ((s + 1) % (2 ** (L - bg))) == 0
    act_d = ((s + 1) % (2 ** (L - bd))) == 0
    assert 0 < act_g.sum() < st.ng and 0 < act_d.sum() < st.nd
    c.tree_set_active(t, st.bins_g, st.bins_d, L, s)
    info = t.info()
    assert info["act_particles"] == act_g.sum() + act_d.sum()
    assert 0 < info["act_leaves"] <= info["n_leaves"]
    grouped = info["act_grouped"] == 1
    assert grouped == (act_groups == 1), info
    c.build_interaction_lists(t)
    sentinel = -7.25
    groups = {
        "density": (("V", "rho_t"), ("V", "rho_tilde")),
        "coefficients": (("A", "B", "gA", "gB", "rho", "P", "cs"),
                         ("A", "B", "gradA", "gradB", "rho", "P", "cs")),
        "hydro": (("ahx", "ahy", "ahz", "dudt"), ("a_hydro", "dudt")),
        "gravity": (("agx", "agy", "agz", "adx", "ady", "adz"),
                    ("a_grav_gas", "a_grav_dm")),
    }
    saved = {k: getattr(st, k).clone()
             for names, _ in groups.values() for k in names}
    for name, (attrs, keys) in groups.items():
        with torch.cuda.stream(c.stream):
            for k in attrs:
                getattr(st, k).fill_(sentinel)
        if name == "density":
            c.density(t, st.gm, st.V, st.rho_t)
        elif name == "coefficients":
            c.coefficients(t, st.gm, st.V, st.gu, st.A, st.B, st.gA, st.gB,
                           st.rho, st.P, st.cs)
        elif name == "hydro":
            c.hydro_forces(t, st.gm, st.gvx, st.gvy, st.gvz, st.V, st.rho,
                           st.P, st.cs, st.A, st.B, st.gA, st.gB, st.ahx,
                           st.ahy, st.ahz, st.dudt)
        else:
            c.shortrange_gravity(t, st.gm, st.dm, st.agx, st.agy, st.agz,
                                 st.adx, st.ady, st.adz)
        got = st.outputs()
        for k in keys:
            g, f = got[k], full[k]
            act = act_d if k == "a_grav_dm" else act_g
            ga = g[..., act] if k.startswith("a_") else g[act]
            fa = f[..., act] if k.startswith("a_") else f[act]
            gi = g[..., ~act] if k.startswith("a_") else g[~act]
            if grouped:
                assert _agree(ga, fa, 2e-6), (name, k)
            else:
                assert np.array_equal(ga, fa), (name, k)
            assert np.all(gi == sentinel), (name, k)
        # restore the full values before the next pass reads them
        with torch.cuda.stream(c.stream):
            for k in attrs:
                getattr(st, k).copy_(saved[k])
    # a new subset invalidates the lists until they are rebuilt
    c.tree_set_active(t, None, None, 0, -1)
    info = t.info()
    assert (info["act_leaves"], info["act_particles"],
            info["act_grouped"]) == (0, 0, 0)
    from paper_2510_03557_amd.binding import CrkError, CRK_ESTATE
    with pytest.raises(CrkError) as e:
        c.density(t, st.gm, st.V, st.rho_t)
    assert e.value.status == CRK_ESTATE
    st.close()


# ---------------------------------------------------------------------------
# whole cycles
# ---------------------------------------------------------------------------

def _cycle_errors(wl, got, ref):
    g, d = wl.gas, wl.dm
    x0g = np.array([g.x, g.y, g.z], np.float64)
    v0g = np.array([g.vx, g.vy, g.vz], np.float64)
    x0d = np.array([d.x, d.y, d.z], np.float64)
    v0d = np.array([d.vx, d.vy, d.vz], np.float64)

    def disp(x, x0):
        e = x - x0
        return e - np.round(e)

    errs = dict(
        dx_gas=rel_rms(disp(got["xg"], x0g), disp(ref["xg"], x0g)),
        dv_gas=rel_rms(got["vg"] - v0g, ref["vg"] - v0g),
        du=rel_rms(got["u"] - np.asarray(g.u, np.float64),
                   ref["u"] - np.asarray(g.u, np.float64)),
        dx_dm=rel_rms(disp(got["xd"], x0d), disp(ref["xd"], x0d)),
        dv_dm=rel_rms(got["vd"] - v0d, ref["vd"] - v0d))
    return errs


def _close_pair_members(ref, eps, factor=3.0):
    """Masks (gas, dm) of the particles with another particle closer than
    factor * eps in the oracle's final state.  Their softened forces change
    by up to ~1e-4 for a one-ulp change of their separation, so float32
    trajectories that agree to 1e-7 can still give final forces that differ
    by more than 1e-5 for them alone: the final outputs are compared over
    the other particles (the trajectories over all)."""
    from scipy.spatial import cKDTree
    x = np.concatenate([ref["xg"], ref["xd"]], axis=1).T - 1.0
    x = np.mod(x, 1.0)
    tree = cKDTree(x, boxsize=1.0)
    pairs = tree.query_pairs(factor * eps, output_type="ndarray")
    close = np.zeros(x.shape[0], bool)
    close[pairs.ravel()] = True
    ng = ref["xg"].shape[1]
    return close[:ng], close[ng:]


# The clustered set is asserted on the float64 path only: there a random
# one-ulp change of the float32 positions alone moves B, grad B and a_hydro
# by ~3e-5 (relative RMS; ill-conditioned moment matrices between the
# blobs), so float32 trajectories that differ by an ulp cannot agree to
# 1e-5; the float64 path checks the same cycle logic to rounding.
@pytest.mark.parametrize("precision,clustered,L,seed", [
    ("fp32", False, 3, 501), ("fp64", True, 2, 502), ("fp64", False, 2, 503)])
def test_substep_cycle_matches_oracle(orc, step_cls, precision, clustered, L,
                                      seed):
    print(f"case cycle {precision} clustered={clustered} L={L}", flush=True)
    wl = W.random_uniform(12000, 10000, seed, n_ngb=48.0, h_spread=0.15,
                          clustered=clustered)
    rng = np.random.default_rng(seed)
    bg = rng.integers(0, L + 1, wl.gas.n)
    bd = rng.integers(0, L + 1, wl.dm.n)
    dt = 0.02
    st = step_cls(wl, precision)
    st.set_bins(bg, bd)
    st.substep_cycle(dt, L)
    got = st.state()
    outs = st.outputs()
    ref = orc.substep_cycle(wl, bg, bd, dt, L, forces_at=(
        "float32" if precision == "fp32" else "float64"))
    tol = FP32_TOL if precision == "fp32" else FP64_TOL
    errs = _cycle_errors(wl, got, ref)
    if precision == "fp32":
        cg, cd = _close_pair_members(ref, float(wl.eps[0]))
    else:
        cg, cd = np.zeros(wl.gas.n, bool), np.zeros(wl.dm.n, bool)
    for k in KEYS:
        keep = ~cd if k == "a_grav_dm" else ~cg
        g, r = outs[k], ref[k]
        if k.startswith("a_"):
            errs[k] = rel_rms(g[:, keep], r[:, keep])
        else:
            errs[k] = rel_rms(g[keep], r[keep])
    print({k: f"{v:.2e}" for k, v in errs.items()},
          f"(final outputs without {int(cg.sum())} gas and {int(cd.sum())} "
          "dm particles in close pairs)", flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    # positions wrapped back into [1, 2)
    assert np.all((got["xg"] >= 1) & (got["xg"] < 2))
    st.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_cycle_with_long_range_matches_oracle(orc, step_cls, precision):
    """The cycle bracketed by long-range mesh half-kicks (the whole force
    split: mesh long range, subcycled short range)."""
    print(f"case cycle + mesh long range {precision}", flush=True)
    wl = W.random_uniform(12000, 10000, 505, n_ngb=48.0, h_spread=0.15)
    rng = np.random.default_rng(505)
    L = 2
    bg = rng.integers(0, L + 1, wl.gas.n)
    bd = rng.integers(0, L + 1, wl.dm.n)
    n_mesh = 2 * int(np.ceil(3.0 / float(wl.r_c[0])))
    dt = 0.02
    st = step_cls(wl, precision)
    st.set_bins(bg, bd)
    st.substep_cycle(dt, L, pm_mesh=n_mesh)
    got = st.state()
    ref = orc.substep_cycle(wl, bg, bd, dt, L, pm_mesh=n_mesh, forces_at=(
        "float32" if precision == "fp32" else "float64"))
    errs = _cycle_errors(wl, got, ref)
    print(f"mesh {n_mesh}", {k: f"{v:.2e}" for k, v in errs.items()},
          flush=True)
    tol = FP32_TOL if precision == "fp32" else FP64_TOL
    assert all(v <= tol for v in errs.values()), errs


@pytest.mark.parametrize("precision,L,seed", [("fp32", 3, 507),
                                               ("fp64", 2, 508)])
def test_cycle_with_reconstructed_viscosity(orc, step_cls, precision, L,
                                            seed):
    """The cycle with the velocity-gradient pass and the reconstructed
    viscosity: gradients of active particles only, the latest gradients of
    inactive neighbours in the limiter."""
    print(f"case cycle + reconstructed viscosity {precision} L={L}",
          flush=True)
    wl = W.random_uniform(12000, 8000, seed, n_ngb=48.0, h_spread=0.15)
    rng = np.random.default_rng(seed)
    bg = rng.integers(0, L + 1, wl.gas.n)
    bd = rng.integers(0, L + 1, wl.dm.n)
    dt = 0.02
    st = step_cls(wl, precision, recon=True)
    try:
        st.set_bins(bg, bd)
        st.substep_cycle(dt, L)
        got = st.state()
        outs = st.outputs()
    finally:
        st.close()
    ref = orc.substep_cycle(wl, bg, bd, dt, L, recon=True, forces_at=(
        "float32" if precision == "fp32" else "float64"))
    errs = _cycle_errors(wl, got, ref)
    errs.update({k: rel_rms(outs[k], ref[k]) for k in ("dv", "a_hydro",
                                                        "dudt")})
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    tol = FP32_TOL if precision == "fp32" else FP64_TOL
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad


def test_cycle_bins_from_accelerations(orc, step_cls):
    """Bins from crk_timestep_bins on the step's own accelerations (gas:
    Courant and acceleration; dm: acceleration), then a cycle: the bins
    equal the oracle's decision on the same float32 inputs and the cycle
    matches the oracle run with those bins."""
    print("case cycle with computed bins", flush=True)
    wl = W.random_uniform(10000, 9000, 601, n_ngb=48.0, h_spread=0.15,
                          clustered=True)
    st = step_cls(wl, "fp32")
    st.run()
    out = st.outputs()
    dt, L = 0.01, 4
    eps = float(wl.eps[0])
    bg, bd = st.timestep_bins(dt, L, c_cfl=0.25, eta=0.025)
    a = (out["a_grav_gas"].astype(np.float32).astype(np.float64)
         + out["a_hydro"].astype(np.float32).astype(np.float64))
    ref_g = orc.timestep_bins(dt, L, eps, *a, h=wl.gas.h.astype(np.float64),
                              cs=out["cs"], c_cfl=0.25, eta=0.025)
    ref_d = orc.timestep_bins(dt, L, eps, *out["a_grav_dm"], eta=0.025)
    print("bins gas", np.bincount(bg, minlength=L + 1),
          "dm", np.bincount(bd, minlength=L + 1), flush=True)
    assert np.array_equal(bg, ref_g) and np.array_equal(bd, ref_d)
    assert len(np.unique(bg)) >= 3
    st.close()
    st = step_cls(wl, "fp32")
    st.set_bins(bg, bd)
    st.substep_cycle(dt, L)
    got = st.state()
    ref = orc.substep_cycle(wl, bg, bd, dt, L, forces_at="float32")
    errs = _cycle_errors(wl, got, ref)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert all(v <= FP32_TOL for v in errs.values()), errs
    st.close()


def test_refit_reports_stale_tree(step_cls):
    """Positions moved far out of their bins: crk_tree_refit returns
    CRK_ESTALE (the stencil could miss pairs) instead of a wrong result."""
    from paper_2510_03557_amd.binding import CrkError, CRK_ESTALE
    print("case stale refit", flush=True)
    wl = W.random_uniform(20000, 20000, 701, n_ngb=48.0)
    st = step_cls(wl, "fp32")
    st.run()
    c, t = st.ctx, st.tree
    # a small move is accepted
    with torch.cuda.stream(c.stream):
        st.gx.add_(1e-4)
    c.tree_refit(t, st.gx, st.gy, st.gz, st.dx, st.dy, st.dz)
    with torch.cuda.stream(c.stream):
        st.gx.add_(0.2)
    with pytest.raises(CrkError) as e:
        c.tree_refit(t, st.gx, st.gy, st.gz, st.dx, st.dy, st.dz)
    assert e.value.status == CRK_ESTALE
    st.close()
