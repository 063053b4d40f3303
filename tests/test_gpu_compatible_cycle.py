"""GPU parity of the compatible energy update inside the hierarchical cycle
(crk_hydro_energy_compatible_block) against the FP64 oracle, through the C
ABI.

The library makes one compatible pass per evaluation, for a particle's
closing half-kick and the opening half-kick of its next step together; the
oracle makes one per half-kick.  The pair work is linear in the centred
velocities and both half-kicks use the same forces, so the two agree up to
rounding: the cycle's changes of x, v and u and the rate of the final
closing kick at relative RMS <= 1e-5 (float32 path) and 1e-9 (float64
path), as for the plain cycle.  With G = 0 and one bin (or non-interacting
clumps in different bins) the float64 path conserves sum m (v^2/2 + u) to
rounding, a property that holds at any size.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_03557_amd import workloads as W  # noqa: E402

FP32_TOL = 1e-5
FP64_TOL = 1e-9


def rel_rms(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.sqrt(np.sum(b * b))
    num = np.sqrt(np.sum((a - b) ** 2))
    return num / den if den > 0 else num


@pytest.fixture()
def step_cls():
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


def _changes(wl, got, ref):
    g, d = wl.gas, wl.dm
    x0g = np.array([g.x, g.y, g.z], np.float64)
    v0g = np.array([g.vx, g.vy, g.vz], np.float64)
    v0d = np.array([d.vx, d.vy, d.vz], np.float64)

    def disp(x, x0):
        e = x - x0
        return e - np.round(e)

    return dict(
        dx_gas=rel_rms(disp(got["xg"], x0g), disp(ref["xg"], x0g)),
        dv_gas=rel_rms(got["vg"] - v0g, ref["vg"] - v0g),
        du=rel_rms(got["u"] - np.asarray(g.u, np.float64),
                   ref["u"] - np.asarray(g.u, np.float64)),
        dv_dm=rel_rms(got["vd"] - v0d, ref["vd"] - v0d))


def _close_gas(ref, eps, factor=3.0):
    """Gas particles with another particle closer than factor * eps: their
    float32 forces (and so the final rate) move by ~1e-4 with one ulp of
    separation; the final rate is compared over the others."""
    from scipy.spatial import cKDTree
    x = np.mod(np.concatenate([ref["xg"], ref["xd"]], axis=1).T - 1.0, 1.0)
    pairs = cKDTree(x, boxsize=1.0).query_pairs(factor * eps,
                                                output_type="ndarray")
    close = np.zeros(x.shape[0], bool)
    close[pairs.ravel()] = True
    return close[:ref["xg"].shape[1]]


@pytest.mark.parametrize("precision,recon,clustered,L,seed", [
    ("fp32", False, False, 3, 601), ("fp64", False, True, 2, 602),
    ("fp64", True, False, 2, 603), ("fp32", True, False, 2, 604)])
def test_compatible_cycle_matches_oracle(orc, step_cls, precision, recon,
                                         clustered, L, seed):
    print(f"case compatible cycle {precision} recon={recon} "
          f"clustered={clustered} L={L}", flush=True)
    wl = W.random_uniform(12000, 8000, seed, n_ngb=48.0, h_spread=0.15,
                          clustered=clustered)
    rng = np.random.default_rng(seed)
    bg = rng.integers(0, L + 1, wl.gas.n)
    bd = rng.integers(0, L + 1, wl.dm.n)
    # short enough that u stays positive in every kick (at 0.02 the
    # clustered set drives some u below zero, plain rate or not)
    dt = 0.005
    st = step_cls(wl, precision, recon=recon, compatible=True)
    st.set_bins(bg, bd)
    st.substep_cycle(dt, L)
    got = st.state()
    outs = st.outputs()
    ref = orc.substep_cycle(wl, bg, bd, dt, L, recon=recon, compatible=True,
                            forces_at=("float32" if precision == "fp32"
                                       else "float64"))
    plain = orc.substep_cycle(wl, bg, bd, dt, L, recon=recon,
                              forces_at=("float32" if precision == "fp32"
                                         else "float64"))
    errs = _changes(wl, got, ref)
    keep = (~_close_gas(ref, float(wl.eps[0])) if precision == "fp32"
            else np.ones(wl.gas.n, bool))
    errs["dudt"] = rel_rms(outs["dudt"][keep], ref["dudt"][keep])
    # the compatible update is not vacuous here: it moves u by far more
    # than the tolerance
    u0 = np.asarray(wl.gas.u, np.float64)
    sep = rel_rms(plain["u"] - u0, ref["u"] - u0)
    print({k: f"{v:.2e}" for k, v in errs.items()},
          f"compatible vs plain du {sep:.2e}", flush=True)
    tol = FP32_TOL if precision == "fp32" else FP64_TOL
    assert np.all(ref["u"] > 0)
    assert sep > 20 * tol
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad


def _energy(wl, s):
    m = np.asarray(wl.gas.m, np.float64)
    return 0.5 * (m * (s["vg"] ** 2).sum(0)).sum() + (m * s["u"]).sum()


def _two_clumps(seed, n):
    base = W.random_uniform(n, 0, seed, n_ngb=40.0)
    g = base.gas
    half = g.n // 2
    off = np.where(np.arange(g.n) < half, 0.05, 0.55)
    pos = [off + 0.3 * (np.asarray(c, np.float64) - 1.0)
           for c in (g.x, g.y, g.z)]
    gas = W._species(pos, [g.vx, g.vy, g.vz], g.m,
                     h=0.3 * np.asarray(g.h, np.float64), u=g.u)
    empty = W._species([np.zeros(0)] * 3, [np.zeros(0)] * 3, np.zeros(0))
    return W._single_box("two_clumps", gas, empty, float(base.r_c[0]),
                         float(base.eps[0]), {}), half


@pytest.mark.parametrize("case", ["one_bin", "two_clumps"])
def test_compatible_cycle_conserves_energy(orc, step_cls, case):
    print(f"case compatible cycle energy {case}", flush=True)
    params = dict(orc.PARAMS, G=0.0)
    if case == "one_bin":
        wl = W.random_uniform(20000, 0, 611, n_ngb=48.0, clustered=True)
        bg = np.full(wl.gas.n, 2)
    else:
        wl, half = _two_clumps(612, 20000)
        assert 2 * float(np.max(wl.gas.h)) < 0.2
        bg = np.where(np.arange(wl.gas.n) < half, 0, 2)
    L = 2
    bd = np.zeros(0, np.int64)
    g = wl.gas
    s0 = dict(vg=np.array([g.vx, g.vy, g.vz], np.float64),
              u=np.asarray(g.u, np.float64))
    E0 = _energy(wl, s0)
    res = {}
    for comp in (True, False):
        st = step_cls(wl, "fp64", params=params, compatible=comp)
        st.run()
        a = np.abs(st.outputs()["a_hydro"]).max()
        dt = 0.4 * np.abs(s0["vg"]).max() / a
        st.set_bins(bg, bd)
        st.substep_cycle(dt, L)
        res[comp] = _energy(wl, st.state())
        st.close()
    print(f"relative energy change: compatible {(res[True] - E0) / E0:.2e}, "
          f"plain {(res[False] - E0) / E0:.2e}", flush=True)
    assert abs(res[True] - E0) < 1e-12 * E0
    assert abs(res[False] - E0) > 1e-7 * E0


def test_compatible_block_checks_the_selection(step_cls):
    """The pass writes the particles crk_tree_set_active selected: a kick
    for another substep is refused."""
    from paper_2510_03557_amd import binding
    wl = W.random_uniform(3000, 2000, 613, n_ngb=40.0)
    st = step_cls(wl, "fp32", compatible=True)
    st.run()
    L = 2
    bg = np.zeros(wl.gas.n, np.int32)
    bg[::2] = 2
    st.set_bins(bg, np.zeros(wl.dm.n, np.int32))
    c, t = st.ctx, st.tree
    c.tree_set_active(t, st.bins_g, st.bins_d, L, 1)
    c.build_interaction_lists(t)
    for s in (0, -1):
        with pytest.raises(binding.CrkError) as e:
            st._compatible_block(0.01, L, s)
        assert e.value.status == binding.CRK_ESTATE
    st._compatible_block(0.01, L, 1)
    with pytest.raises(binding.CrkError) as e:
        st._compatible_block(0.01, L, 4)
    assert e.value.status == binding.CRK_EINVAL
    c.tree_set_active(t, None, None, 0, -1)
    st.sync()
