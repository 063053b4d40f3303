"""GPU parity of the compatible energy update (crk_hydro_energy_compatible
before crk_integrate) against the FP64 oracle, through the C ABI.

Tolerances as for the rest of the step: relative RMS <= 1e-5 per output for
the float32 path, 1e-10 for the float64 path (the state changes over the
step are compared, not the states themselves).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_03557_amd import workloads as W  # noqa: E402

FP32_TOL = 1e-5
FP64_TOL = 1e-10


def rel_rms(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.sqrt(np.sum(b * b))
    num = np.sqrt(np.sum((a - b) ** 2))
    return num / den if den > 0 else num


@pytest.fixture(scope="module")
def step_cls():
    from paper_2510_03557_amd.step import ShortRangeStep
    assert torch.cuda.is_available()
    return ShortRangeStep


def kick_dt(wl, ref):
    v = np.abs(np.array([wl.gas.vx, wl.gas.vy, wl.gas.vz], np.float64)).max()
    a = np.abs(ref["a_hydro"] + ref["a_grav_gas"]).max()
    return 0.2 * v / a


@pytest.mark.parametrize("seed,ng,nd,recon,precision", [
    (801, 3000, 2000, False, "fp64"), (802, 4000, 1000, True, "fp64"),
    (803, 3000, 2000, False, "fp32"), (804, 5000, 2000, True, "fp32")])
def test_compatible_step_matches_oracle(orc, step_cls, seed, ng, nd, recon,
                                        precision):
    print(f"case compatible step random_uniform({ng},{nd},{seed}) "
          f"recon={recon} {precision}", flush=True)
    wl = W.random_uniform(ng, nd, seed, n_ngb=48.0, h_spread=0.15,
                          clustered=True)
    ref = orc.step(wl, recon=recon)
    dt = kick_dt(wl, ref)
    r = orc.compatible_update(wl, ref, dt, recon=recon)
    st = step_cls(wl, precision=precision, dt=dt, recon=recon,
                  compatible=True)
    try:
        st.run(integrate=True)
        got = st.state()
        out = st.outputs()
    finally:
        st.close()
    g = wl.gas
    v0 = np.array([g.vx, g.vy, g.vz], np.float64)
    u0 = np.asarray(g.u, np.float64)
    errs = dict(dudt=rel_rms(out["dudt"], r["dudt"]),
                du=rel_rms(got["u"] - u0, r["u1"] - u0),
                dv=rel_rms(got["vg"] - v0, r["v1"] - v0))
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    # the rate differs from the plain one (the test is not vacuous)
    assert rel_rms(r["dudt"], ref["dudt"]) > 1e-3


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_tiny_and_empty_boxes(orc, step_cls, precision):
    """Boxes with one, two, three or no gas particles (a lone particle, and
    singular moments: the degenerate coefficient branch feeds the gradient
    and the limiter) and an empty box, batched with ordinary ones, with the
    reconstruction and the compatible update."""
    print(f"case compatible + recon tiny and empty boxes {precision}",
          flush=True)
    sizes = [(1, 0), (0, 1), (0, 0), (2, 1), (3, 2), (40, 30), (2000, 1500)]
    boxes = [W.random_uniform(n, m, 1750 + k, n_ngb=20.0 if n < 100 else 48.0,
                              h_spread=0.15,
                              h_rule="knn" if n > 22 else "global")
             for k, (n, m) in enumerate(sizes)]
    wl = W.concat_boxes("tiny", boxes)
    ref = orc.step(wl, recon=True)
    assert (ref["degenerate"][:6] == 1).all()
    dt = kick_dt(wl, ref)
    r = orc.compatible_update(wl, ref, dt, recon=True)
    st = step_cls(wl, precision=precision, dt=dt, recon=True,
                  compatible=True)
    try:
        st.run(integrate=True)
        got = st.state()
        out = st.outputs()
    finally:
        st.close()
    g = wl.gas
    v0 = np.array([g.vx, g.vy, g.vz], np.float64)
    u0 = np.asarray(g.u, np.float64)
    errs = dict(dv=rel_rms(out["dv"], ref["dv"]),
                a_hydro=rel_rms(out["a_hydro"], ref["a_hydro"]),
                dudt=rel_rms(out["dudt"], r["dudt"]),
                du=rel_rms(got["u"] - u0, r["u1"] - u0),
                dvel=rel_rms(got["vg"] - v0, r["v1"] - v0))
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad
    # a lone gas particle: no neighbour, no gradient, no force
    assert np.all(out["dv"][0] == 0) and np.all(out["a_hydro"][:, 0] == 0)


def test_hydro_kick_conserves_energy_fp64(step_cls):
    """Hydro forces alone (no gravity in the kick): the compatible rate from
    the GPU makes sum m (v^2/2 + u) constant to rounding."""
    print("case compatible energy conservation fp64", flush=True)
    wl = W.random_uniform(4000, 0, 811, n_ngb=48.0, h_spread=0.15,
                          clustered=True)
    st = step_cls(wl, precision="fp64")
    try:
        st.run(passes=("density", "coefficients", "hydro"))
        c, t = st.ctx, st.tree
        # (outputs() waits for the library's stream)
        a = st.outputs()["a_hydro"]
        with torch.cuda.stream(c.stream):
            zeros = [torch.zeros_like(st.ahx) for _ in range(3)]
        c.stream.synchronize()
        g = wl.gas
        v = np.array([g.vx, g.vy, g.vz], np.float64)
        dt = 0.2 * np.abs(v).max() / np.abs(a).max()
        c.hydro_energy_compatible(t, st.gm, st.gvx, st.gvy, st.gvz, st.V,
                                  st.rho, st.P, st.cs, st.A, st.B, st.gA,
                                  st.gB, None, 0.8, 0.2, dt, zeros,
                                  (st.ahx, st.ahy, st.ahz), st.dudt)
        dudt = st.outputs()["dudt"]
        c.hydro_forces(t, st.gm, st.gvx, st.gvy, st.gvz, st.V, st.rho, st.P,
                       st.cs, st.A, st.B, st.gA, st.gB, st.ahx, st.ahy,
                       st.ahz, st.dudt)
        plain = st.outputs()["dudt"]
    finally:
        st.close()
    m = g.m.astype(np.float64)
    u = g.u.astype(np.float64)
    v1 = v + dt * a
    E0 = 0.5 * (m * (v * v).sum(0)).sum() + (m * u).sum()
    E1 = 0.5 * (m * (v1 * v1).sum(0)).sum() + (m * (u + dt * dudt)).sum()
    E1p = 0.5 * (m * (v1 * v1).sum(0)).sum() + (m * (u + dt * plain)).sum()
    print(f"relative energy change: compatible {(E1 - E0) / E0:.2e}, plain "
          f"{(E1p - E0) / E0:.2e}", flush=True)
    assert abs(E1 - E0) < 1e-12 * E0
    assert abs(E1p - E0) > 1e-7 * E0


@pytest.mark.parametrize("recon", [False, True])
def test_no_kick_gives_the_force_pass_rate_bitwise(step_cls, recon):
    """dt = 0: v1 = v, the centred velocity difference is the actual one
    and the compatible pass returns the force pass's du/dt to the bit."""
    print(f"case compatible dt=0 recon={recon}", flush=True)
    wl = W.random_uniform(3000, 1000, 841, n_ngb=48.0, h_spread=0.15,
                          clustered=True)
    st = step_cls(wl, precision="fp32", recon=recon)
    try:
        st.run()
        ref = st.outputs()["dudt"]
        c, t = st.ctx, st.tree
        c.hydro_energy_compatible(t, st.gm, st.gvx, st.gvy, st.gvz, st.V,
                                  st.rho, st.P, st.cs, st.A, st.B, st.gA,
                                  st.gB, st.dv if recon else None, 0.8, 0.2,
                                  0.0, (st.agx, st.agy, st.agz),
                                  (st.ahx, st.ahy, st.ahz), st.dudt)
        got = st.outputs()["dudt"]
    finally:
        st.close()
    assert np.array_equal(got, ref)


def test_compatible_graph_replay_equals_eager(step_cls):
    """Two steps with the compatible update: eager, and one eager step plus
    a captured step replayed, give the same state to the last bit."""
    print("case compatible graph replay fp32", flush=True)
    wl = W.random_uniform(3000, 2000, 821, n_ngb=48.0, h_spread=0.15)
    kw = dict(precision="fp32", dt=2e-3, recon=True, compatible=True)
    a = step_cls(wl, **kw)
    b = step_cls(wl, **kw)
    try:
        a.run(integrate=True)
        a.run(integrate=True)
        sa = a.state()
        b.capture(integrate=True)
        b.replay()
        sb = b.state()
    finally:
        a.close()
        b.close()
    for k in ("xg", "vg", "u", "xd", "vd"):
        assert np.array_equal(sa[k], sb[k]), k


def test_compatible_argument_errors(step_cls):
    from paper_2510_03557_amd.binding import CrkError, CRK_EINVAL
    print("case compatible argument errors", flush=True)
    wl = W.random_uniform(500, 0, 831, n_ngb=48.0)
    st = step_cls(wl, precision="fp32")
    try:
        st.run()
        c, t = st.ctx, st.tree
        ag = (st.agx, st.agy, st.agz)
        base = (t, st.gm, st.gvx, st.gvy, st.gvz, st.V, st.rho, st.P, st.cs,
                st.A, st.B, st.gA, st.gB)
        for dv, ec, ef, dt, a in ((None, 0.8, 0.2, float("inf"), ag),
                                  (None, 0.8, 0.2, 1e-3, None),
                                  (st.dv, 0.8, 0.0, 1e-3, ag)):
            with pytest.raises(CrkError) as e:
                c.hydro_energy_compatible(*base, dv, ec, ef, dt, a, None,
                                          st.dudt)
            assert e.value.status == CRK_EINVAL
        # the block form: bins required, dt > 0, substep in [-1, 2^L)
        bins = torch.zeros(wl.gas.n, dtype=torch.int32, device="cuda")
        for L, s, dt, b in ((1, 0, 1e-3, None), (1, -1, 0.0, bins),
                            (1, 2, 1e-3, bins), (31, 0, 1e-3, bins)):
            with pytest.raises(CrkError) as e:
                c.hydro_energy_compatible_block(*base, None, 0.8, 0.2, dt, L,
                                                b, s, ag, None, st.dudt)
            assert e.value.status == CRK_EINVAL
        st.sync()
    finally:
        st.close()
