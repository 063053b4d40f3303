"""GPU parity of the velocity gradient and of the hydro forces with the
viscosity on the limited midpoint reconstruction (crk_velocity_gradient,
crk_hydro_forces_limited) against the FP64 oracle, through the C ABI.

Tolerances as for the rest of the step: relative RMS <= 1e-5 per output for
the float32 path, 1e-10 for the float64 path.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_03557_amd import workloads as W  # noqa: E402

FP32_TOL = 1e-5
FP64_TOL = 1e-10
KEYS = ("V", "A", "B", "gradA", "gradB", "rho", "P", "cs", "dv", "a_hydro",
        "dudt")
F32 = np.float32


def rel_rms(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.sqrt(np.sum(b * b))
    num = np.sqrt(np.sum((a - b) ** 2))
    return num / den if den > 0 else num


def compare(got, ref, tol, keys=KEYS):
    errs = {}
    for k in keys:
        errs[k] = rel_rms(got[k], ref[k])
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, bad


@pytest.fixture(scope="module")
def step_cls():
    from paper_2510_03557_amd.step import ShortRangeStep
    assert torch.cuda.is_available()
    return ShortRangeStep


def run(step_cls, wl, precision, **kw):
    st = step_cls(wl, precision=precision, recon=True, **kw)
    try:
        st.run()
        return st.outputs()
    finally:
        st.close()


@pytest.mark.parametrize("seed,ng,nd,clustered,precision", [
    (701, 3000, 1000, False, "fp64"), (702, 5000, 0, True, "fp64"),
    (703, 3000, 2000, False, "fp32"), (704, 6000, 1000, True, "fp32"),
    (705, 700, 300, False, "fp32")])
def test_small_matches_oracle(orc, step_cls, seed, ng, nd, clustered,
                              precision):
    print(f"case recon random_uniform({ng},{nd},{seed},clustered={clustered})"
          f" {precision}", flush=True)
    wl = W.random_uniform(ng, nd, seed, n_ngb=48.0, h_spread=0.15,
                          clustered=clustered)
    got = run(step_cls, wl, precision)
    ref = orc.step(wl, passes=("density", "coefficients", "hydro"), recon=True)
    compare(got, ref, FP64_TOL if precision == "fp64" else FP32_TOL)


def test_passes_with_oracle_inputs_fp32(orc, step_cls):
    """Each of the two calls fed with the oracle's own float32-rounded
    inputs (isolates the gradient pass and the limited force pass)."""
    print("case recon per-pass random_uniform(4000,0,711) fp32", flush=True)
    wl = W.random_uniform(4000, 0, 711, n_ngb=48.0, h_spread=0.15,
                          clustered=True)
    g = wl.gas
    ref = orc.step(wl, passes=("density", "coefficients"))
    c32 = {k: np.asarray(ref[k], F32) for k in
           ("V", "A", "B", "gradA", "gradB", "rho", "P", "cs")}
    c64 = {k: v.astype(np.float64) for k, v in c32.items()}
    dv_ref = orc.velocity_gradient(g.x, g.y, g.z, g.vx, g.vy, g.vz, g.h,
                                   c64["V"], c64["A"], c64["B"], c64["gradA"],
                                   c64["gradB"])
    st = step_cls(wl, precision="fp32", recon=True)
    try:
        st.run(passes=())
        st.set_inputs(V=c32["V"], A=c32["A"], B=c32["B"].T.ravel(),
                      gA=c32["gradA"].T.ravel(),
                      gB=c32["gradB"].transpose(1, 2, 0).ravel(),
                      rho=c32["rho"], P=c32["P"], cs=c32["cs"])
        c, t = st.ctx, st.tree
        c.velocity_gradient(t, st.gvx, st.gvy, st.gvz, st.V, st.A, st.B,
                            st.gA, st.gB, st.dv)
        got = st.outputs()
        compare(got, {"dv": dv_ref}, FP32_TOL, ("dv",))
        dv32 = dv_ref.astype(F32)
        st.set_inputs(dv=dv32.transpose(1, 2, 0).ravel())
        c.hydro_forces_limited(t, st.gm, st.gvx, st.gvy, st.gvz, st.V, st.rho,
                               st.P, st.cs, st.A, st.B, st.gA, st.gB, st.dv,
                               0.8, 0.2, st.ahx, st.ahy, st.ahz, st.dudt)
        got = st.outputs()
    finally:
        st.close()
    ax, ay, az, du = orc.hydro(g.x, g.y, g.z, g.vx, g.vy, g.vz, g.h, g.m,
                               c64["V"], c64["rho"], c64["P"], c64["cs"],
                               c64["A"], c64["B"], c64["gradA"], c64["gradB"],
                               dv=dv32.astype(np.float64))
    compare(got, {"a_hydro": np.stack([ax, ay, az]), "dudt": du}, FP32_TOL,
            ("a_hydro", "dudt"))


def lattice_patch_workload(k=10, spacing=1.0 / 64, lo=1.25):
    """A k^3 lattice patch (exact float32 positions) with a linear,
    compressive, non-symmetric velocity field and h = 1.2 spacings."""
    M = np.array([[-0.8, 0.3, 0.1], [0.5, 0.2, -0.4], [0.05, -0.6, -0.3]])
    i = lo + spacing * np.arange(k)
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    n = P.shape[1]
    v = M @ (P - 1.5)
    gas = W.Species(x=P[0].astype(F32), y=P[1].astype(F32),
                    z=P[2].astype(F32), vx=v[0].astype(F32),
                    vy=v[1].astype(F32), vz=v[2].astype(F32),
                    m=np.full(n, 1.0 / n, F32),
                    h=np.full(n, 1.2 * spacing, F32), u=np.ones(n, F32))
    e = np.zeros(0, F32)
    dm = W.Species(x=e, y=e, z=e, vx=e, vy=e, vz=e, m=e)
    wl = W.Workload(name="lattice-patch", gas=gas, dm=dm,
                    gas_off=np.array([0, n], np.int64),
                    dm_off=np.array([0, 0], np.int64),
                    r_c=np.array([3.0 / 64]), eps=np.array([3.0 / 64 / 60]))
    return wl, M


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_linear_flow_patch(orc, step_cls, precision):
    """Edges and corners of a lattice patch: the gradient of the linear flow
    comes back on the GPU too, and the forces match the oracle's."""
    print(f"case recon lattice patch {precision}", flush=True)
    wl, M = lattice_patch_workload()
    got = run(step_cls, wl, precision)
    ref = orc.step(wl, passes=("density", "coefficients", "hydro"), recon=True)
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    compare(got, ref, tol)
    assert rel_rms(got["dv"], np.broadcast_to(M, got["dv"].shape)) < 1e-5


def test_zeldovich128_fp32_graph(orc, step_cls):
    """The benchmark box in full, captured in a graph and replayed, with the
    reconstruction, against one oracle step with the reconstruction."""
    print("case recon zeldovich128 (4,194,304 particles) fp32, graph replay",
          flush=True)
    wl = W.make("zeldovich128")
    ref = orc.step(wl, passes=("density", "coefficients", "hydro"), recon=True)
    st = step_cls(wl, precision="fp32", recon=True)
    try:
        st.capture(integrate=False)
        st.replay()
        compare(st.outputs(), ref, FP32_TOL)
    finally:
        st.close()


@pytest.mark.parametrize("tuning", [dict(grid_mult=16), dict(xcd_remap=1),
                                    dict(walk_mask=1 << 2),
                                    dict(grid_mult=8, leaf_max=128)])
def test_launch_shapes_are_bitwise_identical(step_cls, tuning):
    """The queue, the XCD remap and the per-lane hit walk change only which
    workgroup or lane runs a leaf: the gradient and the reconstructed forces
    are bitwise those of one workgroup per leaf with the broadcast sweep."""
    print(f"case recon launch shape {tuning}", flush=True)
    wl = W.random_uniform(6000, 3000, 1601, n_ngb=48.0, clustered=True)
    L = tuning.get("leaf_max", 64)
    base = dict(leaf_max=L, sub_sweep=0, xcd_remap=0)
    ref = run(step_cls, wl, "fp32", tuning=base)
    got = run(step_cls, wl, "fp32", tuning=dict(base, **tuning))
    for k in ("dv", "a_hydro", "dudt"):
        assert np.array_equal(ref[k], got[k]), k


def test_sub_leaf_sweep_matches_whole_leaf_sweep(orc, step_cls):
    """The benchmark's split sweep (a wavefront per sub-leaf) against the
    whole-leaf sweep: only the summation order differs."""
    print("case recon split sweep vs whole-leaf sweep fp32", flush=True)
    wl = W.random_uniform(6000, 3000, 1602, n_ngb=48.0, clustered=True)
    a = run(step_cls, wl, "fp32", tuning=dict(leaf_max=64, sub_sweep=0))
    b = run(step_cls, wl, "fp32", tuning=dict(leaf_max=64, sub_sweep=2))
    compare(b, a, 2e-6, ("dv", "a_hydro", "dudt"))


def test_argument_errors(step_cls):
    from paper_2510_03557_amd.binding import CrkError, CRK_EINVAL
    print("case recon argument errors", flush=True)
    wl = W.random_uniform(500, 0, 721, n_ngb=48.0)
    st = step_cls(wl, precision="fp32", recon=True)
    try:
        st.run()
        c, t = st.ctx, st.tree
        for ec, ef in ((0.8, 0.0), (-1.0, 0.2), (float("nan"), 0.2)):
            with pytest.raises(CrkError) as e:
                c.hydro_forces_limited(t, st.gm, st.gvx, st.gvy, st.gvz, st.V,
                                       st.rho, st.P, st.cs, st.A, st.B, st.gA,
                                       st.gB, st.dv, ec, ef, st.ahx, st.ahy,
                                       st.ahz, st.dudt)
            assert e.value.status == CRK_EINVAL
        with pytest.raises(CrkError) as e:
            c.velocity_gradient(t, st.gvx, st.gvy, st.gvz, st.V, st.A, st.B,
                                st.gA, st.gB, None)
        assert e.value.status == CRK_EINVAL
        st.sync()
    finally:
        st.close()
