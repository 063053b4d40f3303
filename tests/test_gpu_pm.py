"""GPU parity of the long-range mesh gravity (crk_pm_gravity) against the
oracle's particle-mesh solver (same steps in float64 numpy), through the C
ABI.  Tolerance: relative RMS <= 1e-5 (float32 path: float32 mesh and
FFTs), 1e-10 (float64 path)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_03557_amd import workloads as W  # noqa: E402


def rel_rms(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b))


@pytest.fixture()
def step_cls():
    from paper_2510_03557_amd.step import ShortRangeStep
    made = []

    def make(*a, **k):
        st = ShortRangeStep(*a, **k)
        made.append(st)
        return st

    yield make
    for st in made:
        st.close()
    torch.cuda.synchronize()


def _oracle(orc, wl, n_mesh):
    g, d = wl.gas, wl.dm
    X = np.concatenate([g.x, d.x])
    Y = np.concatenate([g.y, d.y])
    Z = np.concatenate([g.z, d.z])
    M = np.concatenate([g.m, d.m])
    a = orc.pm_long_range(X, Y, Z, M, n_mesh, float(wl.r_c[0]))
    return a[:, :g.n], a[:, g.n:]


@pytest.mark.parametrize("precision,n_mesh,ng,nd,seed,clustered", [
    ("fp32", 32, 3000, 2500, 801, False), ("fp32", 64, 5000, 4000, 802, True),
    ("fp64", 32, 3000, 2500, 803, True), ("fp32", 48, 0, 6000, 804, False)])
def test_pm_matches_oracle(orc, step_cls, precision, n_mesh, ng, nd, seed,
                           clustered):
    print(f"case pm {precision} mesh {n_mesh} random({ng},{nd}) "
          f"clustered={clustered}", flush=True)
    wl = W.random_uniform(ng, nd, seed, r_c=6.0 / n_mesh, clustered=clustered)
    st = step_cls(wl, precision)
    g, d = st.pm_gravity(n_mesh)
    rg, rd = _oracle(orc, wl, n_mesh)
    tol = 1e-5 if precision == "fp32" else 1e-10
    errs = {}
    if ng:
        errs["gas"] = rel_rms(g, rg)
    errs["dm"] = rel_rms(d, rd)
    print({k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert all(v <= tol for v in errs.values()), errs
    # momentum: sum m a = 0 up to rounding
    mg = np.asarray(wl.gas.m, np.float64)
    md = np.asarray(wl.dm.m, np.float64)
    tot = (g * mg).sum(1) + (d * md).sum(1)
    scale = (np.abs(g) * mg).sum() + (np.abs(d) * md).sum()
    assert np.max(np.abs(tot)) <= (1e-5 if precision == "fp32" else 1e-12) * scale


def test_pm_lattice32(orc, step_cls):
    """65,536 particles on a jittered lattice, 64^3 mesh (r_c = 3/32 = 6
    cells)."""
    print("case pm lattice32 mesh 64", flush=True)
    wl = W.make("lattice32")
    st = step_cls(wl, "fp32")
    g, d = st.pm_gravity(64)
    rg, rd = _oracle(orc, wl, 64)
    e = (rel_rms(g, rg), rel_rms(d, rd))
    print(f"{e[0]:.2e} {e[1]:.2e}", flush=True)
    assert max(e) <= 1e-5


def test_pm_benchmark_box(orc, step_cls):
    """The benchmark box (4,194,304 particles) on its 256^3 mesh (r_c = 6
    cells), every particle compared."""
    print("case pm zeldovich128 mesh 256", flush=True)
    wl = W.make("zeldovich128")
    st = step_cls(wl, "fp32")
    g, d = st.pm_gravity()
    assert st.pm_gas is not None
    rg, rd = _oracle(orc, wl, 256)
    e = (rel_rms(g, rg), rel_rms(d, rd))
    print(f"{e[0]:.2e} {e[1]:.2e}", flush=True)
    assert max(e) <= 1e-5
