"""GPU friends-of-friends groups (crk_fof) against the oracle, through the
C ABI: labels are integers (the smallest combined caller index of each
group), compared bit for bit."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_03557_amd import workloads as W  # noqa: E402


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


def _oracle_labels(orc, wl, b):
    """Per box, labels in the combined caller index space (all gas of all
    boxes first, then all dark matter)."""
    g, d = wl.gas, wl.dm
    ng = g.n
    lg = np.zeros(ng, np.int64)
    ld = np.zeros(d.n, np.int64)
    for k in range(wl.n_boxes):
        gs = slice(int(wl.gas_off[k]), int(wl.gas_off[k + 1]))
        ds = slice(int(wl.dm_off[k]), int(wl.dm_off[k + 1]))
        idx = np.concatenate([np.arange(gs.start, gs.stop),
                              ng + np.arange(ds.start, ds.stop)])
        if idx.size == 0:
            continue
        X = np.concatenate([g.x[gs], d.x[ds]])
        Y = np.concatenate([g.y[gs], d.y[ds]])
        Z = np.concatenate([g.z[gs], d.z[ds]])
        loc = orc.fof_labels(X, Y, Z, b)
        lab = idx[loc]
        k_g = gs.stop - gs.start
        lg[gs] = lab[:k_g]
        ld[ds] = lab[k_g:]
    return lg, ld


def _check(orc, st, wl, b):
    st.run()
    lg, ld = st.fof(b)
    rg, rd = _oracle_labels(orc, wl, b)
    n_groups = len(np.unique(np.concatenate([rg, rd])))
    sizes = np.bincount(np.concatenate([rg, rd]))
    print(f"groups {n_groups}, largest {sizes.max()}", flush=True)
    assert np.array_equal(lg, rg) and np.array_equal(ld, rd)
    return n_groups, sizes.max()


@pytest.mark.parametrize("precision,ng,nd,seed,clustered,frac", [
    ("fp32", 6000, 5000, 901, False, 0.6), ("fp32", 8000, 6000, 902, True, 0.2),
    ("fp64", 5000, 4000, 903, True, 0.3), ("fp32", 0, 9000, 904, False, 0.7)])
def test_fof_matches_oracle(orc, step_cls, precision, ng, nd, seed, clustered,
                            frac):
    wl = W.random_uniform(ng, nd, seed, n_ngb=48.0, clustered=clustered)
    b = frac * (ng + nd) ** (-1.0 / 3.0)
    print(f"case fof {precision} random({ng},{nd}) clustered={clustered} "
          f"b={b:.4g}", flush=True)
    st = step_cls(wl, precision)
    n_groups, largest = _check(orc, st, wl, b)
    assert 1 < n_groups < ng + nd and largest > 2


def test_fof_batched_boxes(orc, step_cls):
    """Groups never cross boxes; every box labelled in the combined index
    space."""
    boxes = [W.random_uniform(1500 + 300 * k, 1200, 910 + k, n_ngb=48.0,
                              clustered=k % 2 == 1) for k in range(4)]
    wl = W.concat_boxes("fof_batch", boxes)
    b = 0.5 * 2700 ** (-1.0 / 3.0)
    print(f"case fof batch of 4 boxes b={b:.4g}", flush=True)
    st = step_cls(wl, "fp32")
    _check(orc, st, wl, b)


def test_fof_benchmark_box(orc, step_cls):
    """The benchmark box (4,194,304 particles), linking length 0.2 of the
    mean spacing."""
    wl = W.make("zeldovich128")
    b = 0.2 * wl.n_total ** (-1.0 / 3.0)
    print(f"case fof zeldovich128 b={b:.4g}", flush=True)
    st = step_cls(wl, "fp32")
    _check(orc, st, wl, b)


def test_fof_argument_errors(step_cls):
    from paper_2510_03557_amd.binding import CrkError, CRK_EINVAL
    wl = W.random_uniform(1000, 1000, 920)
    st = step_cls(wl, "fp32")
    st.run()
    with pytest.raises(CrkError) as e:
        st.fof(float(wl.r_c[0]) * 1.5)  # beyond the gravity lists' range
    assert e.value.status == CRK_EINVAL
    with pytest.raises(CrkError):
        st.fof(0.0)


# ---------------------------------------------------------------------------
# group properties
# ---------------------------------------------------------------------------

def _check_properties(orc, st, wl, b):
    st.run()
    lg, ld, cnt, mass, cen = st.fof_properties(b)
    rg, rd = _oracle_labels(orc, wl, b)
    assert np.array_equal(lg, rg) and np.array_equal(ld, rd)
    g, d = wl.gas, wl.dm
    X, Y, Z, M = (np.concatenate([getattr(g, k), getattr(d, k)]).astype(
        np.float64) for k in ("x", "y", "z", "m"))
    rc, rm, rcen = orc.fof_properties(X, Y, Z, M, np.concatenate([rg, rd]))
    assert np.array_equal(cnt.astype(np.int64), rc)
    assert np.abs(mass - rm).max() <= 1e-12 * np.abs(rm).max()
    dd = cen - rcen
    dd -= np.round(dd)
    print(f"groups {np.count_nonzero(rc)}, largest {rc.max()}, centre error "
          f"{np.abs(dd).max():.2e}", flush=True)
    assert np.abs(dd).max() < 1e-12
    assert rc.max() > 5


@pytest.mark.parametrize("precision,ng,nd,seed,frac", [
    ("fp32", 8000, 6000, 931, 0.25), ("fp64", 5000, 4000, 932, 0.3)])
def test_fof_properties_match_oracle(orc, step_cls, precision, ng, nd, seed,
                                     frac):
    wl = W.random_uniform(ng, nd, seed, n_ngb=48.0, clustered=True)
    b = frac * (ng + nd) ** (-1.0 / 3.0)
    print(f"case fof properties {precision} random({ng},{nd}) b={b:.4g}",
          flush=True)
    _check_properties(orc, step_cls(wl, precision), wl, b)


def test_fof_properties_batched_boxes(orc, step_cls):
    boxes = [W.random_uniform(1500 + 300 * k, 1200, 940 + k, n_ngb=48.0,
                              clustered=True) for k in range(4)]
    wl = W.concat_boxes("fof_props_batch", boxes)
    b = 0.4 * 2700 ** (-1.0 / 3.0)
    print(f"case fof properties batch of 4 boxes b={b:.4g}", flush=True)
    _check_properties(orc, step_cls(wl, "fp32"), wl, b)


def test_fof_properties_reject_foreign_labels(step_cls):
    """A label outside the particle range is skipped on the device (no
    access out of bounds) and reported by crk_sync."""
    from paper_2510_03557_amd.binding import CrkError, CRK_EINVAL
    print("case fof properties foreign label", flush=True)
    wl = W.random_uniform(500, 400, 950)
    st = step_cls(wl, "fp32")
    st.run()
    c = st.ctx
    n = wl.n_total
    with torch.cuda.stream(c.stream):
        lg = torch.arange(500, dtype=torch.int32, device="cuda")
        ld = torch.arange(500, 900, dtype=torch.int32, device="cuda")
        ld[7] = n + 5
        cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
        mass = torch.zeros(n, dtype=torch.float64, device="cuda")
        cen = torch.zeros(3 * n, dtype=torch.float64, device="cuda")
    c.fof_properties(500, 400, lg, ld, (st.gx, st.gy, st.gz), st.gm,
                     (st.dx, st.dy, st.dz), st.dm, cnt, mass, cen)
    with pytest.raises(CrkError) as e:
        st.sync()
    assert e.value.status == CRK_EINVAL
    c.stream.synchronize()
    assert int(cnt.sum().item()) == n - 1
