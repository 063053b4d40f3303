"""The allocation-free density entry point (crk_density_noalloc) against
crk_density, through the C ABI: two calls in a row on one GPU, the second
with a smaller input (the static scratch keeps the first call's contents,
which must not leak into the second), in both precisions; and the host-side
rejection of a tree with more gas particles than the scratch holds."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2510_03557_amd import workloads as W  # noqa: E402


def _density_both(st):
    """(crk_density outputs, crk_density_noalloc outputs) on the step's
    tree, as host arrays."""
    c, t = st.ctx, st.tree
    with torch.cuda.stream(c.stream):
        V0 = torch.full_like(st.V, -1.0)
        r0 = torch.full_like(st.rho_t, -1.0)
        V1 = torch.full_like(st.V, -2.0)
        r1 = torch.full_like(st.rho_t, -2.0)
    c.stream.synchronize()
    c.density(t, st.gm, V0, r0)
    c.density_noalloc(t, st.gm, V1, r1)
    c.sync()
    n = st.ng
    return ((V0[:n].cpu().numpy(), r0[:n].cpu().numpy()),
            (V1[:n].cpu().numpy(), r1[:n].cpu().numpy()))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_density_noalloc_equals_density_twice(orc, precision):
    from paper_2510_03557_amd.step import ShortRangeStep
    ref_tol = 1e-5 if precision == "fp32" else 1e-10
    for ng, nd, seed in ((40000, 30000, 901), (3000, 2000, 902)):
        print(f"case density_noalloc {precision} random_uniform({ng},{nd},"
              f"{seed})", flush=True)
        wl = W.random_uniform(ng, nd, seed, n_ngb=48.0, h_spread=0.15)
        st = ShortRangeStep(wl, precision=precision)
        try:
            st.run(passes=())  # tree and lists only
            st.sync()
            (V0, r0), (V1, r1) = _density_both(st)
        finally:
            st.close()
        # the same kernels on the same inputs: the same bits
        assert np.array_equal(V0, V1)
        assert np.array_equal(r0, r1)
        ref = orc.step(wl, passes=("density",))
        for a, b in ((V1, ref["V"]), (r1, ref["rho_tilde"])):
            err = np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b))
            assert err <= ref_tol, err


def test_density_noalloc_rejects_more_gas_than_its_scratch():
    from paper_2510_03557_amd.binding import CrkError, CRK_EINVAL, load
    from paper_2510_03557_amd.step import ShortRangeStep
    limit = 2097152  # CRK_NOALLOC_MAX_GAS
    print("case density_noalloc above its scratch", flush=True)
    wl = W.random_uniform(limit + 1, 0, 903, h_rule="global", n_ngb=32.0)
    st = ShortRangeStep(wl, precision="fp32")
    try:
        st.run(passes=())
        st.sync()
        with pytest.raises(CrkError) as e:
            st.ctx.density_noalloc(st.tree, st.gm, st.V, st.rho_t)
        assert e.value.status == CRK_EINVAL
        assert "scratch" in str(e.value)
        st.sync()
    finally:
        st.close()
    assert load() is not None
