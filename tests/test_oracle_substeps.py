"""Pins of the oracle's hierarchical time steps (adaptive integration in
timestep bins, Sec. IV-A; active leaves on a fixed tree, Sec. IV-B.1).

Each test checks the block kick-drift-kick cycle against something other
than itself: exact values of the bin rule at powers of two, free streaming
when nothing interacts, a plain uniform leapfrog when every particle shares
one bin, time reversibility of the gravity-only cycle, and the number of
force evaluations the bins imply.
"""
import dataclasses

import numpy as np
import pytest

from paper_2510_03557_amd import workloads as wl_mod


def _f64_copy(wl, xg=None, vg=None, u=None, xd=None, vd=None):
    """The workload with float64 state arrays (optionally replaced)."""
    g, d = wl.gas, wl.dm
    gas = dataclasses.replace(
        g,
        x=np.asarray(xg[0] if xg is not None else g.x, np.float64),
        y=np.asarray(xg[1] if xg is not None else g.y, np.float64),
        z=np.asarray(xg[2] if xg is not None else g.z, np.float64),
        vx=np.asarray(vg[0] if vg is not None else g.vx, np.float64),
        vy=np.asarray(vg[1] if vg is not None else g.vy, np.float64),
        vz=np.asarray(vg[2] if vg is not None else g.vz, np.float64),
        u=None if g.u is None else np.asarray(u if u is not None else g.u,
                                              np.float64))
    dm = dataclasses.replace(
        d,
        x=np.asarray(xd[0] if xd is not None else d.x, np.float64),
        y=np.asarray(xd[1] if xd is not None else d.y, np.float64),
        z=np.asarray(xd[2] if xd is not None else d.z, np.float64),
        vx=np.asarray(vd[0] if vd is not None else d.vx, np.float64),
        vy=np.asarray(vd[1] if vd is not None else d.vy, np.float64),
        vz=np.asarray(vd[2] if vd is not None else d.vz, np.float64))
    return dataclasses.replace(wl, gas=gas, dm=dm)


def _wrap(x):
    x = np.mod(x - 1.0, 1.0) + 1.0
    return np.where(x >= 2.0, x - 1.0, x)


def _periodic_close(a, b, tol):
    d = np.asarray(a) - np.asarray(b)
    d = d - np.round(d)
    return np.max(np.abs(d)) <= tol


# ---------------------------------------------------------------------------
# the bin rule
# ---------------------------------------------------------------------------

def test_bins_courant_at_powers_of_two(orc):
    """With a = 0 only the Courant condition tau cs <= c h counts: at
    cs dt / (c h) = 2^k exactly the bin is k (equality passes), just above
    it the bin is k + 1, and the deepest bin caps the rest."""
    c = 0.25
    h = np.array([0.5, 0.5, 0.5, 0.5, 0.5])
    dt = 1.0
    # dt cs / (c h) = 1, 4, 4(1 + 2^-40), 2^10, 1/8
    cs = c * h / dt * np.array([1.0, 4.0, 4.0 * (1 + 2.0 ** -40), 1024.0,
                                0.125])
    z = np.zeros(5)
    b = orc.timestep_bins(dt, 6, 0.01, z, z, z, h=h, cs=cs, c_cfl=c)
    assert b.tolist() == [0, 2, 3, 6, 0]


def test_bins_acceleration_at_powers_of_two(orc):
    """Without gas terms only tau^2 |a| <= 2 eta eps counts: |a| =
    2 eta eps / dt^2 * 4^k puts a particle in bin k exactly."""
    eta, eps, dt = 0.025, 1.0 / 64, 0.5
    k = np.array([0, 1, 3, 5])
    amag = 2 * eta * eps / dt ** 2 * 4.0 ** k
    # split the magnitude over three axes (3-4-12 triangle: |(3,4,12)| = 13)
    ax, ay, az = amag * 3 / 13, amag * 4 / 13, amag * 12 / 13
    b = orc.timestep_bins(dt, 8, eps, ax, ay, az, eta=eta)
    # the split can round |a| up by an ulp: then the bin is one deeper
    assert np.all((b == k) | (b == k + 1))
    b2 = orc.timestep_bins(dt, 8, eps, amag * 0.999999, 0 * amag, 0 * amag,
                           eta=eta)
    assert b2.tolist() == k.tolist()
    b3 = orc.timestep_bins(dt, 8, eps, amag * 1.000001, 0 * amag, 0 * amag,
                           eta=eta)
    assert b3.tolist() == (k + 1).tolist()


# ---------------------------------------------------------------------------
# the cycle
# ---------------------------------------------------------------------------

def _isolated(n_side=3, seed=5):
    """n_side^3 gas and dm sites 1/n_side apart with tiny h and r_c: no pair
    interacts (every gas particle has only itself in range)."""
    rng = np.random.default_rng(seed)
    i = (np.arange(n_side) + 0.5) / n_side
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    n = X.size
    pos = [X.ravel(), Y.ravel(), Z.ravel()]
    vel = [rng.standard_normal(n) for _ in range(3)]
    m = np.full(n, 1.0 / n)
    gas = wl_mod._species([p + 0.1 for p in pos], vel, m,
                          h=np.full(n, 0.01), u=np.ones(n))
    dm = wl_mod._species(pos, [-v for v in vel], m)
    return wl_mod._single_box("isolated", gas, dm, 0.02, 0.02 / 60, {})


def test_cycle_free_streaming(orc):
    """Nothing interacts: forces and du/dt vanish, so whatever the bins,
    x(t + dt) = x + v dt, v and u unchanged."""
    wl = _isolated()
    rng = np.random.default_rng(1)
    bg = rng.integers(0, 3, wl.gas.n)
    bd = rng.integers(0, 3, wl.dm.n)
    dt = 0.01
    out = orc.substep_cycle(wl, bg, bd, dt, 2)
    g, d = wl.gas, wl.dm
    xg = np.array([g.x, g.y, g.z], np.float64) + dt * np.array(
        [g.vx, g.vy, g.vz], np.float64)
    xd = np.array([d.x, d.y, d.z], np.float64) + dt * np.array(
        [d.vx, d.vy, d.vz], np.float64)
    assert _periodic_close(out["xg"], xg, 1e-14)
    assert _periodic_close(out["xd"], xd, 1e-14)
    assert np.array_equal(out["vg"], np.array([g.vx, g.vy, g.vz], np.float64))
    assert np.array_equal(out["u"], np.asarray(g.u, np.float64))
    assert np.all(out["a_hydro"] == 0) and np.all(out["a_grav_dm"] == 0)


def _uniform_leapfrog(orc, wl, tau, nsteps):
    """nsteps kick-drift-kick steps of tau for every particle, with full
    evaluations of the step (independent of the bin machinery)."""
    g, d = wl.gas, wl.dm
    xg = np.array([g.x, g.y, g.z], np.float64)
    vg = np.array([g.vx, g.vy, g.vz], np.float64)
    xd = np.array([d.x, d.y, d.z], np.float64)
    vd = np.array([d.vx, d.vy, d.vz], np.float64)
    u = np.asarray(g.u, np.float64).copy()

    def forces():
        w = _f64_copy(wl, _wrap(xg), vg, u, _wrap(xd), vd)
        return orc.step(w)

    s = forces()
    for _ in range(nsteps):
        vg += 0.5 * tau * (s["a_grav_gas"] + s["a_hydro"])
        u += 0.5 * tau * s["dudt"]
        vd += 0.5 * tau * s["a_grav_dm"]
        xg += tau * vg
        xd += tau * vd
        s = forces()
        vg += 0.5 * tau * (s["a_grav_gas"] + s["a_hydro"])
        u += 0.5 * tau * s["dudt"]
        vd += 0.5 * tau * s["a_grav_dm"]
    return _wrap(xg), vg, u, _wrap(xd), vd


@pytest.mark.parametrize("level,L", [(2, 2), (0, 2), (1, 1)])
def test_cycle_equal_bins_is_uniform_leapfrog(orc, level, L):
    """Every particle in bin `level` of a cycle with 2^L substeps: the cycle
    is 2^level plain leapfrog steps of dt / 2^level."""
    wl = wl_mod.jittered_lattice(5, seed=11)
    dt = 0.004
    bg = np.full(wl.gas.n, level)
    bd = np.full(wl.dm.n, level)
    out = orc.substep_cycle(wl, bg, bd, dt, L)
    xg, vg, u, xd, vd = _uniform_leapfrog(orc, wl, dt / 2 ** level,
                                          2 ** level)
    assert _periodic_close(out["xg"], xg, 1e-13)
    assert _periodic_close(out["xd"], xd, 1e-13)
    assert np.allclose(out["vg"], vg, rtol=0, atol=1e-11)
    assert np.allclose(out["vd"], vd, rtol=0, atol=1e-11)
    assert np.allclose(out["u"], u, rtol=1e-12, atol=0)


def test_cycle_gravity_time_reversible(orc):
    """Gravity only (no gas), mixed bins: one cycle forward, velocities
    flipped, one more cycle with the same bins, velocities flipped back,
    returns every particle to its start (block kick-drift-kick with fixed
    bins is time symmetric)."""
    base = wl_mod.jittered_lattice(6, seed=12)
    empty = wl_mod._species([np.zeros(0)] * 3, [np.zeros(0)] * 3,
                            np.zeros(0), h=np.zeros(0), u=np.zeros(0))
    wl = dataclasses.replace(base, gas=empty,
                             gas_off=np.array([0, 0], np.int64))
    # strong clustering of forces is not needed: raise the velocities so
    # the particles move a fraction of r_c in the cycle
    rng = np.random.default_rng(3)
    bd = rng.integers(0, 4, wl.dm.n)
    dt = 0.02
    out = orc.substep_cycle(wl, np.zeros(0, np.int64), bd, dt, 3)
    back = _f64_copy(wl, xd=out["xd"], vd=-out["vd"])
    out2 = orc.substep_cycle(back, np.zeros(0, np.int64), bd, dt, 3)
    x0 = np.array([wl.dm.x, wl.dm.y, wl.dm.z], np.float64)
    moved = out["xd"] - x0
    moved = moved - np.round(moved)
    assert np.max(np.abs(moved)) > 1e-3  # the test is not vacuous
    assert _periodic_close(out2["xd"], x0, 1e-12)
    assert np.allclose(-out2["vd"],
                       np.array([wl.dm.vx, wl.dm.vy, wl.dm.vz], np.float64),
                       rtol=0, atol=1e-12)


def test_cycle_evaluation_counts(orc):
    """A particle of bin b is evaluated once at the start and once at the
    end of each of its 2^b steps."""
    wl = wl_mod.jittered_lattice(4, seed=13)
    rng = np.random.default_rng(4)
    bg = rng.integers(0, 3, wl.gas.n)
    bd = rng.integers(0, 3, wl.dm.n)
    counts = {}
    orc.substep_cycle(wl, bg, bd, 0.001, 2, counts=counts)
    assert np.array_equal(counts["gas"], 1 + 2 ** bg)
    assert np.array_equal(counts["dm"], 1 + 2 ** bd)


def test_cycle_with_long_range_is_split_leapfrog(orc):
    """One level (L = 0) with the long-range mesh force coupled: the cycle
    is the split composition long half-kick, short-range kick-drift-kick of
    dt (forces evaluated after the long kick: the viscosity sees the kicked
    velocities), long half-kick at the new positions."""
    wl = wl_mod.jittered_lattice(5, seed=14)
    n_mesh = 2 * int(np.ceil(3.0 / float(wl.r_c[0])))
    dt = 0.004
    out = orc.substep_cycle(wl, np.zeros(wl.gas.n, np.int64),
                            np.zeros(wl.dm.n, np.int64), dt, 0,
                            pm_mesh=n_mesh)
    g, d = wl.gas, wl.dm
    xg = np.array([g.x, g.y, g.z], np.float64)
    vg = np.array([g.vx, g.vy, g.vz], np.float64)
    xd = np.array([d.x, d.y, d.z], np.float64)
    vd = np.array([d.vx, d.vy, d.vz], np.float64)
    u = np.asarray(g.u, np.float64).copy()

    def long_kick():
        X = np.concatenate([_wrap(xg), _wrap(xd)], axis=1)
        a = orc.pm_long_range(X[0], X[1], X[2], np.concatenate([g.m, d.m]),
                              n_mesh, float(wl.r_c[0]))
        vg[:] += 0.5 * dt * a[:, :g.n]
        vd[:] += 0.5 * dt * a[:, g.n:]

    def short():
        return orc.step(_f64_copy(wl, _wrap(xg), vg, u, _wrap(xd), vd))

    long_kick()
    s = short()
    vg += 0.5 * dt * (s["a_grav_gas"] + s["a_hydro"])
    vd += 0.5 * dt * s["a_grav_dm"]
    u += 0.5 * dt * s["dudt"]
    xg += dt * vg
    xd += dt * vd
    s = short()
    vg += 0.5 * dt * (s["a_grav_gas"] + s["a_hydro"])
    vd += 0.5 * dt * s["a_grav_dm"]
    u += 0.5 * dt * s["dudt"]
    long_kick()
    # the long-range kicks moved velocities noticeably
    no_long = orc.substep_cycle(wl, np.zeros(wl.gas.n, np.int64),
                                np.zeros(wl.dm.n, np.int64), dt, 0)
    assert np.max(np.abs(out["vd"] - no_long["vd"])) > 1e-4
    assert _periodic_close(out["xg"], _wrap(xg), 1e-13)
    assert _periodic_close(out["xd"], _wrap(xd), 1e-13)
    assert np.allclose(out["vg"], vg, rtol=0, atol=1e-11)
    assert np.allclose(out["vd"], vd, rtol=0, atol=1e-11)
    assert np.allclose(out["u"], u, rtol=1e-12, atol=0)
