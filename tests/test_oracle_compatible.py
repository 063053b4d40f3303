"""Pins of the oracle's compatible energy update (CRKSPH's time-centred,
energy-conserving specific-energy update; Sec. IV-A names the method and
its conservation, the form is a reading): du_i/dt = -sum_j F_ij .
(v^c_i - v^c_j) / (2 m_i) with the forces F_ij of the state at the start of
the kick and v^c = (v + v1)/2, v1 the velocities after the kick.

Checked against what the mathematics fixes: with the hydro forces alone a
kick v1 = v + dt a, u1 = u + dt du/dt then conserves sum m (v^2/2 + u)
exactly (to rounding), since sum_i m_i a_i . v^c_i = sum over pairs of
F_ij . (v^c_i - v^c_j); the plain rate (work at v) does not; v1 = v gives
the plain rate bit for bit; a common boost of v and v1 changes nothing.
"""
import numpy as np
import pytest

from paper_2510_03557_amd import workloads as wl_mod

PASSES = ("density", "coefficients", "hydro")


def energy(m, v, u):
    return 0.5 * (m * (v * v).sum(0)).sum() + (m * u).sum()


@pytest.fixture(scope="module")
def gas_step(orc):
    w = wl_mod.random_uniform(2000, 0, 61, n_ngb=48.0, h_spread=0.15,
                              clustered=True)
    return w, orc.step(w, passes=PASSES, brute=True), \
        orc.step(w, passes=PASSES, brute=True, recon=True)


@pytest.mark.parametrize("recon", [False, True])
def test_compatible_kick_conserves_energy(orc, gas_step, recon):
    w, plain, rec = gas_step
    out = rec if recon else plain
    g = w.gas
    m = g.m.astype(np.float64)
    v = np.array([g.vx, g.vy, g.vz], np.float64)
    u = g.u.astype(np.float64)
    # a kick that changes the kinetic energy by a good fraction
    amax = np.abs(out["a_hydro"]).max()
    dt = 0.2 * np.abs(v).max() / amax
    r = orc.compatible_update(w, out, dt, recon=recon, brute=True)
    E0 = energy(m, v, u)
    E1 = energy(m, r["v1"], r["u1"])
    dke = 0.5 * (m * np.abs((r["v1"] ** 2 - v ** 2).sum(0))).sum()
    assert dke > 1e-4 * E0
    assert abs(E1 - E0) < 1e-13 * E0, (E1 - E0) / E0
    # the plain rate (pair work at the start velocities) misses by O(dt^2)
    u_plain = u + dt * out["dudt"]
    assert abs(energy(m, r["v1"], u_plain) - E0) > 1e-6 * E0


def test_no_kick_gives_plain_rate(orc, gas_step):
    w, plain, rec = gas_step
    g = w.gas
    for out, recon in ((plain, False), (rec, True)):
        r = orc.compatible_update(w, out, 0.0, recon=recon, brute=True)
        assert np.array_equal(r["dudt"], out["dudt"])


def test_compatible_rate_galilean(orc, gas_step):
    w, plain, _ = gas_step
    g = w.gas
    args = [g.x, g.y, g.z, g.vx, g.vy, g.vz, g.h, g.m, plain["V"],
            plain["rho"], plain["P"], plain["cs"], plain["A"], plain["B"],
            plain["gradA"], plain["gradB"]]
    v = np.array([g.vx, g.vy, g.vz], np.float64)
    v1 = v + 0.01 * plain["a_hydro"]
    du = orc.hydro(*args, brute=True, v1=v1)[3]
    c = np.array([0.5, -0.25, 0.75])[:, None]
    vb = v + c
    argsb = list(args)
    argsb[3:6] = vb
    dub = orc.hydro(*argsb, brute=True, v1=v1 + c)[3]
    assert np.abs(dub - du).max() < 1e-10 * np.abs(du).max()
