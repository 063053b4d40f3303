"""Pins of the oracle's long-range particle-mesh gravity (the spectral PM
half of the force split, Sec. IV-A).

Checked against what the mathematics fixes: the S2 form factor against a
quadrature of the cloud's radial Fourier integral; no force on a perfect
mesh lattice; momentum conservation of the symmetric deposit/interpolation;
and the split itself, short-range + long-range = the periodic Newtonian
force, against an independent Ewald sum (within the 1 % mesh error for
r_c = 6 mesh cells).
"""
import numpy as np
import pytest
from scipy import integrate
from scipy.special import erfc


def ewald_accel(r, alpha=6.0, nr=2, nk=8):
    """Acceleration of a unit mass at separation vector r from another unit
    mass in the unit periodic box with a neutralising background, G = 1:
    real-space erfc sum over images plus the reciprocal-space sum."""
    r = np.asarray(r, float)
    F = np.zeros(3)
    rng = range(-nr, nr + 1)
    for i in rng:
        for j in rng:
            for k in rng:
                rn = r + np.array([i, j, k])
                d = np.linalg.norm(rn)
                F -= (erfc(alpha * d) + 2 * alpha * d / np.sqrt(np.pi)
                      * np.exp(-alpha ** 2 * d ** 2)) * rn / d ** 3
    n = np.arange(-nk, nk + 1)
    for i in n:
        for j in n:
            for k in n:
                if i == 0 and j == 0 and k == 0:
                    continue
                kv = 2 * np.pi * np.array([i, j, k])
                k2 = kv @ kv
                F -= 4 * np.pi / k2 * np.exp(-k2 / (4 * alpha ** 2)) * kv \
                    * np.sin(kv @ r)
    return F


def test_ewald_reference_is_newtonian_at_short_range():
    """The Ewald helper itself: at small separation it is Newton's force."""
    d = 0.01
    a = ewald_accel([d, 0, 0])
    assert abs(a[0] + 1 / d ** 2) / (1 / d ** 2) < 1e-3
    assert abs(a[1]) < 1e-8 and abs(a[2]) < 1e-8


@pytest.mark.parametrize("kr", [0.05, 0.7, 2.0, 5.0, 11.0])
def test_s2_form_factor_vs_quadrature(orc, kr):
    """S2 cloud of diameter a: density 48 / (pi a^4) (a/2 - r) inside a/2;
    its transform int rho(r) sin(kr)/(kr) 4 pi r^2 dr."""
    a = 0.1
    k = kr / (a / 2)

    def f(r):
        return 48 / (np.pi * a ** 4) * (a / 2 - r) * np.sinc(k * r / np.pi) \
            * 4 * np.pi * r ** 2
    ref = integrate.quad(f, 0, a / 2, epsabs=1e-13, limit=200)[0]
    got = orc.s2_form_factor(np.array([k]), a)[0]
    assert abs(got - ref) < 1e-9


def test_pm_lattice_has_no_force(orc):
    """Equal masses on every mesh node: uniform mesh density, no force."""
    N = 16
    i = np.arange(N) / N + 1.0
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    m = np.full(N ** 3, 1.0 / N ** 3)
    a = orc.pm_long_range(X.ravel(), Y.ravel(), Z.ravel(), m, N, 6.0 / N)
    assert np.max(np.abs(a)) < 1e-10


def test_pm_momentum_conservation(orc):
    """Symmetric deposit and interpolation with an odd force kernel:
    sum m a = 0."""
    rng = np.random.default_rng(3)
    n = 500
    P = 1.0 + rng.random((3, n))
    m = rng.uniform(0.5, 1.5, n) / n
    a = orc.pm_long_range(*P, m, 32, 6.0 / 32)
    tot = (m * a).sum(1)
    scale = (m * np.abs(a)).sum()
    assert np.max(np.abs(tot)) < 1e-12 * scale


@pytest.mark.parametrize("d,direction", [
    (0.5, (1, 0, 0)), (1.0, (0, 1, 0)), (1.5, (1, 1, 0)), (3.0, (1, 2, 2)),
    (6.0, (0, 0, 1)), (9.0, (2, 1, 2))])
def test_short_plus_long_is_periodic_newton(orc, d, direction):
    """Two unit masses at separation d r_c: the short-range force (the
    oracle's g(r)) plus the mesh long-range force equals the periodic
    Newtonian force (Ewald) with the pair's Plummer softening, within 1 %
    for r_c = 6 mesh cells (the mesh error, largest near r_c)."""
    N = 64
    rc = 6.0 / N
    eps = rc / 60
    u = np.asarray(direction, float)
    u /= np.linalg.norm(u)
    r = d * rc
    p0 = np.array([1.31, 1.52, 1.23])
    p1 = p0 + r * u
    P = np.stack([p0, p1], axis=1)
    a = orc.pm_long_range(P[0], P[1], P[2], np.ones(2), N, rc)[:, 1]
    a_short = -orc.grav_g(r, rc, eps) * u  # g: force per unit masses
    # Ewald is unsoftened: add the softening of the direct pair
    soft = -(r / (r * r + eps * eps) ** 1.5 - 1 / r ** 2) * u
    ref = ewald_accel(r * u) + soft
    err = np.linalg.norm(a + a_short - ref) / np.linalg.norm(ref)
    assert err < 1e-2, err
