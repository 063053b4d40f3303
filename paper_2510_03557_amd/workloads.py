"""Seeded synthetic particle sets for the short-range step.

This module only draws inputs: positions, velocities, masses, internal
energies, smoothing lengths and the per-box cutoff.  It holds none of the
method's arithmetic (no kernel, no moments, no forces), so both the GPU path
and the CPU oracle may consume what it produces.

Conventions shared by every generator:

* every box is a periodic unit box; positions are stored as float32 in
  [1, 2), where any two values share one exponent so that their difference is
  exact in float32;
* all values are drawn in float64 and rounded once to float32; the float32
  arrays are the inputs of both implementations;
* each box has total mass 1 (equal masses 1/N_box unless stated otherwise);
* "gas" particles carry velocity, internal energy u and smoothing length h;
  "dm" particles carry velocity and mass only.

The named sets follow the workloads of the short-range benchmark: a jittered
lattice (65,536 particles), a Zel'dovich-displaced random field (4.2 M and
180 M particles), 512 independent boxes of uneven occupancy, and Plummer
spheres over a uniform background (67 M particles).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

F32 = np.float32


@dataclass
class Species:
    """Structure-of-arrays particle set in caller order (all float32)."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray
    h: np.ndarray | None = None  # gas only
    u: np.ndarray | None = None  # gas only

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def fields(self):
        names = ["x", "y", "z", "vx", "vy", "vz", "m", "h", "u"]
        return {k: getattr(self, k) for k in names if getattr(self, k) is not None}


@dataclass
class Workload:
    """A batch of independent periodic boxes.

    ``gas_off``/``dm_off`` are the per-box offsets (length n_boxes + 1) into
    the concatenated species arrays.  ``r_c`` and ``eps`` are per box.
    """

    name: str
    gas: Species
    dm: Species
    gas_off: np.ndarray
    dm_off: np.ndarray
    r_c: np.ndarray
    eps: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_boxes(self) -> int:
        return int(self.gas_off.shape[0] - 1)

    @property
    def n_total(self) -> int:
        return self.gas.n + self.dm.n


# ----------------------------------------------------------------------------
# helpers (no physics here: only rounding, wrapping and drawing)
# ----------------------------------------------------------------------------

def to_box32(p: np.ndarray) -> np.ndarray:
    """Map arbitrary float64 coordinates to float32 values in [1, 2)."""
    f = np.mod(np.asarray(p, dtype=np.float64), 1.0)
    out = (1.0 + f).astype(F32)
    out[out >= F32(2.0)] = F32(1.0)  # rounding up to 2 wraps to 1
    out[out < F32(1.0)] = F32(1.0)
    return out


def _species(pos, vel, m, h=None, u=None) -> Species:
    return Species(
        x=to_box32(pos[0]), y=to_box32(pos[1]), z=to_box32(pos[2]),
        vx=np.asarray(vel[0], F32), vy=np.asarray(vel[1], F32),
        vz=np.asarray(vel[2], F32), m=np.asarray(m, F32),
        h=None if h is None else np.asarray(h, F32),
        u=None if u is None else np.asarray(u, F32),
    )


def h_for_neighbours(n_density: np.ndarray, n_ngb: float) -> np.ndarray:
    """Smoothing length whose 2h-sphere holds n_ngb particles at density n."""
    return 0.5 * (3.0 * n_ngb / (4.0 * np.pi * n_density)) ** (1.0 / 3.0)


def cic_number_density(x01, y01, z01, nm: int) -> np.ndarray:
    """Cloud-in-cell number density on an nm^3 periodic mesh, read back at the
    particles (positions in [0, 1)).  Used only to pick input smoothing
    lengths; it is not part of the method."""
    n = x01.shape[0]
    base = []
    wts = []
    for c in (x01, y01, z01):
        g = c * nm - 0.5
        i0 = np.floor(g).astype(np.int64)
        f = g - i0
        base.append((np.mod(i0, nm), np.mod(i0 + 1, nm)))
        wts.append((1.0 - f, f))
    corners = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    grid = np.zeros(nm * nm * nm, dtype=np.float64)
    for a, b, c in corners:
        flat = (base[0][a] * nm + base[1][b]) * nm + base[2][c]
        grid += np.bincount(flat, weights=wts[0][a] * wts[1][b] * wts[2][c],
                            minlength=nm ** 3)
    dens = np.zeros(n, dtype=np.float64)
    for a, b, c in corners:
        flat = (base[0][a] * nm + base[1][b]) * nm + base[2][c]
        dens += wts[0][a] * wts[1][b] * wts[2][c] * grid[flat]
    return dens * float(nm) ** 3


def zeldovich_displacement(ng: int, spectral_index: float, rms_cells: float,
                           rng: np.random.Generator):
    """Displacement field psi on an ng^3 grid from a Gaussian random field
    with power spectrum P(k) ~ k^n (P(0) = 0); psi(k) = i k delta(k) / k^2,
    scaled so that the 3-D rms of |psi| equals rms_cells grid spacings.
    Returns three float64 arrays of shape (ng, ng, ng) in box units."""
    w = rng.standard_normal((ng, ng, ng))
    wk = np.fft.rfftn(w)
    del w
    kx = np.fft.fftfreq(ng) * ng
    kz = np.fft.rfftfreq(ng) * ng
    k2 = (kx[:, None, None] ** 2 + kx[None, :, None] ** 2
          + kz[None, None, :] ** 2)
    k2[0, 0, 0] = 1.0
    wk *= k2 ** (spectral_index / 4.0)
    wk /= k2
    wk[0, 0, 0] = 0.0
    del k2
    psi = []
    for kk in (kx[:, None, None], kx[None, :, None], kz[None, None, :]):
        psi.append(np.fft.irfftn(1j * kk * wk, s=(ng, ng, ng), axes=(0, 1, 2)))
    del wk
    rms = np.sqrt(np.mean(psi[0] ** 2 + psi[1] ** 2 + psi[2] ** 2))
    scale = rms_cells / ng / rms
    return [p * scale for p in psi]


def _lattice(ng: int, offset: float):
    i = (np.arange(ng, dtype=np.float64) + offset) / ng
    X, Y, Z = np.meshgrid(i, i, i, indexing="ij")
    return X.ravel(), Y.ravel(), Z.ravel()


def _single_box(name, gas, dm, r_c, eps, meta):
    return Workload(name=name, gas=gas, dm=dm,
                    gas_off=np.array([0, gas.n], np.int64),
                    dm_off=np.array([0, dm.n], np.int64),
                    r_c=np.array([r_c], np.float64),
                    eps=np.array([eps], np.float64), meta=meta)


def concat_boxes(name: str, boxes: list[Workload], meta=None) -> Workload:
    """Concatenate independent single- or multi-box workloads."""
    def cat(attr, sp):
        vals = [getattr(getattr(b, sp), attr) for b in boxes]
        if vals[0] is None:
            return None
        return np.concatenate(vals)

    gas = Species(**{k: cat(k, "gas") for k in
                     ["x", "y", "z", "vx", "vy", "vz", "m", "h", "u"]})
    dm = Species(**{k: cat(k, "dm") for k in
                    ["x", "y", "z", "vx", "vy", "vz", "m"]})
    goff = [0]
    doff = [0]
    for b in boxes:
        for i in range(b.n_boxes):
            goff.append(goff[-1] + int(b.gas_off[i + 1] - b.gas_off[i]))
            doff.append(doff[-1] + int(b.dm_off[i + 1] - b.dm_off[i]))
    return Workload(name=name, gas=gas, dm=dm,
                    gas_off=np.array(goff, np.int64),
                    dm_off=np.array(doff, np.int64),
                    r_c=np.concatenate([b.r_c for b in boxes]),
                    eps=np.concatenate([b.eps for b in boxes]),
                    meta=meta or {})


def _lognormal_u(rng, n):
    return 1.0 * np.exp(0.1 * rng.standard_normal(n))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def jittered_lattice(ng: int = 32, seed: int = 1, sigma_cells: float = 0.2,
                     n_ngb: float = 32.0, rc_cells: float = 3.0) -> Workload:
    """ng^3 dm + ng^3 gas on a periodic lattice with Gaussian jitter.

    DM sites sit at cell corners, gas sites half a cell off; each coordinate
    gets an independent N(0, (sigma*cell)^2) offset.  Velocities N(0, 0.1^2)
    per axis, equal masses, u = exp(0.1 z), one global h for n_ngb
    neighbours, r_c = rc_cells / ng and eps = r_c / 60."""
    rng = np.random.default_rng(seed)
    n = ng ** 3
    d = 1.0 / ng
    out = []
    for off in (0.0, 0.5):
        X, Y, Z = _lattice(ng, off)
        pos = [X + sigma_cells * d * rng.standard_normal(n),
               Y + sigma_cells * d * rng.standard_normal(n),
               Z + sigma_cells * d * rng.standard_normal(n)]
        vel = [0.1 * rng.standard_normal(n) for _ in range(3)]
        out.append((pos, vel))
    m = np.full(n, 1.0 / (2 * n))
    h = np.full(n, h_for_neighbours(np.float64(n), n_ngb))
    u = _lognormal_u(rng, n)
    dm = _species(out[0][0], out[0][1], m)
    gas = _species(out[1][0], out[1][1], m, h=h, u=u)
    r_c = rc_cells / ng
    return _single_box(f"lattice{ng}", gas, dm, r_c, r_c / 60.0,
                       {"kind": "jittered_lattice", "ng": ng, "seed": seed})


def zeldovich(ng: int = 128, seed: int = 2, spectral_index: float = -2.0,
              rms_cells: float = 0.5, n_ngb: float = 64.0,
              rc_cells: float = 3.0, mesh: int | None = None,
              name: str | None = None) -> Workload:
    """ng^3 dm + ng^3 gas displaced by a Zel'dovich field.

    psi comes from a Gaussian random field with P(k) ~ k^spectral_index,
    scaled to a 3-D rms of rms_cells grid spacings; both species take psi at
    their lattice index (dm at corners, gas half a cell off); v = kappa psi
    with per-axis rms 0.1; h from the cloud-in-cell gas density on an
    (ng/4)^3 mesh for n_ngb neighbours; r_c = rc_cells / ng."""
    rng = np.random.default_rng(seed)
    n = ng ** 3
    psi = zeldovich_displacement(ng, spectral_index, rms_cells, rng)
    psi = [p.ravel() for p in psi]
    rms_axis = np.sqrt(np.mean(psi[0] ** 2 + psi[1] ** 2 + psi[2] ** 2) / 3.0)
    kappa = 0.1 / rms_axis
    m = np.full(n, 1.0 / (2 * n))
    sp = []
    for off in (0.0, 0.5):
        X, Y, Z = _lattice(ng, off)
        pos = [X + psi[0], Y + psi[1], Z + psi[2]]
        del X, Y, Z
        vel = [kappa * p for p in psi]
        sp.append((pos, vel))
    del psi
    gpos = [np.mod(p, 1.0) for p in sp[1][0]]
    nm = mesh if mesh is not None else max(ng // 4, 1)
    dens = cic_number_density(gpos[0], gpos[1], gpos[2], nm)
    dens = np.maximum(dens, 0.05 * n)
    h = h_for_neighbours(dens, n_ngb)
    h = np.minimum(h, 0.2)
    del gpos, dens
    u = _lognormal_u(rng, n)
    dm = _species(sp[0][0], sp[0][1], m)
    gas = _species(sp[1][0], sp[1][1], m, h=h, u=u)
    r_c = rc_cells / ng
    return _single_box(name or f"zeldovich{ng}", gas, dm, r_c, r_c / 60.0,
                       {"kind": "zeldovich", "ng": ng, "seed": seed,
                        "spectral_index": spectral_index,
                        "rms_cells": rms_cells})


def half_box_shift(c: np.ndarray) -> np.ndarray:
    """Float32 box coordinates in [1, 2) moved by half a box, periodically:
    x - 0.5 for x >= 1.5, x + 0.5 below.  Both branches stay inside [1, 2)
    with the same spacing of float32 values, so the move is exact and every
    minimum-image separation is unchanged."""
    c = np.asarray(c, F32)
    return np.where(c >= F32(1.5), c - F32(0.5), c + F32(0.5)).astype(F32)


def sub_cube(wl: Workload, side: float, halo: float, centre=1.5):
    """The particles of one box inside the cube of the given side about
    ``centre`` (a box coordinate in [1, 2), or one per axis), plus a halo of
    the given width around it, as a workload of its own (one box with the
    same r_c and eps; masses, h and u unchanged).  An axis along which the
    cube with its halo would cross the box's faces is first moved by half a
    box (half_box_shift, exact), so a cube may sit on the periodic faces.
    The cube with its halo must span less than half the box, so that the
    sub-box seen as a periodic unit box gains no pair across its faces.
    Returns (sub, gas_idx, dm_idx, inner_gas, inner_dm): the sub-box
    particles' indices in wl, and masks of those inside the cube proper.
    Selection only: no arithmetic of the method."""
    if wl.n_boxes != 1:
        raise ValueError("sub_cube takes a single-box workload")
    w = 0.5 * side + halo
    if not (2 * w < 0.5):
        raise ValueError("cube with halo must span less than half the box")
    cen = np.broadcast_to(np.asarray(centre, np.float64), (3,)).copy()
    shift = [not (1.0 < c - w and c + w < 2.0) for c in cen]
    for a in range(3):
        if shift[a]:
            cen[a] = cen[a] - 0.5 if cen[a] >= 1.5 else cen[a] + 0.5
    out = []
    for sp in (wl.gas, wl.dm):
        sel = np.ones(sp.n, bool)
        inner = np.ones(sp.n, bool)
        coords = []
        for a, c in enumerate((sp.x, sp.y, sp.z)):
            if shift[a]:
                c = half_box_shift(c)
            coords.append(c)
            c = c.astype(np.float64)
            sel &= (c >= cen[a] - w) & (c < cen[a] + w)
            inner &= (c >= cen[a] - 0.5 * side) & (c < cen[a] + 0.5 * side)
        idx = np.nonzero(sel)[0]
        f = {k: v[idx] for k, v in sp.fields().items()}
        f["x"], f["y"], f["z"] = (c[idx] for c in coords)
        out.append((Species(**f), idx, inner[idx]))
    (gas, gi, ig), (dm, di, idm) = out
    sub = _single_box(f"{wl.name}_cube", gas, dm, float(wl.r_c[0]),
                      float(wl.eps[0]),
                      {"kind": "sub_cube", "parent": wl.name, "side": side,
                       "halo": halo, "centre": cen.tolist(), "shift": shift})
    return sub, gi, di, ig, idm


def uneven_boxes(n_boxes: int = 512, seed: int = 3000, median: float = 20000.0,
                 sigma_ln: float = 0.768, nmin: int = 2000,
                 nmax: int = 200000) -> Workload:
    """Independent periodic boxes of lognormal occupancy.

    Box b draws N_b from a lognormal (median, sigma_ln), redrawn until inside
    [nmin, nmax]; it is then built like the 4.2 M Zel'dovich set at
    ng = round((N_b/2)^(1/3)) (so N_b = 2 ng^3), with its own seed
    seed + b and its own r_c = 3 / ng."""
    rng = np.random.default_rng(seed)
    boxes = []
    ngs = []
    for b in range(n_boxes):
        while True:
            nb = median * np.exp(sigma_ln * rng.standard_normal())
            ng = int(round((nb / 2.0) ** (1.0 / 3.0)))
            if nmin <= 2 * ng ** 3 <= nmax:
                break
        ngs.append(ng)
        boxes.append(zeldovich(ng=ng, seed=seed + b, spectral_index=-2.0,
                               rms_cells=0.5, n_ngb=64.0, rc_cells=3.0,
                               mesh=max(ng // 4, 2)))
    return concat_boxes("uneven_boxes", boxes,
                        {"kind": "uneven_boxes", "n_boxes": n_boxes,
                         "ng": ngs, "seed": seed})


def plummer_spheres(n_total: int = 2 ** 26, seed: int = 5,
                    n_spheres: int = 2000, background: float = 0.1,
                    slope: float = -1.9, mass_range: float = 100.0,
                    a_min: float = 0.001, a_max: float = 0.02,
                    max_contrast: float = 1.0e4, trunc: float = 10.0,
                    n_ngb: float = 64.0, ngb_lo: float = 32.0,
                    ngb_hi: float = 512.0) -> Workload:
    """Plummer spheres over a uniform background in one periodic box.

    A fraction ``background`` of the particles is uniform; the rest sits in
    ``n_spheres`` Plummer spheres whose particle counts follow
    dN/dM ~ M^slope on [M_min, mass_range M_min].  Scale radii are
    log-uniform in [a_min, a_max], raised where needed so that the central
    contrast 3 N_s / (4 pi a^3 N) stays <= max_contrast; radii are drawn
    from the Plummer cumulative mass truncated at trunc * a.  Sphere
    velocities are isotropic Gaussians with sigma^2 = M_s / (6 sqrt(r^2+a^2))
    (G = 1); the background has N(0, 0.1^2).  Half of the particles, chosen
    by a random permutation, are gas.  h follows the local gas density of
    the particle's own sphere plus the background for n_ngb neighbours,
    clamped so that the neighbour counts stay within [ngb_lo, ngb_hi].
    r_c = 3 / (N/2)^(1/3), eps = r_c / 60."""
    rng = np.random.default_rng(seed)
    n_bg = int(round(background * n_total))
    n_sph_tot = n_total - n_bg
    # sphere masses from the power law (inverse CDF)
    g = slope + 1.0
    uu = rng.random(n_spheres)
    M = ((mass_range ** g - 1.0) * uu + 1.0) ** (1.0 / g)
    cnt = np.floor(M / M.sum() * n_sph_tot).astype(np.int64)
    rem = n_sph_tot - int(cnt.sum())
    order = np.argsort(-(M / M.sum() * n_sph_tot - cnt))
    cnt[order[:rem]] += 1
    centres = rng.random((n_spheres, 3))
    a = np.exp(rng.uniform(np.log(a_min), np.log(a_max), n_spheres))
    a_floor = (3.0 * cnt / (4.0 * np.pi * max_contrast * n_total)) ** (1.0 / 3.0)
    a = np.maximum(a, a_floor)
    pos = np.empty((3, n_total), np.float64)
    vel = np.empty((3, n_total), np.float64)
    nloc = np.empty(n_total, np.float64)  # local total number density
    m_part = 1.0 / n_total
    n_bg_density = float(n_bg)  # per unit volume
    pos[:, :n_bg] = rng.random((3, n_bg))
    vel[:, :n_bg] = 0.1 * rng.standard_normal((3, n_bg))
    nloc[:n_bg] = n_bg_density
    k = n_bg
    ftr = trunc ** 3 / (trunc ** 2 + 1.0) ** 1.5
    for s in range(n_spheres):
        ns = int(cnt[s])
        if ns == 0:
            continue
        U = rng.random(ns) * ftr
        U = np.maximum(U, 1e-300)
        r = a[s] / np.sqrt(U ** (-2.0 / 3.0) - 1.0)
        mu = rng.uniform(-1.0, 1.0, ns)
        ph = rng.uniform(0.0, 2.0 * np.pi, ns)
        st = np.sqrt(1.0 - mu * mu)
        pos[0, k:k + ns] = centres[s, 0] + r * st * np.cos(ph)
        pos[1, k:k + ns] = centres[s, 1] + r * st * np.sin(ph)
        pos[2, k:k + ns] = centres[s, 2] + r * mu
        Ms = ns * m_part
        sig = np.sqrt(Ms / (6.0 * np.sqrt(r * r + a[s] ** 2)))
        vel[:, k:k + ns] = sig * rng.standard_normal((3, ns))
        rho0 = 3.0 * ns / (4.0 * np.pi * a[s] ** 3) / ftr
        nloc[k:k + ns] = n_bg_density + rho0 * (1.0 + (r / a[s]) ** 2) ** -2.5
        k += ns
    perm = rng.permutation(n_total)
    n_gas = n_total // 2
    gi = perm[:n_gas]
    di = perm[n_gas:]
    # gas number density is half the total density in expectation
    ngas_loc = 0.5 * nloc[gi]
    h = h_for_neighbours(ngas_loc, n_ngb)
    h_lo = h_for_neighbours(0.5 * nloc.max(), ngb_hi)
    h_hi = h_for_neighbours(0.5 * n_bg_density, ngb_lo * 2.0)
    h = np.clip(h, h_lo, min(h_hi, 0.2))
    m = np.full(n_gas, m_part)
    u = _lognormal_u(rng, n_gas)
    gas = _species(pos[:, gi], vel[:, gi], m, h=h, u=u)
    dm = _species(pos[:, di], vel[:, di], np.full(n_total - n_gas, m_part))
    r_c = 3.0 / (n_total / 2.0) ** (1.0 / 3.0)
    return _single_box("plummer", gas, dm, r_c, r_c / 60.0,
                       {"kind": "plummer", "n_total": n_total, "seed": seed,
                        "n_spheres": n_spheres})


def knn_smoothing_length(x01: np.ndarray, n_ngb: int) -> np.ndarray:
    """h such that the 2h-sphere of every particle holds exactly n_ngb other
    particles of the set (positions (3, n) in [0, 1), periodic): 2h is
    midway between the n_ngb-th and (n_ngb+1)-th neighbour distances."""
    from scipy.spatial import cKDTree
    pts = np.ascontiguousarray(np.mod(x01.T, 1.0))
    tree = cKDTree(pts, boxsize=1.0)
    d, _ = tree.query(pts, k=n_ngb + 2)
    return 0.25 * (d[:, n_ngb] + d[:, n_ngb + 1])


def random_uniform(n_gas: int, n_dm: int, seed: int, n_ngb: float = 32.0,
                   r_c: float | None = None, h_spread: float = 0.3,
                   clustered: bool = False, h_rule: str = "knn") -> Workload:
    """Small random sets for parity cases: uniform (or two-blob clustered)
    positions, unequal masses in [0.5, 1.5]/N, lognormal u, N(0, 0.1^2)
    velocities.  h_rule "knn" (default) gives every gas particle exactly
    n_ngb neighbours inside 2h, as an adaptive smoothing length does;
    "global" draws h lognormally (spread h_spread) around the value for
    n_ngb neighbours at the mean density."""
    rng = np.random.default_rng(seed)
    n = n_gas + n_dm

    def draw(k):
        if not clustered:
            return rng.random((3, k))
        c = rng.random((2, 3))
        which = rng.integers(0, 3, k)
        p = rng.random((3, k))
        for w in (0, 1):
            sel = which == w
            p[:, sel] = (c[w][:, None]
                         + 0.06 * rng.standard_normal((3, int(sel.sum()))))
        return p

    gp = draw(n_gas)
    dp = draw(n_dm)
    h0 = h_for_neighbours(float(max(n_gas, 1)), n_ngb)
    if h_rule == "knn" and n_gas > int(n_ngb) + 2:
        # neighbours of the float32 positions actually used
        g32 = np.stack([to_box32(c) for c in gp]).astype(np.float64) - 1.0
        h = knn_smoothing_length(g32, int(n_ngb))
        rng.standard_normal(n_gas)  # keep the random stream aligned
    else:
        h = h0 * np.exp(h_spread * rng.standard_normal(n_gas))
    h = np.minimum(h, 0.2)
    if r_c is None:
        r_c = min(3.0 / max(n, 1) ** (1.0 / 3.0) * 1.26, 0.4)
    gm = rng.uniform(0.5, 1.5, n_gas) / n
    dmm = rng.uniform(0.5, 1.5, n_dm) / n
    gas = _species(gp, 0.1 * rng.standard_normal((3, n_gas)), gm, h=h,
                   u=_lognormal_u(rng, n_gas))
    dm = _species(dp, 0.1 * rng.standard_normal((3, n_dm)), dmm)
    return _single_box(f"random{n_gas}_{n_dm}_{seed}", gas, dm, r_c,
                       r_c / 60.0, {"kind": "random", "seed": seed,
                                    "clustered": clustered, "h_rule": h_rule})


def perfect_lattice(ng: int, n_ngb: float = 32.0, rc_cells: float = 3.0,
                    u0: float = 1.0) -> Workload:
    """Unperturbed lattice (dm at corners, gas at cell centres), v = 0,
    uniform u: the configuration on which every net force vanishes."""
    n = ng ** 3
    z3 = np.zeros((3, n))
    m = np.full(n, 1.0 / (2 * n))
    h = np.full(n, h_for_neighbours(float(n), n_ngb))
    dm = _species(_lattice(ng, 0.0), z3, m)
    gas = _species(_lattice(ng, 0.5), z3, m, h=h, u=np.full(n, u0))
    r_c = rc_cells / ng
    return _single_box(f"perfect{ng}", gas, dm, r_c, r_c / 60.0,
                       {"kind": "perfect_lattice", "ng": ng})


# the five benchmark configurations, smallest first
CONFIGS = {
    "lattice32": lambda: jittered_lattice(32, seed=1),
    "zeldovich128": lambda: zeldovich(128, seed=2, spectral_index=-2.0,
                                      rms_cells=0.5, n_ngb=64.0),
    "uneven_boxes512": lambda: uneven_boxes(512, seed=3000),
    "zeldovich448": lambda: zeldovich(448, seed=4, spectral_index=-1.5,
                                      rms_cells=1.0, n_ngb=64.0),
    "plummer64M": lambda: plummer_spheres(2 ** 26, seed=5),
}


# smaller sets of the same kinds, for measurements that need many steps
# (hierarchical cycles on clustered matter)
EXTRA = {
    "plummer4M": lambda: plummer_spheres(2 ** 22, seed=6),
}


def make(name: str) -> Workload:
    if name in EXTRA:
        return EXTRA[name]()
    return CONFIGS[name]()
