"""ctypes front end of the FP64 C oracle (test infrastructure only).

Every function takes numpy arrays (any float dtype; widened to float64,
which is exact for the float32 inputs of the GPU path) and returns float64
results.  ``targets`` selects the particles whose outputs are computed; the
sums still run over every particle of the box.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "crk_oracle.c"
_LIB = _HERE / "libcrk_oracle.so"

# Constants of the step (readings of the method; the paper prints none):
# ideal gas gamma = 5/3, Monaghan viscosity C_l = 1, C_q = 2 with eps_Q = 0.01,
# gravitational constant G = 1.
PARAMS = dict(gamma=5.0 / 3.0, Cl=1.0, Cq=2.0, epsQ=0.01, G=1.0)

# Limiter of the reconstructed viscosity (a reading; CRKSPH is named in
# Sec. IV-A without its constants): close pairs, r / max(h_i, h_j) below
# eta_crit (about the mean spacing at ~64 neighbours inside 2h), are damped
# with a Gaussian of width eta_fold.
RECON = dict(eta_crit=0.8, eta_fold=0.2)

_lib = None


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (plain C, -O2, OpenMP)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                        "-std=c11", "-o", str(tmp), str(_SRC), "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        _lib = ctypes.CDLL(str(_LIB))
        _lib.orc_s2_force.restype = ctypes.c_double
        _lib.orc_s2_force.argtypes = [ctypes.c_double, ctypes.c_double]
        _lib.orc_grav_g.restype = ctypes.c_double
        _lib.orc_grav_g.argtypes = [ctypes.c_double] * 3
        _lib.orc_num_threads.restype = ctypes.c_int
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _targets(targets, n):
    if targets is None:
        return n, None
    t = np.ascontiguousarray(targets, dtype=np.int64)
    return t.shape[0], t


def _i64(v):
    return ctypes.c_int64(int(v))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def kernel(r, h):
    """Cubic spline W(r, h) and dW/dr (scalar)."""
    W = ctypes.c_double()
    dW = ctypes.c_double()
    _load().orc_kernel(ctypes.c_double(r), ctypes.c_double(h),
                       ctypes.byref(W), ctypes.byref(dW))
    return W.value, dW.value


def s2_force(r, a):
    return _load().orc_s2_force(float(r), float(a))


def grav_g(r, r_c, eps):
    return _load().orc_grav_g(float(r), float(r_c), float(eps))


def neighbours(x, y, z, h, mode, targets=None, brute=False):
    """Lists of gas neighbours of each target (mode 0: r < 2 h_i; mode 1:
    r < 2 max(h_i, h_j)); returns (offsets, indices)."""
    lib = _load()
    x, y, z, h = _d(x), _d(y), _d(z), _d(h)
    n = x.shape[0]
    nt, t = _targets(targets, n)
    counts = np.zeros(nt, np.int64)
    if lib.orc_neighbours(_i64(n), _p(x), _p(y), _p(z), _p(h),
                          ctypes.c_int(mode), _i64(nt), _p(t),
                          ctypes.c_int(int(brute)), _p(counts), None, None):
        raise MemoryError("oracle neighbour search failed")
    off = np.zeros(nt + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    idx = np.zeros(int(off[-1]), np.int64)
    if lib.orc_neighbours(_i64(n), _p(x), _p(y), _p(z), _p(h),
                          ctypes.c_int(mode), _i64(nt), _p(t),
                          ctypes.c_int(int(brute)), _p(counts), _p(off),
                          _p(idx)):
        raise MemoryError("oracle neighbour search failed")
    return off, idx


def density(x, y, z, h, m, targets=None, brute=False):
    lib = _load()
    x, y, z, h, m = _d(x), _d(y), _d(z), _d(h), _d(m)
    nt, t = _targets(targets, x.shape[0])
    V = np.zeros(nt)
    rt = np.zeros(nt)
    if lib.orc_density(_i64(x.shape[0]), _p(x), _p(y), _p(z), _p(h), _p(m),
                       _i64(nt), _p(t), ctypes.c_int(int(brute)), _p(V),
                       _p(rt)):
        raise MemoryError("oracle density failed")
    return V, rt


def coefficients(x, y, z, h, m, V, u, gamma=PARAMS["gamma"], targets=None,
                 brute=False):
    """A, B (n,3), gradA (n,3), gradB (n,3,3) with gradB[:, g, a] = d_g B^a,
    rho, P, cs and the degenerate-moment flags."""
    lib = _load()
    x, y, z, h, m, V, u = (_d(a) for a in (x, y, z, h, m, V, u))
    nt, t = _targets(targets, x.shape[0])
    out = dict(A=np.zeros(nt), B=np.zeros((nt, 3)), gradA=np.zeros((nt, 3)),
               gradB=np.zeros((nt, 3, 3)), rho=np.zeros(nt), P=np.zeros(nt),
               cs=np.zeros(nt))
    deg = np.zeros(nt, np.int32)
    if lib.orc_coefficients(_i64(x.shape[0]), _p(x), _p(y), _p(z), _p(h),
                            _p(m), _p(V), _p(u), ctypes.c_double(gamma),
                            _i64(nt), _p(t), ctypes.c_int(int(brute)),
                            _p(out["A"]), _p(out["B"]), _p(out["gradA"]),
                            _p(out["gradB"]), _p(out["rho"]), _p(out["P"]),
                            _p(out["cs"]), _p(deg)):
        raise MemoryError("oracle coefficients failed")
    out["degenerate"] = deg
    return out


def velocity_gradient(x, y, z, vx, vy, vz, h, V, A, B, gradA, gradB,
                      targets=None, brute=False):
    """Corrected-kernel velocity gradient at the targets, (nt, 3, 3) with
    dv[:, a, b] = d v^a / d x^b."""
    lib = _load()
    arrs = [_d(a) for a in (x, y, z, vx, vy, vz, h, V, A)]
    B = _d(np.reshape(B, (-1, 3)))
    gradA = _d(np.reshape(gradA, (-1, 3)))
    gradB = _d(np.reshape(gradB, (-1, 3, 3)))
    n = arrs[0].shape[0]
    nt, t = _targets(targets, n)
    dv = np.zeros((nt, 3, 3))
    if lib.orc_velocity_gradient(_i64(n), *[_p(a) for a in arrs], _p(B),
                                 _p(gradA), _p(gradB), _i64(nt), _p(t),
                                 ctypes.c_int(int(brute)), _p(dv)):
        raise MemoryError("oracle velocity gradient failed")
    return dv


def hydro(x, y, z, vx, vy, vz, h, m, V, rho, P, cs, A, B, gradA, gradB,
          Cl=PARAMS["Cl"], Cq=PARAMS["Cq"], epsQ=PARAMS["epsQ"],
          targets=None, brute=False, dv=None, eta_crit=RECON["eta_crit"],
          eta_fold=RECON["eta_fold"], v1=None):
    """a_hydro (3 arrays) and du/dt at the targets.  With ``dv`` (the
    velocity gradient of every particle, (n, 3, 3)) the viscosity acts on the
    limited linear reconstruction of the two velocities at the pair
    midpoint.  With ``v1`` (the velocities after a kick, (3, n)) du/dt takes
    the pair work at the time-centred velocities (v + v1)/2 (the forces
    stay those of the state at v)."""
    lib = _load()
    arrs = [_d(a) for a in (x, y, z, vx, vy, vz, h, m, V, rho, P, cs, A)]
    B = _d(np.reshape(B, (-1, 3)))
    gradA = _d(np.reshape(gradA, (-1, 3)))
    gradB = _d(np.reshape(gradB, (-1, 3, 3)))
    n = arrs[0].shape[0]
    if dv is not None:
        dv = _d(np.reshape(dv, (n, 3, 3)))
    w1 = [None, None, None]
    if v1 is not None:
        w1 = [_d(a) for a in v1]
    nt, t = _targets(targets, n)
    ax, ay, az, du = (np.zeros(nt) for _ in range(4))
    if lib.orc_hydro(_i64(n), *[_p(a) for a in arrs], _p(B), _p(gradA),
                     _p(gradB), ctypes.c_double(Cl), ctypes.c_double(Cq),
                     ctypes.c_double(epsQ),
                     _p(dv) if dv is not None else None,
                     ctypes.c_double(eta_crit), ctypes.c_double(eta_fold),
                     *[_p(a) for a in w1],
                     _i64(nt), _p(t), ctypes.c_int(int(brute)), _p(ax),
                     _p(ay), _p(az), _p(du)):
        raise MemoryError("oracle hydro failed")
    return ax, ay, az, du


def gravity(x, y, z, m, r_c, eps, G=PARAMS["G"], targets=None, brute=False):
    lib = _load()
    x, y, z, m = _d(x), _d(y), _d(z), _d(m)
    nt, t = _targets(targets, x.shape[0])
    ax, ay, az = (np.zeros(nt) for _ in range(3))
    if lib.orc_gravity(_i64(x.shape[0]), _p(x), _p(y), _p(z), _p(m),
                       ctypes.c_double(r_c), ctypes.c_double(eps),
                       ctypes.c_double(G), _i64(nt), _p(t),
                       ctypes.c_int(int(brute)), _p(ax), _p(ay), _p(az)):
        raise MemoryError("oracle gravity failed")
    return ax, ay, az


def compatible_update(wl, out, dt, params=PARAMS, recon=False,
                      brute=False):
    """The compatible energy update of one kick of the gas of a step whose
    passes gave ``out`` (from step()): v1 = v + dt (a_grav + a_hydro), the
    specific-energy rate from the same pair forces with the pair work at
    the time-centred velocities (v + v1)/2, and u1 = u + dt du/dt.
    Returns dict(v1 (3, n), dudt, u1)."""
    g = wl.gas
    v = np.array([g.vx, g.vy, g.vz], np.float64)
    v1 = v + dt * (out["a_grav_gas"] + out["a_hydro"])
    dudt = np.zeros(g.n)
    for b, gs, ds in _box_slices(wl):
        if gs.stop == gs.start:
            continue
        _, _, _, du = hydro(
            g.x[gs], g.y[gs], g.z[gs], g.vx[gs], g.vy[gs], g.vz[gs],
            g.h[gs], g.m[gs], out["V"][gs], out["rho"][gs], out["P"][gs],
            out["cs"][gs], out["A"][gs], out["B"][gs], out["gradA"][gs],
            out["gradB"][gs], params["Cl"], params["Cq"], params["epsQ"],
            brute=brute, dv=out["dv"][gs] if recon else None,
            v1=v1[:, gs])
        dudt[gs] = du
    return dict(v1=v1, dudt=dudt,
                u1=np.asarray(g.u, np.float64) + dt * dudt)


def integrate(dt, x, v, u, a_grav, a_hydro=None, dudt=None):
    """One FP64 kick-drift: v += dt a, x += dt v (wrapped into [1, 2)),
    u += dt du/dt.  x, v, a_* are (3, n) arrays."""
    x = np.array(x, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    a = np.array(a_grav, dtype=np.float64)
    if a_hydro is not None:
        a = a + np.asarray(a_hydro, dtype=np.float64)
    v = v + dt * a
    x = x + dt * v
    x = np.where(x >= 2.0, x - 1.0, x)
    x = np.where(x < 1.0, x + 1.0, x)
    out = dict(x=x, v=v)
    if u is not None:
        out["u"] = np.asarray(u, np.float64) + dt * np.asarray(dudt, np.float64)
    return out


# ----------------------------------------------------------------------------
# whole step and sampled step over a workload (duck-typed: any object with
# gas/dm species, per-box offsets, r_c and eps)
# ----------------------------------------------------------------------------

def _box_slices(wl):
    for b in range(wl.n_boxes):
        yield (b, slice(int(wl.gas_off[b]), int(wl.gas_off[b + 1])),
               slice(int(wl.dm_off[b]), int(wl.dm_off[b + 1])))


def step(wl, params=PARAMS, brute=False, passes=("density", "coefficients",
                                                   "hydro", "gravity"),
         recon=False):
    """Every output of the short-range step for every particle, box by box,
    each pass fed with the previous passes' FP64 results.  With ``recon``
    the velocity gradient is computed after the coefficients and the
    viscosity acts on the limited midpoint reconstruction."""
    g, d = wl.gas, wl.dm
    ng, nd = g.n, d.n
    out = {k: np.zeros(ng) for k in ("V", "rho_tilde", "A", "rho", "P", "cs",
                                     "dudt")}
    out.update(B=np.zeros((ng, 3)), gradA=np.zeros((ng, 3)),
               gradB=np.zeros((ng, 3, 3)), a_hydro=np.zeros((3, ng)),
               a_grav_gas=np.zeros((3, ng)), a_grav_dm=np.zeros((3, nd)),
               degenerate=np.zeros(ng, np.int32), dv=np.zeros((ng, 3, 3)))
    for b, gs, ds in _box_slices(wl):
        if "density" in passes and gs.stop > gs.start:
            V, rt = density(g.x[gs], g.y[gs], g.z[gs], g.h[gs], g.m[gs],
                            brute=brute)
            out["V"][gs], out["rho_tilde"][gs] = V, rt
        if "coefficients" in passes and gs.stop > gs.start:
            c = coefficients(g.x[gs], g.y[gs], g.z[gs], g.h[gs], g.m[gs],
                             out["V"][gs], g.u[gs], params["gamma"],
                             brute=brute)
            for k in ("A", "B", "gradA", "gradB", "rho", "P", "cs",
                      "degenerate"):
                out[k][gs] = c[k]
        if recon and gs.stop > gs.start:
            out["dv"][gs] = velocity_gradient(
                g.x[gs], g.y[gs], g.z[gs], g.vx[gs], g.vy[gs], g.vz[gs],
                g.h[gs], out["V"][gs], out["A"][gs], out["B"][gs],
                out["gradA"][gs], out["gradB"][gs], brute=brute)
        if "hydro" in passes and gs.stop > gs.start:
            ax, ay, az, du = hydro(
                g.x[gs], g.y[gs], g.z[gs], g.vx[gs], g.vy[gs], g.vz[gs],
                g.h[gs], g.m[gs], out["V"][gs], out["rho"][gs], out["P"][gs],
                out["cs"][gs], out["A"][gs], out["B"][gs], out["gradA"][gs],
                out["gradB"][gs], params["Cl"], params["Cq"], params["epsQ"],
                brute=brute, dv=out["dv"][gs] if recon else None)
            out["a_hydro"][:, gs] = (ax, ay, az)
            out["dudt"][gs] = du
        if "gravity" in passes:
            X = np.concatenate([g.x[gs], d.x[ds]])
            Y = np.concatenate([g.y[gs], d.y[ds]])
            Z = np.concatenate([g.z[gs], d.z[ds]])
            M = np.concatenate([g.m[gs], d.m[ds]])
            if X.shape[0]:
                ax, ay, az = gravity(X, Y, Z, M, float(wl.r_c[b]),
                                     float(wl.eps[b]), params["G"],
                                     brute=brute)
                k = gs.stop - gs.start
                out["a_grav_gas"][:, gs] = (ax[:k], ay[:k], az[:k])
                out["a_grav_dm"][:, ds] = (ax[k:], ay[k:], az[k:])
    return out


def step_sampled(wl, gas_targets, dm_targets, params=PARAMS, recon=False,
                 progress=None):
    """The step's outputs at sampled particles only (global indices into the
    gas and dm arrays).  Each sampled gas particle pulls in the
    neighbourhoods its outputs depend on: coefficients (and, with
    ``recon``, velocity gradients) at its force neighbours, and volumes at
    their gather neighbours.  ``progress(msg)``, if given, is called after
    each stage (large sets take minutes)."""
    say = progress or (lambda msg: None)
    g, d = wl.gas, wl.dm
    gas_targets = np.asarray(gas_targets, np.int64)
    dm_targets = np.asarray(dm_targets, np.int64)
    res = dict(gas_idx=gas_targets, dm_idx=dm_targets)
    nt = gas_targets.shape[0]
    res.update(V=np.zeros(nt), rho_tilde=np.zeros(nt), A=np.zeros(nt),
               rho=np.zeros(nt), P=np.zeros(nt), cs=np.zeros(nt),
               dudt=np.zeros(nt), B=np.zeros((nt, 3)), gradA=np.zeros((nt, 3)),
               gradB=np.zeros((nt, 3, 3)), a_hydro=np.zeros((3, nt)),
               a_grav_gas=np.zeros((3, nt)),
               a_grav_dm=np.zeros((3, dm_targets.shape[0])),
               dv=np.zeros((nt, 3, 3)))
    for b, gs, ds in _box_slices(wl):
        sel = np.nonzero((gas_targets >= gs.start) & (gas_targets < gs.stop))[0]
        dsel = np.nonzero((dm_targets >= ds.start) & (dm_targets < ds.stop))[0]
        if sel.size == 0 and dsel.size == 0:
            continue
        gx, gy, gz = g.x[gs], g.y[gs], g.z[gs]
        gh, gm = g.h[gs], g.m[gs]
        n = gs.stop - gs.start
        if sel.size:
            T = gas_targets[sel] - gs.start
            off, idx = neighbours(gx, gy, gz, gh, 1, targets=T)
            S1 = np.unique(np.concatenate([T, idx]))
            say(f"oracle box {b}: {T.size} targets, {S1.size} force "
                "neighbours")
            off2, idx2 = neighbours(gx, gy, gz, gh, 0, targets=S1)
            S2 = np.unique(np.concatenate([S1, idx2]))
            say(f"oracle box {b}: {S2.size} particles of the volume closure")
            V = np.full(n, np.nan)
            rt = np.full(n, np.nan)
            V[S2], rt[S2] = density(gx, gy, gz, gh, gm, targets=S2)
            say(f"oracle box {b}: volumes done")
            c = coefficients(gx, gy, gz, gh, gm, V, g.u[gs], params["gamma"],
                             targets=S1)
            say(f"oracle box {b}: coefficients done")
            full = {}
            for k in ("A", "rho", "P", "cs"):
                full[k] = np.full(n, np.nan)
                full[k][S1] = c[k]
            for k, shp in (("B", (3,)), ("gradA", (3,)), ("gradB", (3, 3))):
                full[k] = np.full((n,) + shp, np.nan)
                full[k][S1] = c[k]
            dvf = None
            if recon:
                # gradients at the force neighbours: their own coefficients
                # and the volumes of their gather neighbours (inside S2)
                dvf = np.full((n, 3, 3), np.nan)
                dvf[S1] = velocity_gradient(
                    gx, gy, gz, g.vx[gs], g.vy[gs], g.vz[gs], gh, V,
                    full["A"], full["B"], full["gradA"], full["gradB"],
                    targets=S1)
                res["dv"][sel] = dvf[T]
            ax, ay, az, du = hydro(
                gx, gy, gz, g.vx[gs], g.vy[gs], g.vz[gs], gh, gm, V,
                full["rho"], full["P"], full["cs"], full["A"], full["B"],
                full["gradA"], full["gradB"], params["Cl"], params["Cq"],
                params["epsQ"], targets=T, dv=dvf)
            res["V"][sel], res["rho_tilde"][sel] = V[T], rt[T]
            for k in ("A", "rho", "P", "cs", "B", "gradA", "gradB"):
                res[k][sel] = full[k][T]
            res["a_hydro"][:, sel] = (ax, ay, az)
            res["dudt"][sel] = du
            say(f"oracle box {b}: hydro forces done")
        X = np.concatenate([gx, d.x[ds]])
        Y = np.concatenate([gy, d.y[ds]])
        Z = np.concatenate([gz, d.z[ds]])
        M = np.concatenate([gm, d.m[ds]])
        tg = np.concatenate([gas_targets[sel] - gs.start,
                             dm_targets[dsel] - ds.start + n])
        ax, ay, az = gravity(X, Y, Z, M, float(wl.r_c[b]), float(wl.eps[b]),
                             params["G"], targets=tg)
        k = sel.size
        res["a_grav_gas"][:, sel] = (ax[:k], ay[:k], az[:k])
        res["a_grav_dm"][:, dsel] = (ax[k:], ay[k:], az[k:])
        say(f"oracle box {b}: gravity done")
    return res


# ----------------------------------------------------------------------------
# hierarchical time steps on a fixed tree (adaptive integration, Sec. IV-A;
# active leaves, Sec. IV-B.1).  The paper describes the scheme but prints no
# formulas; the readings below are stated where they are used.
# ----------------------------------------------------------------------------

# Time-step constants (readings): Courant factor for gas, accuracy parameter
# of the acceleration criterion dt = sqrt(2 eta eps / |a|).
STEP_PARAMS = dict(c_cfl=0.25, eta=0.025)


def timestep_bins(dt, max_level, eps, ax, ay, az, h=None, cs=None,
                  c_cfl=STEP_PARAMS["c_cfl"], eta=STEP_PARAMS["eta"]):
    """Bin level b in [0, max_level] of every particle: the smallest b whose
    step tau_b = dt / 2^b satisfies tau_b^4 |a|^2 <= (2 eta eps)^2 (the
    acceleration criterion squared twice) and, for gas (h and cs given),
    tau_b cs <= c_cfl h (Courant); max_level when none does.  Every
    quantity is a double product or sum rounded once, in this order, so
    that another implementation taking the same steps takes the same
    integer decision."""
    ax, ay, az = (np.asarray(a, np.float64) for a in (ax, ay, az))
    a2 = (ax * ax + ay * ay) + az * az
    r = 2.0 * eta * eps
    rhs_a = r * r
    n = ax.shape[0]
    bins = np.full(n, max_level, np.int32)
    done = np.zeros(n, bool)
    if h is not None:
        rhs_c = c_cfl * np.asarray(h, np.float64)
        cs = np.asarray(cs, np.float64)
    for b in range(max_level + 1):
        tau = dt * 2.0 ** (-b)
        t2 = tau * tau
        ok = (t2 * t2) * a2 <= rhs_a
        if h is not None:
            ok &= tau * cs <= rhs_c
        new = ok & ~done
        bins[new] = b
        done |= ok
    return bins


def _wrap(x):
    x = x - np.floor(x - 1.0)
    return np.where(x >= 2.0, x - 1.0, x)


def substep_cycle(wl, bins_gas, bins_dm, dt, max_level, params=PARAMS,
                  counts=None, forces_at="float64", pm_mesh=None,
                  recon=False, compatible=False):
    """One interval dt of hierarchical block steps (kick-drift-kick) with
    2^max_level substeps of dt / 2^max_level.  A particle of bin b takes
    steps tau_b = dt / 2^b, starting at substeps s with s % 2^(L-b) == 0
    (L = max_level) and ending after substeps s with (s + 1) % 2^(L-b) == 0.

    Readings: all particles are evaluated at the start; at each substep the
    particles starting a step get the opening half-kick v += a tau_b / 2,
    u += du/dt tau_b / 2 with their latest a and du/dt; every particle
    drifts x += v dt / 2^L; then the four passes run for the particles
    ending a step (density, coefficients, hydro forces and gravity at those
    particles only, over all neighbours at their current positions, with
    the latest values of inactive neighbours, their half-kicked v and u
    included) and they get the closing half-kick with the new a and du/dt.
    Smoothing lengths and masses stay fixed; positions are wrapped into
    [1, 2) at the end.  forces_at="float32" evaluates the passes at the
    float32 roundings of the double positions (not wrapped inside the
    interval), velocities and energies: the mixed-precision split of
    Sec. IV-A, where the short-range solver works on float32 copies of a
    double state.  pm_mesh (single box): the long-range mesh force brackets
    the interval, a half-kick v += a_long dt / 2 of every particle before
    the first substep (positions at the start) and after the last one
    (positions at the end, wrapped), as a long PM step encloses the short
    subcycles.  Returns the final x, v, u (float64, (3, n) / n per species)
    and the state of the last evaluation.  counts, if a dict, receives the
    number of evaluations of every particle.  recon: the hydro forces use
    the viscosity on the limited midpoint reconstruction, with the velocity
    gradients evaluated with the coefficients (latest values of inactive
    neighbours, like every other field).

    compatible: every half-kick of the gas takes the compatible energy
    update of CRKSPH (its energy conservation, Sec. IV-A) in place of the
    plain rate: a kick of the set K by widths w_i = tau_i / 2 changes u_i
    by w_i du_i/dt, where du_i/dt comes from the pair forces of i's latest
    evaluation (the velocities of that evaluation included) with the pair
    work taken at the kick's centred velocities c = v + w a / 2 for the
    particles of K and c = v for every other particle.  With one bin, or
    bins that differ only between particles that do not interact, and G = 0,
    sum m (v^2/2 + u) is then conserved to rounding; the returned dudt is
    the rate of each particle's final closing kick."""
    f32 = forces_at == "float32"

    def q(a):
        return a.astype(np.float32).astype(np.float64) if f32 else a
    g, d = wl.gas, wl.dm
    ng, nd = g.n, d.n
    L = int(max_level)
    bg = np.asarray(bins_gas, np.int64)
    bd = np.asarray(bins_dm, np.int64)
    xg = np.array([g.x, g.y, g.z], np.float64)
    vg = np.array([g.vx, g.vy, g.vz], np.float64)
    xd = np.array([d.x, d.y, d.z], np.float64)
    vd = np.array([d.vx, d.vy, d.vz], np.float64)
    u = np.asarray(g.u, np.float64).copy() if ng else np.zeros(0)
    st = {k: np.zeros(ng) for k in ("V", "rho_tilde", "A", "rho", "P", "cs",
                                     "dudt")}
    st.update(B=np.zeros((ng, 3)), gradA=np.zeros((ng, 3)),
              gradB=np.zeros((ng, 3, 3)), a_hydro=np.zeros((3, ng)),
              a_grav_gas=np.zeros((3, ng)), a_grav_dm=np.zeros((3, nd)),
              dv=np.zeros((ng, 3, 3)))
    ev_g = np.zeros(ng, np.int64)
    ev_d = np.zeros(nd, np.int64)
    v_eval = vg.copy()      # gas velocities at each particle's latest evaluation

    def evaluate(act_g, act_d):
        ev_g[act_g] += 1
        ev_d[act_d] += 1
        v_eval[:] = vg
        for b, gs, ds in _box_slices(wl):
            n = gs.stop - gs.start
            X = _wrap(q(xg[:, gs]))
            Tg = np.nonzero(act_g[gs])[0]
            if Tg.size:
                hh, mm = g.h[gs], g.m[gs]
                V, rt = density(X[0], X[1], X[2], hh, mm, targets=Tg)
                st["V"][gs.start + Tg] = V
                st["rho_tilde"][gs.start + Tg] = rt
                c = coefficients(X[0], X[1], X[2], hh, mm, st["V"][gs],
                                 q(u[gs]), params["gamma"], targets=Tg)
                for k in ("A", "B", "gradA", "gradB", "rho", "P", "cs"):
                    st[k][gs.start + Tg] = c[k]
                V3 = q(vg[:, gs])
                if recon:
                    st["dv"][gs.start + Tg] = velocity_gradient(
                        X[0], X[1], X[2], V3[0], V3[1], V3[2], hh,
                        st["V"][gs], st["A"][gs], st["B"][gs],
                        st["gradA"][gs], st["gradB"][gs], targets=Tg)
                ax, ay, az, du = hydro(
                    X[0], X[1], X[2], V3[0], V3[1], V3[2], hh, mm,
                    st["V"][gs], st["rho"][gs], st["P"][gs], st["cs"][gs],
                    st["A"][gs], st["B"][gs], st["gradA"][gs],
                    st["gradB"][gs], params["Cl"], params["Cq"],
                    params["epsQ"], targets=Tg,
                    dv=st["dv"][gs] if recon else None)
                st["a_hydro"][:, gs.start + Tg] = (ax, ay, az)
                st["dudt"][gs.start + Tg] = du
            Td = np.nonzero(act_d[ds])[0]
            if Tg.size or Td.size:
                XD = _wrap(q(xd[:, ds]))
                XA = np.concatenate([X, XD], axis=1)
                M = np.concatenate([g.m[gs], d.m[ds]])
                ax, ay, az = gravity(XA[0], XA[1], XA[2], M, float(wl.r_c[b]),
                                     float(wl.eps[b]), params["G"],
                                     targets=np.concatenate([Tg, Td + n]))
                k = Tg.size
                st["a_grav_gas"][:, gs.start + Tg] = (ax[:k], ay[:k], az[:k])
                st["a_grav_dm"][:, ds.start + Td] = (ax[k:], ay[k:], az[k:])

    def compatible_rate(act_g, w):
        """du/dt of the gas of the kick set act_g with kick widths w (n_gas,
        zero outside the set): the latest pair forces, whose velocities are
        v_eval, with the pair work at the centred velocities c, passed to
        hydro() as the velocities 2 c - v_eval after a kick from v_eval."""
        c = vg + 0.5 * w * (st["a_grav_gas"] + st["a_hydro"])
        v1 = 2.0 * c - v_eval
        rate = st["dudt"].copy()
        for b, gs, ds in _box_slices(wl):
            Tg = np.nonzero(act_g[gs])[0]
            if not Tg.size:
                continue
            X = _wrap(q(xg[:, gs]))
            V3 = q(v_eval[:, gs])
            _, _, _, du = hydro(
                X[0], X[1], X[2], V3[0], V3[1], V3[2], g.h[gs], g.m[gs],
                st["V"][gs], st["rho"][gs], st["P"][gs], st["cs"][gs],
                st["A"][gs], st["B"][gs], st["gradA"][gs], st["gradB"][gs],
                params["Cl"], params["Cq"], params["epsQ"], targets=Tg,
                dv=st["dv"][gs] if recon else None, v1=v1[:, gs])
            rate[gs.start + Tg] = du
        return rate

    def kick(act_g, act_d):
        tg = dt * 2.0 ** (-bg[act_g].astype(np.float64)) * 0.5
        td = dt * 2.0 ** (-bd[act_d].astype(np.float64)) * 0.5
        if compatible and ng:
            w = np.zeros(ng)
            w[act_g] = tg
            rate = compatible_rate(act_g, w)
            u[act_g] += rate[act_g] * tg
            st["dudt"][act_g] = rate[act_g]
        else:
            u[act_g] += st["dudt"][act_g] * tg
        vg[:, act_g] += (st["a_grav_gas"][:, act_g] + st["a_hydro"][:, act_g]) * tg
        vd[:, act_d] += st["a_grav_dm"][:, act_d] * td

    def long_kick():
        X = q(np.concatenate([xg, xd], axis=1))
        X = _wrap(X)
        M = np.concatenate([g.m, d.m])
        a = pm_long_range(X[0], X[1], X[2], M, pm_mesh, float(wl.r_c[0]),
                          params["G"])
        vg[:] += a[:, :ng] * (0.5 * dt)
        vd[:] += a[:, ng:] * (0.5 * dt)

    if pm_mesh:
        long_kick()
    evaluate(np.ones(ng, bool), np.ones(nd, bool))
    delta = dt * 2.0 ** (-L)
    for s in range(2 ** L):
        start_g = (s % (2 ** (L - bg))) == 0
        start_d = (s % (2 ** (L - bd))) == 0
        kick(start_g, start_d)
        xg += vg * delta
        xd += vd * delta
        end_g = ((s + 1) % (2 ** (L - bg))) == 0
        end_d = ((s + 1) % (2 ** (L - bd))) == 0
        evaluate(end_g, end_d)
        kick(end_g, end_d)
    if pm_mesh:
        xg[:] = _wrap(xg)
        xd[:] = _wrap(xd)
        long_kick()
    if counts is not None:
        counts["gas"] = ev_g
        counts["dm"] = ev_d
    out = dict(xg=_wrap(xg), vg=vg, u=u, xd=_wrap(xd), vd=vd)
    out.update(st)
    return out


# ----------------------------------------------------------------------------
# long-range gravity on a mesh, matched to the short-range split (the
# spectral particle-mesh part of Sec. IV-A; the paper's filtered PM method
# and SWFFT are not printed, so the steps below are the textbook
# particle-mesh method with the S2 split of Hockney & Eastwood).
# ----------------------------------------------------------------------------

def s2_form_factor(k, r_c):
    """Fourier transform of the S2 cloud of diameter r_c (unit mass, density
    falling linearly from the centre to radius r_c / 2): with x = k r_c / 2,
    12 (2 - 2 cos x - x sin x) / x^4, 1 at k = 0 (series below x = 1e-2)."""
    x = np.asarray(k, np.float64) * (0.5 * r_c)
    out = np.ones_like(x)
    big = x > 1e-2
    xb = x[big]
    out[big] = 12.0 * (2.0 - 2.0 * np.cos(xb) - xb * np.sin(xb)) / xb ** 4
    xs = x[~big]
    out[~big] = 1.0 - xs ** 2 / 15.0 + xs ** 4 / 560.0
    return out


def pm_long_range(x, y, z, m, n_mesh, r_c, G=PARAMS["G"]):
    """Long-range acceleration of every particle of one periodic unit box
    (coordinates in [1, 2)): the force between S2 clouds of diameter r_c,
    i.e. the complement of the short-range force, on an n_mesh^3 mesh.
    Steps: cloud-in-cell deposit of the masses on the nodes j / n_mesh;
    FFT; multiplication by -4 pi G S2(k)^2 / k^2 (the mean removed) divided
    by the squared CIC window prod_a sinc^4(k_a / (2 n_mesh)) (deposit and
    interpolation); spectral gradient i k (Nyquist planes zeroed); three
    inverse FFTs; cloud-in-cell interpolation back to the particles."""
    N = int(n_mesh)
    P = np.stack([np.asarray(a, np.float64) for a in (x, y, z)])
    m = np.asarray(m, np.float64)
    u = (P - 1.0) * N
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    i0 %= N
    i1 = (i0 + 1) % N
    rho = np.zeros((N, N, N))
    for cx in (0, 1):
        wx = f[0] if cx else 1.0 - f[0]
        ix = i1[0] if cx else i0[0]
        for cy in (0, 1):
            wy = f[1] if cy else 1.0 - f[1]
            iy = i1[1] if cy else i0[1]
            for cz in (0, 1):
                wz = f[2] if cz else 1.0 - f[2]
                iz = i1[2] if cz else i0[2]
                np.add.at(rho, (ix, iy, iz), m * wx * wy * wz)
    rho *= N ** 3  # mass per cell volume
    rk = np.fft.rfftn(rho)
    n1 = np.fft.fftfreq(N, 1.0 / N)
    nz = np.fft.rfftfreq(N, 1.0 / N)
    KX, KY, KZ = np.meshgrid(2 * np.pi * n1, 2 * np.pi * n1, 2 * np.pi * nz,
                             indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k = np.sqrt(k2)
    h = 0.5 / N

    def sinc(t):
        return np.where(t == 0, 1.0, np.sin(t) / np.where(t == 0, 1.0, t))

    W = (sinc(KX * h) * sinc(KY * h) * sinc(KZ * h)) ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        gk = np.where(k2 > 0, 4 * np.pi * G * s2_form_factor(k, r_c) ** 2
                      / (k2 * W * W), 0.0)
    nyq = N // 2
    acc = []
    for K, axis_ny in ((KX, np.abs(n1)[:, None, None] == nyq),
                       (KY, np.abs(n1)[None, :, None] == nyq),
                       (KZ, (nz == nyq)[None, None, :])):
        Kd = np.where(axis_ny, 0.0, K)
        field = np.fft.irfftn(1j * Kd * gk * rk, s=(N, N, N), axes=(0, 1, 2))
        a = np.zeros(P.shape[1])
        for cx in (0, 1):
            wx = f[0] if cx else 1.0 - f[0]
            ix = i1[0] if cx else i0[0]
            for cy in (0, 1):
                wy = f[1] if cy else 1.0 - f[1]
                iy = i1[1] if cy else i0[1]
                for cz in (0, 1):
                    wz = f[2] if cz else 1.0 - f[2]
                    iz = i1[2] if cz else i0[2]
                    a += wx * wy * wz * field[ix, iy, iz]
        acc.append(a)
    return np.stack(acc)


# ----------------------------------------------------------------------------
# friends-of-friends groups on the same box (the in-situ halo finding of
# Sec. IV-B.3, as a second pair workload: links instead of sums)
# ----------------------------------------------------------------------------

def _link_r2(P, i, j):
    """Squared minimum-image separations of index pairs (i, j), each
    difference and the sum formed in double in this order."""
    d = P[:, i] - P[:, j]
    d = d - np.round(d)
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2]


def fof_labels(x, y, z, b, brute=False):
    """Friends-of-friends groups of one periodic unit box (coordinates in
    [1, 2)): particles closer than the linking length b (strictly) are
    friends, groups are the connected components of the friendship graph,
    and every particle is labelled with the smallest index in its group.
    Candidate pairs come from a periodic k-d tree queried slightly beyond
    b (or from all pairs when brute), then the exact test r^2 < b^2 in
    double decides."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    P = np.stack([np.asarray(a, np.float64) for a in (x, y, z)])
    n = P.shape[1]
    if n == 0:
        return np.zeros(0, np.int64)
    if brute:
        ii, jj = np.triu_indices(n, 1)
    else:
        from scipy.spatial import cKDTree
        pts = np.mod(P.T - 1.0, 1.0)
        pairs = cKDTree(pts, boxsize=1.0).query_pairs(b * (1 + 1e-9),
                                                      output_type="ndarray")
        ii, jj = (pairs[:, 0], pairs[:, 1]) if len(pairs) else (
            np.zeros(0, np.int64), np.zeros(0, np.int64))
    b2 = b * b
    keep = _link_r2(P, ii, jj) < b2
    ii, jj = ii[keep], jj[keep]
    g = coo_matrix((np.ones(ii.size), (ii, jj)), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    first = np.full(comp.max() + 1, n, np.int64)
    np.minimum.at(first, comp, np.arange(n))
    return first[comp]


def fof_properties(x, y, z, m, labels):
    """Per group of a friends-of-friends labelling (groups indexed by their
    label, the smallest member index; Sec. IV-B.3 finds halos in situ):
    member count, total mass and the periodic centre of mass -- every member
    taken at its minimum image about the labelling particle, the
    mass-weighted mean of those images, wrapped into [1, 2).  Returns
    count (n,), mass (n,) and centre (3, n), zero at indices that label no
    group."""
    P = np.stack([np.asarray(a, np.float64) for a in (x, y, z)])
    m = np.asarray(m, np.float64)
    lab = np.asarray(labels, np.int64)
    n = lab.shape[0]
    count = np.bincount(lab, minlength=n).astype(np.int64)
    mass = np.bincount(lab, weights=m, minlength=n)
    com = np.zeros((3, n))
    has = count > 0
    for a in range(3):
        d = P[a] - P[a][lab]
        d = d - np.round(d)
        s = np.bincount(lab, weights=m * d, minlength=n)
        c = P[a] + np.where(has, s / np.where(has, mass, 1.0), 0.0)
        c = np.where(c >= 2.0, c - 1.0, np.where(c < 1.0, c + 1.0, c))
        com[a] = np.where(has, c, 0.0)
    return count, mass, com
