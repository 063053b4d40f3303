"""ctypes binding of libcrk.so (the C ABI declared in include/crk.h).

Argument marshalling only: every step of the short-range step runs in the
library's HIP kernels.  torch tensors serve as device buffers and the torch
stream as the HIP stream.  The binding raises if the library is missing;
there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
LIB_PATH = Path(os.environ.get("CRK_LIB", _HERE / "libcrk.so"))

CRK_OK, CRK_EINVAL, CRK_ECAPACITY, CRK_EDEVICE, CRK_ESTATE = 0, -1, -2, -3, -4
CRK_ESTALE = -5
CRK_FP64, CRK_FP32 = 0, 1
PASS_NAMES = ("tree", "lists", "density", "coefficients", "hydro", "gravity",
              "integrate", "velocity_gradient", "energy")

EXPORTS = (
    "crk_ctx_create", "crk_ctx_destroy", "crk_set_tuning", "crk_get_tuning",
    "crk_last_error", "crk_sync", "build_tree", "build_interaction_lists",
    "crk_density", "crk_coefficients", "crk_hydro_forces",
    "shortrange_gravity", "crk_integrate", "crk_tree_get_info",
    "crk_tree_get_leaves", "crk_count_pairs", "crk_graph_begin", "crk_graph_end",
    "crk_graph_launch", "crk_tree_free", "crk_timing_enable",
    "crk_pass_times", "crk_timestep_bins", "crk_tree_set_active",
    "crk_tree_refit", "crk_kick", "crk_drift", "crk_pm_gravity", "crk_fof",
    "crk_velocity_gradient", "crk_hydro_forces_limited",
    "crk_hydro_energy_compatible", "crk_fof_properties",
)


class CrkError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"crk status {status}: {msg}")
        self.status = status


class crk_params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("Cl", ctypes.c_double),
                ("Cq", ctypes.c_double), ("epsQ", ctypes.c_double),
                ("G", ctypes.c_double)]


class crk_boxes(ctypes.Structure):
    _fields_ = [("n_boxes", ctypes.c_int32),
                ("gas_off", ctypes.POINTER(ctypes.c_int64)),
                ("dm_off", ctypes.POINTER(ctypes.c_int64)),
                ("r_c", ctypes.POINTER(ctypes.c_double)),
                ("eps", ctypes.POINTER(ctypes.c_double)),
                ("h_max", ctypes.POINTER(ctypes.c_double))]


class crk_tuning(ctypes.Structure):
    _fields_ = [("leaf_max", ctypes.c_int32), ("cm_factor", ctypes.c_double),
                ("grid_mult", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("walk_mask", ctypes.c_int32), ("sub_sweep", ctypes.c_int32),
                ("tree_lds", ctypes.c_int32)]


class crk_tree_info(ctypes.Structure):
    _fields_ = [("n_gas", ctypes.c_int64), ("n_dm", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("n_gas_leaves", ctypes.c_int64),
                ("n_bins", ctypes.c_int64), ("grav_entries", ctypes.c_int64),
                ("hydro_entries", ctypes.c_int64), ("kd_levels", ctypes.c_int32)]


_lib = None
_exiting = False
_live_trees = weakref.WeakSet()
_live_ctxs = weakref.WeakSet()


def _release_all():
    """Destroys every tree and context still alive at interpreter exit, while
    the HIP runtime is still fully up (trees first, then contexts); native
    teardown is skipped for anything finalised later."""
    global _exiting
    for t in list(_live_trees):
        try:
            t.free()
        except Exception:
            pass
    for c in list(_live_ctxs):
        try:
            c.close()
        except Exception:
            pass
    _exiting = True


atexit.register(_release_all)


def load(path: Path | str | None = None):
    """Loads libcrk.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise ImportError(f"{p} is missing: build it with "
                          "`python -m paper_2510_03557_amd.build`")
    lib = ctypes.CDLL(str(p))
    vp = ctypes.c_void_p
    lib.crk_last_error.restype = ctypes.c_char_p
    lib.crk_last_error.argtypes = []
    lib.crk_ctx_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp,
                                   ctypes.POINTER(crk_params)]
    lib.crk_ctx_destroy.argtypes = [vp]
    lib.crk_set_tuning.argtypes = [vp, ctypes.POINTER(crk_tuning)]
    lib.crk_get_tuning.argtypes = [vp, ctypes.POINTER(crk_tuning)]
    lib.crk_sync.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.build_tree.argtypes = [vp, ctypes.POINTER(crk_boxes)] + [vp] * 7 + \
        [ctypes.POINTER(vp)]
    lib.build_interaction_lists.argtypes = [vp, vp]
    lib.crk_density.argtypes = [vp, vp, vp, vp, vp]
    lib.crk_coefficients.argtypes = [vp] * 12
    lib.crk_hydro_forces.argtypes = [vp] * 18
    lib.crk_velocity_gradient.argtypes = [vp] * 11
    lib.crk_hydro_forces_limited.argtypes = [vp] * 15 + [ctypes.c_double] * 2 \
        + [vp] * 4
    lib.crk_hydro_energy_compatible.argtypes = [vp] * 15 + \
        [ctypes.c_double] * 3 + [ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.shortrange_gravity.argtypes = [vp] * 10
    lib.crk_integrate.argtypes = [vp, ctypes.c_int64, ctypes.c_double, vp, vp,
                                  vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  vp]
    lib.crk_tree_get_info.argtypes = [vp, ctypes.POINTER(crk_tree_info)]
    lib.crk_tree_get_leaves.argtypes = [vp, vp, vp, vp, vp]
    lib.crk_count_pairs.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int64)]
    lib.crk_graph_begin.argtypes = [vp]
    lib.crk_graph_end.argtypes = [vp]
    lib.crk_graph_launch.argtypes = [vp]
    lib.crk_tree_free.argtypes = [vp]
    lib.crk_timing_enable.argtypes = [vp, ctypes.c_int]
    lib.crk_pass_times.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_int64)]
    P = ctypes.POINTER(vp)
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.crk_timestep_bins.argtypes = [vp, i64, f64, i32, f64, f64, f64, P, P,
                                      vp, vp, vp]
    lib.crk_tree_set_active.argtypes = [vp, vp, vp, vp, i32, i64]
    lib.crk_tree_refit.argtypes = [vp, vp] + [vp] * 6
    lib.crk_kick.argtypes = [vp, i64, f64, i32, i64, i32, vp, vp, vp, P, P, vp,
                             P, vp]
    lib.crk_drift.argtypes = [vp, i64, f64, i32, vp, vp, P]
    lib.crk_pm_gravity.argtypes = [vp, i32, f64, i64, vp, vp, vp, vp, i64, vp,
                                   vp, vp, vp, P, P]
    lib.crk_fof.argtypes = [vp, vp, f64, vp, vp]
    lib.crk_fof_properties.argtypes = [vp, i64, i64, vp, vp, P, vp, P, vp,
                                       vp, vp, vp]
    for name in EXPORTS:
        getattr(lib, name).restype = (ctypes.c_char_p if name == "crk_last_error"
                                      else ctypes.c_int)
    if path is None:
        _lib = lib
    return lib


def last_error() -> str:
    return load().crk_last_error().decode()


def check(status: int):
    if status != CRK_OK:
        raise CrkError(status, last_error())


def _ptr(t):
    """Device address of a torch tensor (None -> NULL)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _arr(ctype, vals):
    a = (ctype * len(vals))(*vals)
    return a


class Context:
    """A library context bound to one HIP stream."""

    def __init__(self, precision: str = "fp32", stream=None, params=None):
        import torch
        self.lib = load()
        self.precision = precision
        self.torch = torch
        self.dtype = torch.float32 if precision == "fp32" else torch.float64
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self._boxes_keep = None
        h = ctypes.c_void_p()
        p = None
        if params is not None:
            p = ctypes.byref(crk_params(**params))
        check(self.lib.crk_ctx_create(
            ctypes.byref(h), CRK_FP32 if precision == "fp32" else CRK_FP64,
            ctypes.c_void_p(self.stream.cuda_stream), p))
        self.handle = h
        _live_ctxs.add(self)

    def close(self):
        if getattr(self, "handle", None) and not _exiting:
            self.lib.crk_ctx_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, leaf_max=64, cm_factor=0.0, grid_mult=0, xcd_remap=1,
                   walk_mask=0, sub_sweep=2, tree_lds=1):
        check(self.lib.crk_set_tuning(self.handle, ctypes.byref(
            crk_tuning(int(leaf_max), float(cm_factor), int(grid_mult),
                       int(xcd_remap), int(walk_mask), int(sub_sweep),
                       int(tree_lds)))))

    def sync(self):
        req = ctypes.c_int64()
        check(self.lib.crk_sync(self.handle, ctypes.byref(req)))
        return req.value

    def build_tree(self, tree, gas_off, dm_off, r_c, eps, h_max, gx, gy, gz,
                   gh, dx, dy, dz):
        """tree: a Tree object (created empty) whose handle is filled."""
        go = np.ascontiguousarray(gas_off, np.int64)
        do = np.ascontiguousarray(dm_off, np.int64)
        rc = np.ascontiguousarray(r_c, np.float64)
        ep = np.ascontiguousarray(eps, np.float64)
        hm = np.ascontiguousarray(h_max, np.float64)
        keep = (go, do, rc, ep, hm)
        b = crk_boxes(len(go) - 1,
                      go.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      do.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      rc.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      ep.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                      hm.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self._boxes_keep = (keep, b)
        check(self.lib.build_tree(self.handle, ctypes.byref(b), _ptr(gx),
                                  _ptr(gy), _ptr(gz), _ptr(gh), _ptr(dx),
                                  _ptr(dy), _ptr(dz),
                                  ctypes.byref(tree.handle)))

    def build_interaction_lists(self, tree):
        check(self.lib.build_interaction_lists(self.handle, tree.handle))

    def density(self, tree, m, V, rho_t):
        check(self.lib.crk_density(self.handle, tree.handle, _ptr(m), _ptr(V),
                                   _ptr(rho_t)))

    def coefficients(self, tree, m, V, u, A, B, gA, gB, rho, P, cs):
        check(self.lib.crk_coefficients(self.handle, tree.handle, _ptr(m),
                                        _ptr(V), _ptr(u), _ptr(A), _ptr(B),
                                        _ptr(gA), _ptr(gB), _ptr(rho), _ptr(P),
                                        _ptr(cs)))

    def hydro_forces(self, tree, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB,
                     ax, ay, az, dudt):
        check(self.lib.crk_hydro_forces(
            self.handle, tree.handle, _ptr(m), _ptr(vx), _ptr(vy), _ptr(vz),
            _ptr(V), _ptr(rho), _ptr(P), _ptr(cs), _ptr(A), _ptr(B), _ptr(gA),
            _ptr(gB), _ptr(ax), _ptr(ay), _ptr(az), _ptr(dudt)))

    def velocity_gradient(self, tree, vx, vy, vz, V, A, B, gA, gB, dv):
        check(self.lib.crk_velocity_gradient(
            self.handle, tree.handle, _ptr(vx), _ptr(vy), _ptr(vz), _ptr(V),
            _ptr(A), _ptr(B), _ptr(gA), _ptr(gB), _ptr(dv)))

    def hydro_forces_limited(self, tree, m, vx, vy, vz, V, rho, P, cs, A, B,
                             gA, gB, dv, eta_crit, eta_fold, ax, ay, az, dudt):
        check(self.lib.crk_hydro_forces_limited(
            self.handle, tree.handle, _ptr(m), _ptr(vx), _ptr(vy), _ptr(vz),
            _ptr(V), _ptr(rho), _ptr(P), _ptr(cs), _ptr(A), _ptr(B), _ptr(gA),
            _ptr(gB), _ptr(dv), float(eta_crit), float(eta_fold), _ptr(ax),
            _ptr(ay), _ptr(az), _ptr(dudt)))

    def hydro_energy_compatible(self, tree, m, vx, vy, vz, V, rho, P, cs, A,
                                B, gA, gB, dv, eta_crit, eta_fold, dt, a_grav,
                                a_hydro, dudt):
        P3 = ctypes.c_void_p * 3
        ag = P3(*[t.data_ptr() for t in a_grav]) if a_grav is not None else None
        ah = P3(*[t.data_ptr() for t in a_hydro]) if a_hydro is not None else None
        check(self.lib.crk_hydro_energy_compatible(
            self.handle, tree.handle, _ptr(m), _ptr(vx), _ptr(vy), _ptr(vz),
            _ptr(V), _ptr(rho), _ptr(P), _ptr(cs), _ptr(A), _ptr(B), _ptr(gA),
            _ptr(gB), _ptr(dv), float(eta_crit), float(eta_fold), float(dt),
            ag, ah, _ptr(dudt)))

    def shortrange_gravity(self, tree, m_gas, m_dm, axg, ayg, azg, axd, ayd,
                           azd):
        check(self.lib.shortrange_gravity(
            self.handle, tree.handle, _ptr(m_gas), _ptr(m_dm), _ptr(axg),
            _ptr(ayg), _ptr(azg), _ptr(axd), _ptr(ayd), _ptr(azd)))

    def integrate(self, n, dt, x64, v64, u64, a_grav, a_hydro, dudt, x, v, u):
        P3 = ctypes.c_void_p * 3
        ag = P3(*[t.data_ptr() for t in a_grav])
        ah = P3(*[t.data_ptr() for t in a_hydro]) if a_hydro is not None else None
        xo = P3(*[t.data_ptr() for t in x])
        vo = P3(*[t.data_ptr() for t in v])
        check(self.lib.crk_integrate(
            self.handle, int(n), float(dt), _ptr(x64), _ptr(v64), _ptr(u64),
            ag, ah, _ptr(dudt), xo, vo, _ptr(u)))

    # hierarchical time steps ------------------------------------------------
    @staticmethod
    def _p3(ts):
        if ts is None:
            return None
        return (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ts])

    def timestep_bins(self, n, dt, max_level, eps, c_cfl, eta, a_grav,
                      a_hydro, h, cs, bins):
        check(self.lib.crk_timestep_bins(
            self.handle, int(n), float(dt), int(max_level), float(eps),
            float(c_cfl), float(eta), self._p3(a_grav), self._p3(a_hydro),
            _ptr(h), _ptr(cs), _ptr(bins)))

    def tree_set_active(self, tree, bins_gas, bins_dm, max_level, substep):
        check(self.lib.crk_tree_set_active(
            self.handle, tree.handle, _ptr(bins_gas), _ptr(bins_dm),
            int(max_level), int(substep)))

    def tree_refit(self, tree, gx, gy, gz, dx, dy, dz):
        check(self.lib.crk_tree_refit(self.handle, tree.handle, _ptr(gx),
                                      _ptr(gy), _ptr(gz), _ptr(dx), _ptr(dy),
                                      _ptr(dz)))

    def kick(self, n, dt, max_level, substep, phase, bins, v64, u64, a_grav,
             a_hydro, dudt, v, u):
        check(self.lib.crk_kick(
            self.handle, int(n), float(dt), int(max_level), int(substep),
            int(phase), _ptr(bins), _ptr(v64), _ptr(u64), self._p3(a_grav),
            self._p3(a_hydro), _ptr(dudt), self._p3(v), _ptr(u)))

    def drift(self, n, delta, wrap, x64, v64, x):
        check(self.lib.crk_drift(self.handle, int(n), float(delta),
                                 int(bool(wrap)), _ptr(x64), _ptr(v64),
                                 self._p3(x)))

    def pm_gravity(self, n_mesh, r_c, n_gas, gx, gy, gz, m_gas, n_dm, dx, dy,
                   dz, m_dm, a_gas, a_dm):
        check(self.lib.crk_pm_gravity(
            self.handle, int(n_mesh), float(r_c), int(n_gas), _ptr(gx),
            _ptr(gy), _ptr(gz), _ptr(m_gas), int(n_dm), _ptr(dx), _ptr(dy),
            _ptr(dz), _ptr(m_dm), self._p3(a_gas), self._p3(a_dm)))

    def fof(self, tree, b, labels_gas, labels_dm):
        check(self.lib.crk_fof(self.handle, tree.handle, float(b),
                               _ptr(labels_gas), _ptr(labels_dm)))

    def fof_properties(self, n_gas, n_dm, labels_gas, labels_dm, gas_x, m_gas,
                       dm_x, m_dm, count, mass, centre):
        check(self.lib.crk_fof_properties(
            self.handle, int(n_gas), int(n_dm), _ptr(labels_gas),
            _ptr(labels_dm), self._p3(gas_x), _ptr(m_gas), self._p3(dm_x),
            _ptr(m_dm), _ptr(count), _ptr(mass), _ptr(centre)))

    def count_pairs(self, tree):
        """In-range ordered pairs (gather, hydro, gravity), then the swept
        candidate pairs of the same three sweeps."""
        a = (ctypes.c_int64 * 6)()
        check(self.lib.crk_count_pairs(self.handle, tree.handle, a))
        return tuple(int(v) for v in a)

    def graph_begin(self):
        check(self.lib.crk_graph_begin(self.handle))

    def graph_end(self):
        check(self.lib.crk_graph_end(self.handle))

    def graph_launch(self):
        check(self.lib.crk_graph_launch(self.handle))

    def timing(self, enable=True):
        check(self.lib.crk_timing_enable(self.handle, int(bool(enable))))

    def pass_times(self):
        a = (ctypes.c_double * 9)()
        b = (ctypes.c_double * 9)()
        c = (ctypes.c_int64 * 9)()
        check(self.lib.crk_pass_times(self.handle, a, b, c))
        return ({k: a[i] for i, k in enumerate(PASS_NAMES)},
                {k: b[i] for i, k in enumerate(PASS_NAMES)},
                {k: c[i] for i, k in enumerate(PASS_NAMES)})


class Tree:
    """An opaque tree handle (built by Context.build_tree)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.handle = ctypes.c_void_p()
        _live_trees.add(self)

    def info(self):
        i = crk_tree_info()
        check(self.ctx.lib.crk_tree_get_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in crk_tree_info._fields_}

    def leaves(self):
        inf = self.info()
        n = inf["n_gas"] + inf["n_dm"]
        nl = inf["n_leaves"]
        perm = np.zeros(n, np.int64)
        st = np.zeros(nl, np.int64)
        cn = np.zeros(nl, np.int64)
        check(self.ctx.lib.crk_tree_get_leaves(
            self.ctx.handle, self.handle, perm.ctypes.data_as(ctypes.c_void_p),
            st.ctypes.data_as(ctypes.c_void_p),
            cn.ctypes.data_as(ctypes.c_void_p)))
        return perm, st, cn

    def free(self):
        if self.handle and not _exiting:
            self.ctx.lib.crk_tree_free(self.handle)
        self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
