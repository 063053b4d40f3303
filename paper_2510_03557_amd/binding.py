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
    "crk_density", "crk_density_noalloc", "crk_coefficients",
    "crk_hydro_forces",
    "shortrange_gravity", "crk_integrate", "crk_tree_get_info",
    "crk_tree_get_leaves", "crk_count_pairs", "crk_graph_begin", "crk_graph_end",
    "crk_graph_launch", "crk_graph_reset", "crk_tree_free", "crk_timing_enable",
    "crk_pass_times", "crk_timestep_bins", "crk_tree_set_active",
    "crk_tree_refit", "crk_kick", "crk_drift", "crk_pm_gravity", "crk_fof",
    "crk_velocity_gradient", "crk_hydro_forces_limited",
    "crk_hydro_energy_compatible", "crk_hydro_energy_compatible_block",
    "crk_fof_properties",
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
                ("tree_lds", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("act_groups", ctypes.c_int32)]


class crk_tree_info(ctypes.Structure):
    _fields_ = [("n_gas", ctypes.c_int64), ("n_dm", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("n_gas_leaves", ctypes.c_int64),
                ("n_bins", ctypes.c_int64), ("grav_entries", ctypes.c_int64),
                ("hydro_entries", ctypes.c_int64), ("kd_levels", ctypes.c_int32),
                ("act_leaves", ctypes.c_int64), ("act_particles", ctypes.c_int64),
                ("act_grouped", ctypes.c_int32)]


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
    lib.crk_density_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.crk_coefficients.argtypes = [vp] * 12
    lib.crk_hydro_forces.argtypes = [vp] * 18
    lib.crk_velocity_gradient.argtypes = [vp] * 11
    lib.crk_hydro_forces_limited.argtypes = [vp] * 15 + [ctypes.c_double] * 2 \
        + [vp] * 4
    lib.crk_hydro_energy_compatible.argtypes = [vp] * 15 + \
        [ctypes.c_double] * 3 + [ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
    lib.crk_hydro_energy_compatible_block.argtypes = [vp] * 15 + \
        [ctypes.c_double] * 3 + [ctypes.c_int32, vp, ctypes.c_int64,
                                 ctypes.POINTER(vp), ctypes.POINTER(vp), vp]
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
    lib.crk_graph_reset.argtypes = [vp]
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
    """Device address of a torch tensor (None -> NULL), unchecked: for
    buffers the caller of this module never supplies."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def check_tensor(t, dtype, n: int, name: str):
    """Raises CrkError(CRK_EINVAL) unless t is a contiguous device tensor of
    dtype with at least n elements; the library reads and writes raw
    addresses, so a wrong type or a short array would be misread or
    overrun rather than reported.  None passes (a NULL argument, which the
    library checks)."""
    if t is None:
        return
    if t.dtype != dtype:
        raise CrkError(CRK_EINVAL, f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise CrkError(CRK_EINVAL, f"{name}: not contiguous")
    if t.numel() < n:
        raise CrkError(CRK_EINVAL,
                       f"{name}: {t.numel()} elements, at least {n} needed")
    if not t.is_cuda:
        raise CrkError(CRK_EINVAL, f"{name}: not a device tensor")


def _dev(t, dtype, n, name):
    """check_tensor, then the device address (None -> NULL)."""
    check_tensor(t, dtype, n, name)
    return _ptr(t)


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
                   walk_mask=0, sub_sweep=2, tree_lds=1, tile=0,
                   act_groups=1):
        check(self.lib.crk_set_tuning(self.handle, ctypes.byref(
            crk_tuning(int(leaf_max), float(cm_factor), int(grid_mult),
                       int(xcd_remap), int(walk_mask), int(sub_sweep),
                       int(tree_lds), int(tile), int(act_groups)))))

    def get_tuning(self) -> dict:
        t = crk_tuning()
        check(self.lib.crk_get_tuning(self.handle, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in crk_tuning._fields_}

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
        F = self.dtype
        ng, nd = int(go[-1]), int(do[-1])
        args = [_dev(gx, F, ng, "gx"), _dev(gy, F, ng, "gy"),
                _dev(gz, F, ng, "gz"), _dev(gh, F, ng, "gh"),
                _dev(dx, F, nd, "dx"), _dev(dy, F, nd, "dy"),
                _dev(dz, F, nd, "dz")]
        check(self.lib.build_tree(self.handle, ctypes.byref(b), *args,
                                  ctypes.byref(tree.handle)))
        tree.n_gas, tree.n_dm = ng, nd

    def build_interaction_lists(self, tree):
        check(self.lib.build_interaction_lists(self.handle, tree.handle))

    # argument checks: F is the context precision; gas arrays hold n_gas
    # values per plane, dm arrays n_dm (from the tree)
    def _g(self, tree, t, planes, name, dtype=None):
        return _dev(t, dtype or self.dtype, planes * tree.n_gas, name)

    def _p3(self, ts, n, name, dtype=None):
        """Three plane pointers (None -> NULL), each checked for n values."""
        if ts is None:
            return None
        ts = list(ts)
        if len(ts) != 3:
            raise CrkError(CRK_EINVAL, f"{name}: three planes expected")
        for k, t in enumerate(ts):
            if t is None:
                raise CrkError(CRK_EINVAL, f"{name}[{k}]: null plane")
        for k, t in enumerate(ts):
            check_tensor(t, dtype or self.dtype, n, f"{name}[{k}]")
        return (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ts])

    def density(self, tree, m, V, rho_t):
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        check(self.lib.crk_density(self.handle, tree.handle, g(m, 1, "m"),
                                   g(V, 1, "V"), g(rho_t, 1, "rho_tilde")))

    def density_noalloc(self, tree, m, V, rho_t):
        """crk_density with the library's static scratch (no allocation)."""
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        check(self.lib.crk_density_noalloc(self.handle, tree.handle,
                                           g(m, 1, "m"), g(V, 1, "V"),
                                           g(rho_t, 1, "rho_tilde")))

    def coefficients(self, tree, m, V, u, A, B, gA, gB, rho, P, cs):
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        check(self.lib.crk_coefficients(
            self.handle, tree.handle, g(m, 1, "m"), g(V, 1, "V"), g(u, 1, "u"),
            g(A, 1, "A"), g(B, 3, "B"), g(gA, 3, "gradA"), g(gB, 9, "gradB"),
            g(rho, 1, "rho"), g(P, 1, "P"), g(cs, 1, "cs")))

    def _hydro_in(self, tree, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB):
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        return [g(m, 1, "m"), g(vx, 1, "vx"), g(vy, 1, "vy"), g(vz, 1, "vz"),
                g(V, 1, "V"), g(rho, 1, "rho"), g(P, 1, "P"), g(cs, 1, "cs"),
                g(A, 1, "A"), g(B, 3, "B"), g(gA, 3, "gradA"),
                g(gB, 9, "gradB")]

    def hydro_forces(self, tree, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB,
                     ax, ay, az, dudt):
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        check(self.lib.crk_hydro_forces(
            self.handle, tree.handle,
            *self._hydro_in(tree, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB),
            g(ax, 1, "ax"), g(ay, 1, "ay"), g(az, 1, "az"),
            g(dudt, 1, "dudt")))

    def velocity_gradient(self, tree, vx, vy, vz, V, A, B, gA, gB, dv):
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        check(self.lib.crk_velocity_gradient(
            self.handle, tree.handle, g(vx, 1, "vx"), g(vy, 1, "vy"),
            g(vz, 1, "vz"), g(V, 1, "V"), g(A, 1, "A"), g(B, 3, "B"),
            g(gA, 3, "gradA"), g(gB, 9, "gradB"), g(dv, 9, "dv")))

    def hydro_forces_limited(self, tree, m, vx, vy, vz, V, rho, P, cs, A, B,
                             gA, gB, dv, eta_crit, eta_fold, ax, ay, az, dudt):
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        check(self.lib.crk_hydro_forces_limited(
            self.handle, tree.handle,
            *self._hydro_in(tree, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB),
            g(dv, 9, "dv"), float(eta_crit), float(eta_fold), g(ax, 1, "ax"),
            g(ay, 1, "ay"), g(az, 1, "az"), g(dudt, 1, "dudt")))

    def hydro_energy_compatible(self, tree, m, vx, vy, vz, V, rho, P, cs, A,
                                B, gA, gB, dv, eta_crit, eta_fold, dt, a_grav,
                                a_hydro, dudt):
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        n = tree.n_gas
        check(self.lib.crk_hydro_energy_compatible(
            self.handle, tree.handle,
            *self._hydro_in(tree, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB),
            g(dv, 9, "dv"), float(eta_crit), float(eta_fold), float(dt),
            self._p3(a_grav, n, "a_grav"), self._p3(a_hydro, n, "a_hydro"),
            g(dudt, 1, "dudt")))

    def hydro_energy_compatible_block(self, tree, m, vx, vy, vz, V, rho, P,
                                      cs, A, B, gA, gB, dv, eta_crit,
                                      eta_fold, dt, max_level, bins_gas,
                                      substep, a_grav, a_hydro, dudt):
        import torch
        g = lambda t, k, nm: self._g(tree, t, k, nm)
        n = tree.n_gas
        check(self.lib.crk_hydro_energy_compatible_block(
            self.handle, tree.handle,
            *self._hydro_in(tree, m, vx, vy, vz, V, rho, P, cs, A, B, gA, gB),
            g(dv, 9, "dv"), float(eta_crit), float(eta_fold), float(dt),
            int(max_level), _dev(bins_gas, torch.int32, n, "bins_gas"),
            int(substep), self._p3(a_grav, n, "a_grav"),
            self._p3(a_hydro, n, "a_hydro"), g(dudt, 1, "dudt")))

    def shortrange_gravity(self, tree, m_gas, m_dm, axg, ayg, azg, axd, ayd,
                           azd):
        F, ng, nd = self.dtype, tree.n_gas, tree.n_dm
        check(self.lib.shortrange_gravity(
            self.handle, tree.handle, _dev(m_gas, F, ng, "m_gas"),
            _dev(m_dm, F, nd, "m_dm"), _dev(axg, F, ng, "ax_gas"),
            _dev(ayg, F, ng, "ay_gas"), _dev(azg, F, ng, "az_gas"),
            _dev(axd, F, nd, "ax_dm"), _dev(ayd, F, nd, "ay_dm"),
            _dev(azd, F, nd, "az_dm")))

    def integrate(self, n, dt, x64, v64, u64, a_grav, a_hydro, dudt, x, v, u):
        import torch
        F, D, n = self.dtype, torch.float64, int(n)
        check(self.lib.crk_integrate(
            self.handle, n, float(dt), _dev(x64, D, 3 * n, "x64"),
            _dev(v64, D, 3 * n, "v64"), _dev(u64, D, n, "u64"),
            self._p3(a_grav, n, "a_grav"), self._p3(a_hydro, n, "a_hydro"),
            _dev(dudt, F, n, "dudt"), self._p3(x, n, "x"), self._p3(v, n, "v"),
            _dev(u, F, n, "u")))

    # hierarchical time steps ------------------------------------------------
    def timestep_bins(self, n, dt, max_level, eps, c_cfl, eta, a_grav,
                      a_hydro, h, cs, bins):
        import torch
        F, n = self.dtype, int(n)
        check(self.lib.crk_timestep_bins(
            self.handle, n, float(dt), int(max_level), float(eps),
            float(c_cfl), float(eta), self._p3(a_grav, n, "a_grav"),
            self._p3(a_hydro, n, "a_hydro"), _dev(h, F, n, "h"),
            _dev(cs, F, n, "cs"), _dev(bins, torch.int32, n, "bins")))

    def tree_set_active(self, tree, bins_gas, bins_dm, max_level, substep):
        import torch
        I = torch.int32
        check(self.lib.crk_tree_set_active(
            self.handle, tree.handle, _dev(bins_gas, I, tree.n_gas, "bins_gas"),
            _dev(bins_dm, I, tree.n_dm, "bins_dm"), int(max_level),
            int(substep)))

    def tree_refit(self, tree, gx, gy, gz, dx, dy, dz):
        F, ng, nd = self.dtype, tree.n_gas, tree.n_dm
        check(self.lib.crk_tree_refit(
            self.handle, tree.handle, _dev(gx, F, ng, "gx"),
            _dev(gy, F, ng, "gy"), _dev(gz, F, ng, "gz"),
            _dev(dx, F, nd, "dx"), _dev(dy, F, nd, "dy"),
            _dev(dz, F, nd, "dz")))

    def kick(self, n, dt, max_level, substep, phase, bins, v64, u64, a_grav,
             a_hydro, dudt, v, u):
        import torch
        F, D, n = self.dtype, torch.float64, int(n)
        check(self.lib.crk_kick(
            self.handle, n, float(dt), int(max_level), int(substep),
            int(phase), _dev(bins, torch.int32, n, "bins"),
            _dev(v64, D, 3 * n, "v64"), _dev(u64, D, n, "u64"),
            self._p3(a_grav, n, "a_grav"), self._p3(a_hydro, n, "a_hydro"),
            _dev(dudt, F, n, "dudt"), self._p3(v, n, "v"), _dev(u, F, n, "u")))

    def drift(self, n, delta, wrap, x64, v64, x):
        import torch
        D, n = torch.float64, int(n)
        check(self.lib.crk_drift(self.handle, n, float(delta),
                                 int(bool(wrap)), _dev(x64, D, 3 * n, "x64"),
                                 _dev(v64, D, 3 * n, "v64"),
                                 self._p3(x, n, "x")))

    def pm_gravity(self, n_mesh, r_c, n_gas, gx, gy, gz, m_gas, n_dm, dx, dy,
                   dz, m_dm, a_gas, a_dm):
        F, ng, nd = self.dtype, int(n_gas), int(n_dm)
        check(self.lib.crk_pm_gravity(
            self.handle, int(n_mesh), float(r_c), ng, _dev(gx, F, ng, "gx"),
            _dev(gy, F, ng, "gy"), _dev(gz, F, ng, "gz"),
            _dev(m_gas, F, ng, "m_gas"), nd, _dev(dx, F, nd, "dx"),
            _dev(dy, F, nd, "dy"), _dev(dz, F, nd, "dz"),
            _dev(m_dm, F, nd, "m_dm"), self._p3(a_gas, ng, "a_gas"),
            self._p3(a_dm, nd, "a_dm")))

    def fof(self, tree, b, labels_gas, labels_dm):
        import torch
        I = torch.int32
        check(self.lib.crk_fof(self.handle, tree.handle, float(b),
                               _dev(labels_gas, I, tree.n_gas, "labels_gas"),
                               _dev(labels_dm, I, tree.n_dm, "labels_dm")))

    def fof_properties(self, n_gas, n_dm, labels_gas, labels_dm, gas_x, m_gas,
                       dm_x, m_dm, count, mass, centre):
        import torch
        F, I, D = self.dtype, torch.int32, torch.float64
        ng, nd = int(n_gas), int(n_dm)
        n = ng + nd
        check(self.lib.crk_fof_properties(
            self.handle, ng, nd, _dev(labels_gas, I, ng, "labels_gas"),
            _dev(labels_dm, I, nd, "labels_dm"), self._p3(gas_x, ng, "gas_x"),
            _dev(m_gas, F, ng, "m_gas"), self._p3(dm_x, nd, "dm_x"),
            _dev(m_dm, F, nd, "m_dm"), _dev(count, I, n, "count"),
            _dev(mass, D, n, "mass"), _dev(centre, D, 3 * n, "centre")))

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

    def graph_reset(self):
        check(self.lib.crk_graph_reset(self.handle))

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
        self.n_gas = self.n_dm = 0  # set by Context.build_tree
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
