"""One short-range step on the GPU for a workload: device buffers (torch
tensors), the call sequence of the C ABI, and optional HIP-graph capture.

Argument marshalling only; all arithmetic runs in libcrk.so.
"""
from __future__ import annotations

import numpy as np

from .binding import Context, Tree

OUTPUTS_GAS = ("V", "rho_tilde", "A", "B", "gradA", "gradB", "rho", "P", "cs",
               "a_hydro", "dudt", "a_grav_gas")


class ShortRangeStep:
    """Device-resident inputs, outputs and double-precision state of one
    workload.  ``run()`` enqueues build_tree, build_interaction_lists and the
    four passes (and crk_integrate when ``integrate`` is set) on the
    context's stream.  With ``recon`` the hydro forces take the velocity
    gradient and the viscosity on the limited midpoint reconstruction
    (crk_velocity_gradient, then crk_hydro_forces_limited).  With
    ``compatible`` the integration's energy update takes the compatible rate
    (crk_hydro_energy_compatible before crk_integrate; in substep_cycle,
    crk_hydro_energy_compatible_block at every kick)."""

    def __init__(self, wl, precision: str = "fp32", tuning: dict | None = None,
                 dt: float = 0.0, device: str = "cuda", params=None,
                 recon: bool = False, eta_crit: float = 0.8,
                 eta_fold: float = 0.2, compatible: bool = False):
        import torch
        self.torch = torch
        self.wl = wl
        self.dt = float(dt)
        self.recon = bool(recon)
        self.compatible = bool(compatible)
        self.eta_crit, self.eta_fold = float(eta_crit), float(eta_fold)
        self.ctx = Context(precision, params=params)
        if tuning:
            self.ctx.set_tuning(**tuning)
        self.tree = Tree(self.ctx)
        T = self.ctx.dtype
        npT = np.float32 if precision == "fp32" else np.float64
        g, d = wl.gas, wl.dm
        self.ng, self.nd = g.n, d.n
        ng, nd = self.ng, self.nd
        # per-box h bound (host): the largest h of each box
        hm = []
        for b in range(wl.n_boxes):
            s = slice(int(wl.gas_off[b]), int(wl.gas_off[b + 1]))
            hm.append(float(np.max(g.h[s])) if s.stop > s.start else 1e-3)
        self.h_max = np.array(hm, np.float64)

        def up(a, dtype=None):
            a = np.ascontiguousarray(a, dtype or npT)
            return torch.from_numpy(a).to(device, non_blocking=False)

        def zeros(n, dtype=T):
            return torch.zeros(max(n, 1), dtype=dtype, device=device)

        with torch.cuda.stream(self.ctx.stream):
            self.gx, self.gy, self.gz = up(g.x), up(g.y), up(g.z)
            self.gh, self.gm, self.gu = up(g.h), up(g.m), up(g.u)
            self.gvx, self.gvy, self.gvz = up(g.vx), up(g.vy), up(g.vz)
            self.dx, self.dy, self.dz = up(d.x), up(d.y), up(d.z)
            self.dm = up(d.m)
            self.dvx, self.dvy, self.dvz = up(d.vx), up(d.vy), up(d.vz)
            f64 = np.float64
            self.gx64 = up(np.concatenate([g.x, g.y, g.z]), f64)
            self.gv64 = up(np.concatenate([g.vx, g.vy, g.vz]), f64)
            self.gu64 = up(g.u, f64)
            self.dx64 = up(np.concatenate([d.x, d.y, d.z]), f64)
            self.dv64 = up(np.concatenate([d.vx, d.vy, d.vz]), f64)
            self.V, self.rho_t = zeros(ng), zeros(ng)
            self.A, self.rho, self.P, self.cs = (zeros(ng) for _ in range(4))
            self.B, self.gA, self.gB = zeros(3 * ng), zeros(3 * ng), zeros(9 * ng)
            self.dv = zeros(9 * ng)
            self.ahx, self.ahy, self.ahz, self.dudt = (zeros(ng) for _ in range(4))
            self.agx, self.agy, self.agz = (zeros(ng) for _ in range(3))
            self.adx, self.ady, self.adz = (zeros(nd) for _ in range(3))
        self.ctx.stream.synchronize()
        self.graph = False

    # --------------------------------------------------------------------
    def run(self, integrate: bool = False, passes=("density", "coefficients",
                                                    "hydro", "gravity")):
        c, t, wl = self.ctx, self.tree, self.wl
        if wl.n_total == 0:
            return  # the library rejects an empty tree; outputs stay empty
        c.build_tree(t, wl.gas_off, wl.dm_off, wl.r_c, wl.eps, self.h_max,
                     self.gx, self.gy, self.gz, self.gh, self.dx, self.dy,
                     self.dz)
        c.build_interaction_lists(t)
        if "density" in passes:
            c.density(t, self.gm, self.V, self.rho_t)
        if "coefficients" in passes:
            c.coefficients(t, self.gm, self.V, self.gu, self.A, self.B,
                           self.gA, self.gB, self.rho, self.P, self.cs)
        if "hydro" in passes:
            self._hydro()
        if "gravity" in passes:
            c.shortrange_gravity(t, self.gm, self.dm, self.agx, self.agy,
                                 self.agz, self.adx, self.ady, self.adz)
        if integrate:
            self.integrate()

    def integrate(self):
        c = self.ctx
        if self.ng and self.compatible:
            c.hydro_energy_compatible(
                self.tree, self.gm, self.gvx, self.gvy, self.gvz, self.V,
                self.rho, self.P, self.cs, self.A, self.B, self.gA, self.gB,
                self.dv if self.recon else None, self.eta_crit, self.eta_fold,
                self.dt, (self.agx, self.agy, self.agz),
                (self.ahx, self.ahy, self.ahz), self.dudt)
        if self.ng:
            c.integrate(self.ng, self.dt, self.gx64, self.gv64, self.gu64,
                        (self.agx, self.agy, self.agz),
                        (self.ahx, self.ahy, self.ahz), self.dudt,
                        (self.gx, self.gy, self.gz),
                        (self.gvx, self.gvy, self.gvz), self.gu)
        if self.nd:
            c.integrate(self.nd, self.dt, self.dx64, self.dv64, None,
                        (self.adx, self.ady, self.adz), None, None,
                        (self.dx, self.dy, self.dz),
                        (self.dvx, self.dvy, self.dvz), None)

    # --------------------------------------------------------------------
    def _passes(self):
        c, t = self.ctx, self.tree
        c.build_interaction_lists(t)
        if self.ng:
            c.density(t, self.gm, self.V, self.rho_t)
            c.coefficients(t, self.gm, self.V, self.gu, self.A, self.B,
                           self.gA, self.gB, self.rho, self.P, self.cs)
            self._hydro()
        c.shortrange_gravity(t, self.gm, self.dm, self.agx, self.agy,
                             self.agz, self.adx, self.ady, self.adz)

    def _hydro(self):
        c, t = self.ctx, self.tree
        if not self.recon:
            c.hydro_forces(t, self.gm, self.gvx, self.gvy, self.gvz, self.V,
                           self.rho, self.P, self.cs, self.A, self.B, self.gA,
                           self.gB, self.ahx, self.ahy, self.ahz, self.dudt)
            return
        c.velocity_gradient(t, self.gvx, self.gvy, self.gvz, self.V, self.A,
                            self.B, self.gA, self.gB, self.dv)
        c.hydro_forces_limited(t, self.gm, self.gvx, self.gvy, self.gvz,
                               self.V, self.rho, self.P, self.cs, self.A,
                               self.B, self.gA, self.gB, self.dv,
                               self.eta_crit, self.eta_fold, self.ahx,
                               self.ahy, self.ahz, self.dudt)

    def _kick(self, dt, L, s, phase):
        c = self.ctx
        if self.ng:
            c.kick(self.ng, dt, L, s, phase, self.bins_g, self.gv64,
                   self.gu64, (self.agx, self.agy, self.agz),
                   (self.ahx, self.ahy, self.ahz), self.dudt,
                   (self.gvx, self.gvy, self.gvz), self.gu)
        if self.nd:
            c.kick(self.nd, dt, L, s, phase, self.bins_d, self.dv64, None,
                   (self.adx, self.ady, self.adz), None, None,
                   (self.dvx, self.dvy, self.dvz), None)

    def _drift(self, delta, wrap):
        c = self.ctx
        if self.ng:
            c.drift(self.ng, delta, wrap, self.gx64, self.gv64,
                    (self.gx, self.gy, self.gz))
        if self.nd:
            c.drift(self.nd, delta, wrap, self.dx64, self.dv64,
                    (self.dx, self.dy, self.dz))

    def set_bins(self, bins_gas, bins_dm):
        """Timestep bins (numpy int, caller order) for substep_cycle."""
        torch = self.torch
        with torch.cuda.stream(self.ctx.stream):
            self.bins_g = torch.from_numpy(np.ascontiguousarray(
                bins_gas, np.int32).reshape(-1)).to("cuda") if self.ng else None
            self.bins_d = torch.from_numpy(np.ascontiguousarray(
                bins_dm, np.int32).reshape(-1)).to("cuda") if self.nd else None
        self.ctx.stream.synchronize()

    def timestep_bins(self, dt, max_level, c_cfl=0.25, eta=0.025):
        """Bins from the current accelerations (crk_timestep_bins), per
        box with that box's softening; kept for substep_cycle and returned
        as numpy arrays (gas, dm)."""
        torch, c, wl = self.torch, self.ctx, self.wl
        with torch.cuda.stream(c.stream):
            bg = torch.zeros(max(self.ng, 1), dtype=torch.int32, device="cuda")
            bd = torch.zeros(max(self.nd, 1), dtype=torch.int32, device="cuda")
        for b in range(wl.n_boxes):
            g0, g1 = int(wl.gas_off[b]), int(wl.gas_off[b + 1])
            d0, d1 = int(wl.dm_off[b]), int(wl.dm_off[b + 1])
            eps = float(wl.eps[b])
            if g1 > g0:
                sl = slice(g0, g1)
                c.timestep_bins(g1 - g0, dt, max_level, eps, c_cfl, eta,
                                (self.agx[sl], self.agy[sl], self.agz[sl]),
                                (self.ahx[sl], self.ahy[sl], self.ahz[sl]),
                                self.gh[sl], self.cs[sl], bg[sl])
            if d1 > d0:
                sl = slice(d0, d1)
                c.timestep_bins(d1 - d0, dt, max_level, eps, c_cfl, eta,
                                (self.adx[sl], self.ady[sl], self.adz[sl]),
                                None, None, None, bd[sl])
        self.bins_g = bg if self.ng else None
        self.bins_d = bd if self.nd else None
        c.stream.synchronize()
        return (bg[:self.ng].cpu().numpy(), bd[:self.nd].cpu().numpy())

    def _long_kick(self, dt, n_mesh):
        """v += a_long dt / 2 for every particle (crk_pm_gravity, then
        crk_kick with one level: every particle selected, tau = dt)."""
        torch, c = self.torch, self.ctx
        self.pm_gravity(n_mesh)
        if getattr(self, "_zero_bins", None) is None:
            with torch.cuda.stream(c.stream):
                self._zero_bins = torch.zeros(max(self.ng, self.nd, 1),
                                              dtype=torch.int32, device="cuda")
        if self.ng:
            c.kick(self.ng, dt, 0, 0, 0, self._zero_bins, self.gv64, None,
                   self.pm_gas, None, None, (self.gvx, self.gvy, self.gvz), None)
        if self.nd:
            c.kick(self.nd, dt, 0, 0, 0, self._zero_bins, self.dv64, None,
                   self.pm_dm, None, None, (self.dvx, self.dvy, self.dvz), None)

    def substep_cycle(self, dt, max_level, pm_mesh: int | None = None):
        """One interval dt of hierarchical block steps with 2^max_level
        substeps on one tree (built here at the start): every particle is
        evaluated first; each substep kicks the particles starting a step,
        drifts all, refits the leaf boxes, rebuilds the lists, evaluates the
        particles ending a step (active leaves only) and kicks them; the
        positions are wrapped at the end.  Bins come from set_bins or
        timestep_bins.  With pm_mesh (single box), the long-range mesh
        force brackets the interval: a half-kick of every particle before
        the first substep and after the last one (positions wrapped).
        With ``compatible`` every gas kick takes the compatible energy rate
        (crk_hydro_energy_compatible_block): once for the opening half-kick
        of the interval and once after each evaluation, for the closing
        half-kick and the next opening one together.  ``cycle_subsets``
        keeps, per substep, the active leaves and particles and whether the
        sweeps took active groups."""
        c, t, wl = self.ctx, self.tree, self.wl
        self.cycle_subsets = []
        L = int(max_level)
        if pm_mesh:
            self._long_kick(dt, pm_mesh)
        c.build_tree(t, wl.gas_off, wl.dm_off, wl.r_c, wl.eps, self.h_max,
                     self.gx, self.gy, self.gz, self.gh, self.dx, self.dy,
                     self.dz)
        self._passes()
        self._compatible_block(dt, L, -1)
        delta = dt / 2 ** L
        for s in range(2 ** L):
            self._kick(dt, L, s, 0)
            self._drift(delta, False)
            c.tree_refit(t, self.gx, self.gy, self.gz, self.dx, self.dy,
                         self.dz)
            c.tree_set_active(t, self.bins_g, self.bins_d, L, s)
            i = t.info()
            self.cycle_subsets.append((i["act_leaves"], i["act_particles"],
                                       i["act_grouped"]))
            self._passes()
            self._compatible_block(dt, L, s)
            self._kick(dt, L, s, 1)
        c.tree_set_active(t, None, None, 0, -1)
        self._drift(0.0, True)
        if pm_mesh:
            self._long_kick(dt, pm_mesh)

    def _compatible_block(self, dt, L, s):
        if not (self.compatible and self.ng):
            return
        self.ctx.hydro_energy_compatible_block(
            self.tree, self.gm, self.gvx, self.gvy, self.gvz, self.V,
            self.rho, self.P, self.cs, self.A, self.B, self.gA, self.gB,
            self.dv if self.recon else None, self.eta_crit, self.eta_fold,
            dt, L, self.bins_g, s, (self.agx, self.agy, self.agz),
            (self.ahx, self.ahy, self.ahz), self.dudt)

    _STATE = ("gx64", "gv64", "gu64", "dx64", "dv64", "gx", "gy", "gz",
              "gvx", "gvy", "gvz", "gu", "dx", "dy", "dz", "dvx", "dvy", "dvz")

    def snapshot(self) -> dict:
        """Device copies of the state a cycle or an integration changes
        (positions, velocities, energies and their working copies)."""
        with self.torch.cuda.stream(self.ctx.stream):
            snap = {k: getattr(self, k).clone() for k in self._STATE}
        self.ctx.stream.synchronize()
        return snap

    def restore(self, snap: dict):
        """Puts back a snapshot's state (device to device)."""
        with self.torch.cuda.stream(self.ctx.stream):
            for k, t in snap.items():
                getattr(self, k).copy_(t)
        self.ctx.stream.synchronize()

    def state(self) -> dict:
        """The double-precision state (numpy, (3, n) / n)."""
        self.ctx.sync()
        ng, nd = self.ng, self.nd

        def h3(t, n):
            return t[:3 * n].cpu().numpy().reshape(3, n) if n else np.zeros((3, 0))

        return dict(xg=h3(self.gx64, ng), vg=h3(self.gv64, ng),
                    u=self.gu64[:ng].cpu().numpy() if ng else np.zeros(0),
                    xd=h3(self.dx64, nd), vd=h3(self.dv64, nd))

    def pm_gravity(self, n_mesh: int | None = None):
        """Long-range accelerations of a single-box workload on an n_mesh^3
        mesh (default: r_c = 6 mesh cells), into self.pm_gas / self.pm_dm
        (3 tensors each); returns them as numpy (3, n) arrays."""
        wl, c, torch = self.wl, self.ctx, self.torch
        if wl.n_boxes != 1:
            raise ValueError("the mesh solver takes one periodic box")
        rc = float(wl.r_c[0])
        if n_mesh is None:
            n_mesh = int(2 * np.ceil(3.0 / rc))
        T = c.dtype
        if getattr(self, "pm_gas", None) is None:
            with torch.cuda.stream(c.stream):
                self.pm_gas = [torch.zeros(max(self.ng, 1), dtype=T,
                                           device="cuda") for _ in range(3)]
                self.pm_dm = [torch.zeros(max(self.nd, 1), dtype=T,
                                          device="cuda") for _ in range(3)]
        c.pm_gravity(n_mesh, rc, self.ng, self.gx, self.gy, self.gz, self.gm,
                     self.nd, self.dx, self.dy, self.dz, self.dm,
                     self.pm_gas if self.ng else None,
                     self.pm_dm if self.nd else None)
        c.stream.synchronize()
        g = np.stack([t[:self.ng].double().cpu().numpy() for t in self.pm_gas])
        d = np.stack([t[:self.nd].double().cpu().numpy() for t in self.pm_dm])
        return g, d

    def fof(self, b: float):
        """Friends-of-friends labels (gas, dm) with linking length b over the
        current tree and lists (crk_fof); numpy int arrays, the smallest
        combined caller index of each group."""
        torch, c = self.torch, self.ctx
        with torch.cuda.stream(c.stream):
            lg = torch.zeros(max(self.ng, 1), dtype=torch.int32, device="cuda")
            ld = torch.zeros(max(self.nd, 1), dtype=torch.int32, device="cuda")
        c.fof(self.tree, b, lg if self.ng else None, ld if self.nd else None)
        c.stream.synchronize()
        return lg[:self.ng].cpu().numpy(), ld[:self.nd].cpu().numpy()

    def fof_properties(self, b: float):
        """Friends-of-friends groups with linking length b and their
        properties (crk_fof, then crk_fof_properties): labels (gas, dm) and,
        per combined index, member count, mass and periodic centre of mass
        (numpy; zero at indices that label no group)."""
        torch, c = self.torch, self.ctx
        n = self.ng + self.nd
        with torch.cuda.stream(c.stream):
            lg = torch.zeros(max(self.ng, 1), dtype=torch.int32, device="cuda")
            ld = torch.zeros(max(self.nd, 1), dtype=torch.int32, device="cuda")
            cnt = torch.zeros(max(n, 1), dtype=torch.int32, device="cuda")
            mass = torch.zeros(max(n, 1), dtype=torch.float64, device="cuda")
            cen = torch.zeros(3 * max(n, 1), dtype=torch.float64, device="cuda")
        c.fof(self.tree, b, lg if self.ng else None, ld if self.nd else None)
        c.fof_properties(self.ng, self.nd, lg if self.ng else None,
                         ld if self.nd else None,
                         (self.gx, self.gy, self.gz) if self.ng else None,
                         self.gm if self.ng else None,
                         (self.dx, self.dy, self.dz) if self.nd else None,
                         self.dm if self.nd else None, cnt, mass, cen)
        c.stream.synchronize()
        return (lg[:self.ng].cpu().numpy(), ld[:self.nd].cpu().numpy(),
                cnt[:n].cpu().numpy(), mass[:n].cpu().numpy(),
                cen[:3 * n].cpu().numpy().reshape(3, n))

    def capture(self, integrate: bool = True):
        """Runs the step once eagerly (sizes), then captures it in a graph."""
        self.run(integrate=integrate)
        self.ctx.sync()
        self.ctx.graph_begin()
        try:
            self.run(integrate=integrate)
        finally:
            self.ctx.graph_end()
        self.graph = True

    def replay(self):
        if not self.graph:
            raise RuntimeError("no step captured: call capture() first")
        self.ctx.graph_launch()

    def drop_graph(self):
        """Forgets the captured step (a later replay() raises)."""
        self.ctx.graph_reset()
        self.graph = False

    def sync(self):
        return self.ctx.sync()

    # --------------------------------------------------------------------
    def set_inputs(self, **fields):
        """Overwrites device inputs (numpy, caller order), e.g. V=..."""
        T = self.ctx.dtype
        for k, v in fields.items():
            dst = getattr(self, k)
            src = self.torch.from_numpy(np.ascontiguousarray(
                v, np.float32 if T == self.torch.float32 else np.float64))
            with self.torch.cuda.stream(self.ctx.stream):
                dst.copy_(src.reshape(dst.shape).to(dst.device))
        self.ctx.stream.synchronize()

    def outputs(self) -> dict:
        self.ctx.sync()
        ng, nd = self.ng, self.nd

        def h(t, n):
            return t[:n].double().cpu().numpy() if n else np.zeros(0)

        out = dict(V=h(self.V, ng), rho_tilde=h(self.rho_t, ng), A=h(self.A, ng),
                   rho=h(self.rho, ng), P=h(self.P, ng), cs=h(self.cs, ng),
                   dudt=h(self.dudt, ng))
        out["B"] = h(self.B, 3 * ng).reshape(3, ng).T
        out["gradA"] = h(self.gA, 3 * ng).reshape(3, ng).T
        out["gradB"] = h(self.gB, 9 * ng).reshape(3, 3, ng).transpose(2, 0, 1)
        out["dv"] = h(self.dv, 9 * ng).reshape(3, 3, ng).transpose(2, 0, 1)
        out["a_hydro"] = np.stack([h(self.ahx, ng), h(self.ahy, ng),
                                   h(self.ahz, ng)])
        out["a_grav_gas"] = np.stack([h(self.agx, ng), h(self.agy, ng),
                                      h(self.agz, ng)])
        out["a_grav_dm"] = np.stack([h(self.adx, nd), h(self.ady, nd),
                                     h(self.adz, nd)])
        return out

    def outputs_at(self, gas_idx, dm_idx) -> dict:
        """outputs() at the listed gas and dm indices only (gathered on the
        device: at 180 M particles the full outputs would not fit a host
        copy comfortably).  Same layout as outputs(), n = len(indices)."""
        self.ctx.sync()
        torch = self.torch
        dev = self.V.device
        gi = torch.as_tensor(np.asarray(gas_idx, np.int64), device=dev)
        di = torch.as_tensor(np.asarray(dm_idx, np.int64), device=dev)
        ng, nd = self.ng, self.nd
        k = int(gi.numel())

        def h(t, planes, n, idx):
            if idx.numel() == 0:
                return np.zeros((planes, 0))
            v = t[:planes * n].view(planes, n)[:, idx]
            return v.double().cpu().numpy()

        with torch.cuda.stream(self.ctx.stream):
            out = {key: h(getattr(self, a), 1, ng, gi)[0]
                   for key, a in (("V", "V"), ("rho_tilde", "rho_t"), ("A", "A"),
                                  ("rho", "rho"), ("P", "P"), ("cs", "cs"),
                                  ("dudt", "dudt"))}
            out["B"] = h(self.B, 3, ng, gi).T
            out["gradA"] = h(self.gA, 3, ng, gi).T
            out["gradB"] = h(self.gB, 9, ng, gi).reshape(3, 3, k).transpose(2, 0, 1)
            out["dv"] = h(self.dv, 9, ng, gi).reshape(3, 3, k).transpose(2, 0, 1)
            out["a_hydro"] = np.concatenate([h(t, 1, ng, gi) for t in
                                             (self.ahx, self.ahy, self.ahz)])
            out["a_grav_gas"] = np.concatenate([h(t, 1, ng, gi) for t in
                                                (self.agx, self.agy, self.agz)])
            out["a_grav_dm"] = np.concatenate([h(t, 1, nd, di) for t in
                                               (self.adx, self.ady, self.adz)])
        self.ctx.stream.synchronize()
        return out

    def close(self):
        self.tree.free()
        self.ctx.close()
