"""Hierarchical kick-drift-kick integration with individual time steps
(Sec. 3.2, Figure KDK) on the device, over the 28-byte particle store of
Sec. 3.4.

The schedule is host logic; every per-particle step runs in the library's
kernels: drifts on the integer grid (mgrav_store_drift), half kicks
(mgrav_store_kick), the time-step criterion (mgrav_store_rungs), the
active mask (mgrav_store_active), and each force computation as tree build,
checklist walk and PP + PC (+ Ewald) evaluation of the active particles,
reading positions from the store (pos_q).  A substep whose active particles
are fewer than ``dual_below`` of all builds the fixed tree of the inactive
particles and the very active tree of the active ones (Sec. 3.2) and walks
both for the active sinks only.

Base step of 2^R substeps of tau = dt_base / 2^R: half kick of every
particle with its last force; then per substep: drift all by tau, force on
the particles whose step ends at the new boundary (rung >= R - trailing
zeros of k), half kick of those, new rung from dt_i = eta sqrt(eps/|a_i|)
(no shallower than the boundary allows), and, except at the end of the
base step, the opening half kick of their next step.

With ``dual_mode="fixed"`` (periodic boxes) the fixed tree of Sec. 3.2 is
kept: where an interval of a fixed rung opens (the shallowest rung r,
at most R - 1, whose particles and the deeper ones are fewer than
``dual_below`` of all, at a step boundary of rung r - 1), the particles on
rungs below r drift half the interval at once, their tree is built once
and kept, and each substep inside the interval drifts only the very
active particles and rebuilds only their tree behind the kept one; at
the interval's end the fixed particles drift the other half and the
force is the usual single-tree one.
"""
from __future__ import annotations

import time
from typing import Optional


def boundary_rung(k: int, rung_max: int) -> int:
    """Shallowest rung whose step boundary is substep boundary k."""
    if k == 0 or k == (1 << rung_max):
        return 0
    tz = (k & -k).bit_length() - 1
    return rung_max - min(tz, rung_max)


class Integrator:
    def __init__(self, ctx, pos_dev, vel_dev, mass: float, eps: float, theta: float,
                 box_L: float, dt_base: float, rung_max: int, eta: float = 0.2,
                 origin=None, scale: Optional[float] = None, dual_below: float = 0.05,
                 bucket: int = 16, dual_mode: str = "rebuild"):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.n = int(pos_dev.shape[0])
        self.mass = float(mass)
        self.eps, self.theta, self.L = float(eps), float(theta), float(box_L)
        self.dt, self.R, self.eta = float(dt_base), int(rung_max), float(eta)
        self.periodic = self.L > 0
        self.dual_below = float(dual_below)
        self.bucket = bucket
        if dual_mode not in ("rebuild", "fixed"):
            raise ValueError("dual_mode is 'rebuild' or 'fixed'")
        if dual_mode == "fixed" and not self.periodic:
            raise ValueError("dual_mode 'fixed' needs a periodic box")
        self.dual_mode = dual_mode
        if self.periodic:
            origin, scale = (0.0, 0.0, 0.0), self.L / 4294967296.0
        self.dev = pos_dev.device
        self.store = ctx.store_alloc(self.n, origin, scale)
        ctx.store_encode(self.store, pos_dev.to(torch.float64), vel_dev.to(torch.float32),
                         self.periodic)
        self.ids = torch.arange(self.n, dtype=torch.int64, device=self.dev)
        self.acc = torch.zeros(3 * self.n, dtype=torch.float32, device=self.dev)
        self.pot = torch.zeros(self.n, dtype=torch.float32, device=self.dev)
        self.mass_dev = torch.full((self.n,), self.mass, dtype=torch.float64, device=self.dev)
        self.log = []  # (boundary, rung_lo, active, dual tree) per substep
        self.kept = []  # boundaries whose force used the kept fixed tree
        self.seconds = []  # wall time per substep (every call blocks)

    # ---- one force computation -------------------------------------------------
    def _reorder(self, perm):
        """Store, forces and ids into the order of a new tree."""
        self.store = self.ctx.store_permute(self.store, perm)
        a = self.acc.view(3, self.n)
        self.acc = a.index_select(1, perm).contiguous().view(-1)
        self.pot = self.pot.index_select(0, perm)
        self.ids = self.ids.index_select(0, perm)

    def forces(self, rung_lo: int):
        """Force on the particles with rung >= rung_lo (all at 0)."""
        ctx = self.ctx
        act = ctx.store_active(self.store, rung_lo)
        n_act = int(act.sum().item())
        if n_act == 0:
            return 0, False
        dual = 0 < n_act < self.dual_below * self.n
        pos = ctx.store_decode(self.store)
        tree = ctx.tree_build(pos, self.mass_dev, self.L, self.bucket,
                              group_dev=act if dual else None)
        del pos
        self._evaluate(tree, dual, rung_lo, n_act)
        return n_act, dual

    def _evaluate(self, tree, second: bool, rung_lo: int, n_act: int):
        """Reorder into the tree's order, walk (the second tree's buckets
        only for a forest), and compute the force on rungs >= rung_lo."""
        ctx = self.ctx
        self._reorder(tree.perm)
        lists = ctx.lists_build(tree, self.theta, self.eps, sinks="second" if second else "all")
        keep, p = ctx.problem_device(tree, lists, self.eps, self.theta)
        # positions from the store's integer grid, equal masses
        p.pos = None
        p.pos_q = self.store.q.data_ptr()
        for k in range(3):
            p.q_origin[k] = self.store.origin[k]
        p.q_scale = self.store.scale
        p.mass = None
        p.mass_uniform = self.mass
        keep["q"] = self.store.q
        ctx.bind(p, keep)
        mask = ctx.store_active(self.store, rung_lo) if n_act < self.n else None
        ctx.set_active(mask)
        ctx.compute(self.acc, self.pot)
        ctx.wait(300.0)
        ctx.set_active(None)

    # ---- the fixed tree of Sec. 3.2 ---------------------------------------------
    def _fixed_rung(self, k: int):
        """The fixed rung of an interval opening at boundary k, or None."""
        if self.dual_mode != "fixed":
            return None
        counts = self.torch.bincount(self.store.rung.to(self.torch.int64),
                                     minlength=self.R + 1).cpu().tolist()
        for r in range(1, self.R):
            if k % (1 << (self.R - r + 1)):
                continue
            m = sum(counts[r:])
            if 0 < m < self.dual_below * self.n:
                return r
        return None

    def _keep_fixed(self, r: int):
        """The fixed tree of the particles on rungs below r, built once; the
        store, forces and ids reordered to put them first in its order."""
        torch, ctx = self.torch, self.ctx
        very = (self.store.rung >= r).to(torch.uint8)
        pos = ctx.store_decode(self.store)
        kf = ctx.forest_keep(pos, self.mass_dev, self.L, very, self.bucket)
        del pos
        n0 = kf.n_first
        self._reorder(torch.cat([kf.arrays["perm"][:n0], kf.ids_second]))
        # the store is now in the kept order: relabel the kept tree to it
        kf.arrays["perm"][:n0] = torch.arange(n0, dtype=torch.int64, device=self.dev)
        kf.ids_second = torch.arange(n0, self.n, dtype=torch.int64, device=self.dev)
        return kf

    def _forces_kept(self, kf, rung_lo: int):
        """Force on rungs >= rung_lo (all very active) with the kept fixed
        tree and the very active tree rebuilt behind it."""
        ctx = self.ctx
        n_act = int(ctx.store_active(self.store, rung_lo).sum().item())
        if n_act == 0:
            return 0
        pos = ctx.store_decode(self.store)
        tree = ctx.forest_rebuild(kf, pos, self.mass_dev)
        del pos
        self._evaluate(tree, True, rung_lo, n_act)
        return n_act

    # ---- the integrator --------------------------------------------------------
    def start(self):
        """Force on every particle and the first rungs."""
        self.forces(0)
        self.ctx.store_rungs(self.store, self.acc, self.eps, self.eta, self.dt, 0, 0, self.R)

    def _close(self, k1: int, lo: int, n_act: int):
        """Half kick, new rungs and the next half kick of the active ones."""
        ctx = self.ctx
        if n_act > 0:
            ctx.store_kick(self.store, self.acc, self.dt, lo)
            ctx.store_rungs(self.store, self.acc, self.eps, self.eta, self.dt, lo, lo, self.R)
            if k1 < (1 << self.R):
                ctx.store_kick(self.store, self.acc, self.dt, lo)

    def base_step(self):
        ctx = self.ctx
        nsub = 1 << self.R
        tau = self.dt / nsub
        ctx.store_kick(self.store, self.acc, self.dt, 0)
        k = 0
        while k < nsub:
            r = self._fixed_rung(k)
            if r is None:
                t0 = time.perf_counter()
                ctx.store_drift(self.store, tau, self.periodic)
                k1 = k + 1
                lo = boundary_rung(k1, self.R)
                n_act, dual = self.forces(lo)
                self._close(k1, lo, n_act)
                self.log.append((k1, lo, n_act, dual))
                self.seconds.append(time.perf_counter() - t0)
                k = k1
                continue
            # an interval of the fixed rung r - 1: fixed particles at its midpoint
            span = 1 << (self.R - r + 1)
            half = 0.5 * span * tau
            t0 = time.perf_counter()
            ctx.store_drift_rungs(self.store, half, self.periodic, 0, r)
            kf = self._keep_fixed(r)
            for j in range(1, span + 1):
                ctx.store_drift_rungs(self.store, tau, self.periodic, r, 256)
                k1 = k + j
                lo = boundary_rung(k1, self.R)
                if j < span:
                    n_act = self._forces_kept(kf, lo)
                    second = True
                    self.kept.append(k1)
                else:
                    del kf
                    ctx.store_drift_rungs(self.store, half, self.periodic, 0, r)
                    n_act, second = self.forces(lo)
                self._close(k1, lo, n_act)
                self.log.append((k1, lo, n_act, second))
                self.seconds.append(time.perf_counter() - t0)
                t0 = time.perf_counter()
            k += span

    # ---- state in input order ------------------------------------------------------
    def state(self):
        """Positions (double), velocities, rungs, accelerations and
        potentials in the order of the particles given to the constructor."""
        torch = self.torch
        pos, vel = self.ctx.store_decode(self.store, with_vel=True)
        inv = torch.empty_like(self.ids)
        inv[self.ids] = torch.arange(self.n, dtype=torch.int64, device=self.dev)
        rung = (self.store.aux & 0xff).index_select(0, inv)
        acc = self.acc.view(3, self.n).index_select(1, inv).t()
        return (pos.index_select(0, inv), vel.index_select(0, inv), rung, acc,
                self.pot.index_select(0, inv))

    def energies(self):
        pos, vel, rung, acc, pot = self.state()
        v = vel.double()
        ke = 0.5 * self.mass * float((v * v).sum().item())
        pe = 0.5 * self.mass * float(pot.double().sum().item())
        return ke, pe
