"""FP64 oracle of the particle store (Sec. 3.4) and of the hierarchical
kick-drift-kick integrator with individual time steps (Sec. 3.2, Figure
KDK).

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.
Plain numpy, one particle array at a time, in the order the paper gives
the steps.  Parity unpinned: none of the functions here (each is pinned by
tests/test_oracle_kdk.py against closed forms, a Kepler orbit,
time-reversal, the order of convergence and the schedule of rungs).

Store (Sec. 3.4): a position is three 32-bit integers on a grid of step
`scale` from `origin` (a periodic box of side L: origin 0, scale L/2^32,
the integers wrapping with the box); velocities are single-precision
floats; the rung is an integer per particle.

Integrator (Sec. 3.2): particle i takes steps dt_base / 2^rung_i; the base
step is cut into 2^R substeps of tau = dt_base / 2^R, and at substep
boundary t_k the particles whose step ends there are those with
2^(R - rung) dividing k, i.e. rung >= R - (trailing zero bits of k) (every
particle at k = 0 and k = 2^R).  A step is: half kick with the force at its
start, drifts of every particle substep by substep, force at its end for
the particles ending a step (the active ones), half kick with that force.
The time-step criterion dt_i = eta sqrt(eps / |a_i|) with eta = 0.2 picks a
particle's rung at the end of each of its steps: the smallest l with
dt_base / 2^l <= dt_i, no shallower than the shallowest rung whose step
boundary is now, no deeper than R.
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np

TWO32 = 4294967296.0


def quantize(pos: np.ndarray, origin, scale: float, periodic: bool) -> np.ndarray:
    """Nearest grid point (ties to even), modulo 2^32 when periodic.
    Returns int64 values in [0, 2^32)."""
    u = np.rint((np.asarray(pos, np.float64) - np.asarray(origin, np.float64)) / scale)
    if periodic:
        u = u - TWO32 * np.floor(u / TWO32)
    elif np.any(u < 0) or np.any(u > TWO32 - 1):
        raise ValueError("position off the integer grid")
    return u.astype(np.int64)


def decode(q: np.ndarray, origin, scale: float) -> np.ndarray:
    return np.asarray(origin, np.float64) + q.astype(np.float64) * scale


def drift(q: np.ndarray, vel: np.ndarray, dt: float, scale: float, periodic: bool) -> np.ndarray:
    """x += v dt on the grid: q + nearest integer of v dt / scale."""
    u = q.astype(np.float64) + np.rint(vel.astype(np.float64) * dt / scale)
    if periodic:
        u = u - TWO32 * np.floor(u / TWO32)
    elif np.any(u < 0) or np.any(u > TWO32 - 1):
        raise ValueError("drift left the integer grid")
    return u.astype(np.int64)


def half_kick(vel: np.ndarray, acc: np.ndarray, rung: np.ndarray, dt_base: float,
              sel: np.ndarray) -> np.ndarray:
    """v += a dt_rung / 2 for the selected particles (stored as float)."""
    out = vel.copy()
    h = 0.5 * dt_base / np.power(2.0, rung[sel])
    out[sel] = (vel[sel].astype(np.float64) + acc[sel] * h[:, None]).astype(np.float32)
    return out


def rung_of(acc_mag: np.ndarray, eps: float, eta: float, dt_base: float, rung_floor: int,
            rung_max: int) -> np.ndarray:
    """Smallest l with dt_base / 2^l <= eta sqrt(eps / |a|), within
    [rung_floor, rung_max] (|a| = 0: the floor)."""
    out = np.empty(acc_mag.shape[0], np.int64)
    for i, a in enumerate(np.asarray(acc_mag, np.float64)):
        if a > 0:
            dti = eta * np.sqrt(eps / a)
            l = 0
            while l < rung_max and dt_base / 2.0 ** l > dti:
                l += 1
        else:
            l = 0
        out[i] = max(l, rung_floor)
    return out


def boundary_rung(k: int, rung_max: int) -> int:
    """Shallowest rung whose step boundary is substep boundary k."""
    if k == 0 or k == (1 << rung_max):
        return 0
    tz = (k & -k).bit_length() - 1
    return rung_max - min(tz, rung_max)


@dataclasses.dataclass
class State:
    q: np.ndarray        # int64 [n, 3], values of the 32-bit grid
    vel: np.ndarray      # float32 [n, 3]
    rung: np.ndarray     # int64 [n]
    acc: np.ndarray      # float64 [n, 3], the last force of every particle
    pot: np.ndarray      # float64 [n]
    origin: tuple
    scale: float
    periodic: bool


def start(state: State, forces: Callable, eps: float, eta: float, dt_base: float,
          rung_max: int) -> State:
    """Force on every particle and its first rung."""
    pos = decode(state.q, state.origin, state.scale)
    allp = np.ones(state.q.shape[0], bool)
    acc, pot = forces(pos, allp)
    rung = rung_of(np.linalg.norm(acc, axis=1), eps, eta, dt_base, 0, rung_max)
    return dataclasses.replace(state, acc=acc, pot=pot, rung=rung)


def base_step(state: State, forces: Callable, eps: float, eta: float, dt_base: float,
              rung_max: int, log: list | None = None) -> State:
    """One base step.  forces(pos, active) -> (acc, pot) of the active
    particles (rows of inactive ones ignored)."""
    s = dataclasses.replace(state)
    n = s.q.shape[0]
    nsub = 1 << rung_max
    tau = dt_base / nsub
    allp = np.ones(n, bool)
    s.vel = half_kick(s.vel, s.acc, s.rung, dt_base, allp)
    for k in range(nsub):
        s.q = drift(s.q, s.vel, tau, s.scale, s.periodic)
        k1 = k + 1
        lo = boundary_rung(k1, rung_max)
        act = s.rung >= lo
        if log is not None:
            log.append((k1, lo, int(act.sum())))
        acc, pot = forces(decode(s.q, s.origin, s.scale), act)
        s.acc = s.acc.copy()
        s.pot = s.pot.copy()
        s.acc[act] = acc[act]
        s.pot[act] = pot[act]
        s.vel = half_kick(s.vel, s.acc, s.rung, dt_base, act)
        new = rung_of(np.linalg.norm(s.acc[act], axis=1), eps, eta, dt_base, lo, rung_max)
        s.rung = s.rung.copy()
        s.rung[act] = new
        if k1 < nsub:
            s.vel = half_kick(s.vel, s.acc, s.rung, dt_base, act)
    return s


def fixed_rung(rung: np.ndarray, k: int, rung_max: int, dual_below: float):
    """Sec. 3.2's fixed rung for an interval starting at substep boundary k:
    the shallowest r in 1 .. rung_max - 1 such that k is a step boundary of
    rung r - 1 (k a multiple of 2^(rung_max - r + 1)) and the particles on
    rungs >= r (the very active ones) are some, but fewer than dual_below
    of all; None if there is none.  r <= rung_max - 1 keeps at least two
    rungs below the fixed rung r - 1, the condition under which the paper
    builds the second tree.  The interval is one step of rung r - 1."""
    n = rung.shape[0]
    for r in range(1, rung_max):
        if k % (1 << (rung_max - r + 1)):
            continue
        m = int(np.count_nonzero(rung >= r))
        if 0 < m < dual_below * n:
            return r
    return None


def base_step_fixed(state: State, forces: Callable, eps: float, eta: float, dt_base: float,
                    rung_max: int, dual_below: float, log: list | None = None) -> State:
    """One base step with the fixed tree of Sec. 3.2.  Where an interval of
    the fixed rung r - 1 starts (fixed_rung), the particles on rungs below r
    (fixed: none of them is kicked inside the interval) drift half the
    interval at once and stay there, the very active ones drift substep by
    substep, and their forces at the substeps inside the interval are taken
    with the fixed particles at that midpoint: forces(pos, active, group)
    with group the very active particles (the second tree's).  At the
    interval's end the fixed particles drift the other half and the force
    is the usual one, forces(pos, active).  Elsewhere as base_step.  The log
    holds (k, lowest active rung, active count, second tree used)."""
    s = dataclasses.replace(state)
    n = s.q.shape[0]
    nsub = 1 << rung_max
    tau = dt_base / nsub
    allp = np.ones(n, bool)
    s.vel = half_kick(s.vel, s.acc, s.rung, dt_base, allp)

    def drift_sel(sel, dt):
        q = s.q.copy()
        q[sel] = drift(s.q[sel], s.vel[sel], dt, s.scale, s.periodic)
        s.q = q

    def force_step(k1, group):
        lo = boundary_rung(k1, rung_max)
        act = s.rung >= lo
        if log is not None:
            log.append((k1, lo, int(act.sum()), group is not None))
        pos = decode(s.q, s.origin, s.scale)
        acc, pot = forces(pos, act) if group is None else forces(pos, act, group)
        s.acc = s.acc.copy()
        s.pot = s.pot.copy()
        s.acc[act] = acc[act]
        s.pot[act] = pot[act]
        s.vel = half_kick(s.vel, s.acc, s.rung, dt_base, act)
        new = rung_of(np.linalg.norm(s.acc[act], axis=1), eps, eta, dt_base, lo, rung_max)
        s.rung = s.rung.copy()
        s.rung[act] = new
        if k1 < nsub:
            s.vel = half_kick(s.vel, s.acc, s.rung, dt_base, act)

    k = 0
    while k < nsub:
        r = fixed_rung(s.rung, k, rung_max, dual_below)
        if r is None:
            drift_sel(allp, tau)
            force_step(k + 1, None)
            k += 1
            continue
        span = 1 << (rung_max - r + 1)
        fixed = s.rung < r
        very = ~fixed
        half = 0.5 * span * tau
        drift_sel(fixed, half)
        for j in range(1, span + 1):
            drift_sel(very, tau)
            if j < span:
                force_step(k + j, very)
            else:
                drift_sel(fixed, half)
                force_step(k + j, None)
        k += span
    return s


def energies(state: State, mass: np.ndarray):
    """Kinetic and potential energy at a base-step boundary (velocities
    synchronised, potentials of the last force computation)."""
    v = state.vel.astype(np.float64)
    return 0.5 * float(np.sum(mass * np.sum(v * v, 1))), 0.5 * float(np.sum(mass * state.pot))
