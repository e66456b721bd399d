"""Pins of the store and integrator oracle (oracle/kdk.py) against closed
forms: the integer grid, the schedule of rungs, the time-step criterion, a
Kepler orbit, time reversal, second-order convergence and energy
conservation with individual time steps.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import kdk

SCALE = 1.0 / kdk.TWO32


def test_grid_rounds_to_nearest_even_and_wraps():
    x = np.array([[0.5 * SCALE, 1.5 * SCALE, 2.5 * SCALE], [0.25, 0.75, 1.0 - 0.3 * SCALE]])
    q = kdk.quantize(x, (0, 0, 0), SCALE, True)
    assert q.tolist() == [[0, 2, 2], [1 << 30, 3 << 30, 0]]
    assert np.all(np.abs(kdk.decode(kdk.quantize(x[1:], (0, 0, 0), SCALE, True), (0, 0, 0),
                                    SCALE) - np.array([[0.25, 0.75, 0.0]])) == 0)
    rng = np.random.default_rng(1)
    y = rng.uniform(0, 1, (1000, 3))
    err = kdk.decode(kdk.quantize(y, (0, 0, 0), SCALE, True), (0, 0, 0), SCALE) - y
    err[err > 0.5] -= 1.0  # wrapped to the periodic image
    assert np.abs(err).max() <= 0.5 * SCALE
    with pytest.raises(ValueError):
        kdk.quantize(np.array([[2.0, 0, 0]]), (0, 0, 0), SCALE, False)


def test_drift_is_integer_and_wraps():
    q = np.array([[kdk.TWO32 - 1, 5, 0]], dtype=np.int64)
    v = np.array([[2.4, -5.6, 0.5]], dtype=np.float32)
    q2 = kdk.drift(q, v, SCALE, SCALE, True)  # one grid step per unit velocity
    assert q2.tolist() == [[1, 5 - 6, 0]] or q2.tolist() == [[1, kdk.TWO32 - 1, 0]]
    assert q2[0, 1] == kdk.TWO32 - 1  # 5 - 6 wraps
    assert q2[0, 0] == 1 and q2[0, 2] == 0  # rint(0.5) = 0 (ties to even)


def test_schedule_of_rungs():
    assert [kdk.boundary_rung(k, 3) for k in range(9)] == [0, 3, 2, 3, 1, 3, 2, 3, 0]
    # a particle on rung l is active 2^l times per base step
    for l in range(4):
        assert sum(1 for k in range(1, 9) if l >= kdk.boundary_rung(k, 3)) == 1 << l


def test_time_step_criterion_closed_form():
    eps, eta, dt = 0.01, 0.2, 0.1
    a = np.array([1e-6, 0.3, 1.0, 3.0, 40.0, 1e6, 0.0])
    r = kdk.rung_of(a, eps, eta, dt, 0, 6)
    for ai, ri in zip(a, r):
        if ai == 0:
            assert ri == 0
            continue
        want = max(0, math.ceil(math.log2(dt / (eta * math.sqrt(eps / ai)))))
        assert ri == min(want, 6)
    assert np.all(kdk.rung_of(a, eps, eta, dt, 2, 6) >= 2)


def _kepler(e=0.0, n_per_orbit=400):
    """Two bodies of mass 1/2 at separation 1 (apocentre for e > 0): the
    relative orbit has period 2 pi (G M = 1, semi-major axis 1/(1+e))."""
    a = 1.0 / (1.0 + e)
    v_apo = math.sqrt((1 - e) / (1 + e) / a)  # relative speed at apocentre
    pos = np.array([[-0.5, 0.0, 0.0], [0.5, 0.0, 0.0]])
    vel = np.array([[0.0, -0.5 * v_apo, 0.0], [0.0, 0.5 * v_apo, 0.0]], dtype=np.float32)
    mass = np.array([0.5, 0.5])
    period = 2 * math.pi * a ** 1.5
    return pos, vel, mass, period


def _direct(mass, eps):
    def forces(pos, active):
        return oracle.direct_open(pos, mass, eps)
    return forces


def _run(pos, vel, mass, eps, dt, steps, rung_max=0, eta=1e9):
    origin, scale = (-4.0, -4.0, -4.0), 8.0 / kdk.TWO32
    st = kdk.State(kdk.quantize(pos, origin, scale, False), vel.astype(np.float32),
                   np.zeros(len(mass), np.int64), None, None, origin, scale, False)
    f = _direct(mass, eps)
    st = kdk.start(st, f, eps, eta, dt, rung_max)
    e0 = sum(kdk.energies(st, mass))
    for _ in range(steps):
        st = kdk.base_step(st, f, eps, eta, dt, rung_max)
    return st, e0


def test_kepler_orbit_closes_and_conserves_energy():
    pos, vel, mass, period = _kepler(e=0.0)
    steps = 400
    st, e0 = _run(pos, vel, mass, 1e-6, period / steps, steps)
    x = kdk.decode(st.q, st.origin, st.scale)
    assert np.abs(x - pos).max() < 2e-3  # phase error O(dt^2)
    e1 = sum(kdk.energies(st, mass))
    assert abs(e1 - e0) < 1e-5 * abs(e0)
    # momentum: pairwise forces, both bodies kicked together
    p = (mass[:, None] * st.vel.astype(np.float64)).sum(0)
    assert np.abs(p).max() < 1e-7


def test_leapfrog_is_second_order():
    pos, vel, mass, period = _kepler(e=0.5)
    errs = []
    for steps in (200, 400):
        st, e0 = _run(pos, vel, mass, 1e-6, 0.5 * period / steps, steps)
        errs.append(abs(sum(kdk.energies(st, mass)) - e0))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_time_reversal_returns_to_the_start():
    pos, vel, mass, period = _kepler(e=0.5)
    dt, steps = period / 300, 120
    st, _ = _run(pos, vel, mass, 1e-6, dt, steps)
    back = kdk.State(st.q, (-st.vel).astype(np.float32), st.rung, None, None, st.origin,
                     st.scale, False)
    f = _direct(mass, 1e-6)
    back = kdk.start(back, f, 1e-6, 1e9, dt, 0)
    for _ in range(steps):
        back = kdk.base_step(back, f, 1e-6, 1e9, dt, 0)
    x = kdk.decode(back.q, back.origin, back.scale)
    assert np.abs(x - pos).max() < 1e-5
    assert np.abs(back.vel + vel).max() < 1e-5


def test_individual_time_steps_conserve_energy_on_a_plummer_sphere():
    import workloads
    ps = workloads.plummer(512, seed=5, eps=0.05, fp32_positions=False)
    eps, eta, dt, R = ps.eps, 0.2, 0.25, 4
    origin, scale = (-60.0, -60.0, -60.0), 120.0 / kdk.TWO32
    # virial velocities: isotropic, sigma^2 from the potential
    rng = np.random.default_rng(2)
    _, pot = oracle.direct_open(ps.pos, ps.mass, eps)
    v = np.sqrt(np.maximum(-pot, 0) / 3.0)[:, None] * rng.normal(size=(ps.n, 3)) * 0.7
    st = kdk.State(kdk.quantize(ps.pos, origin, scale, False), v.astype(np.float32),
                   np.zeros(ps.n, np.int64), None, None, origin, scale, False)
    f = _direct(ps.mass, eps)
    st = kdk.start(st, f, eps, eta, dt, R)
    hist = np.bincount(st.rung, minlength=R + 1)
    assert (hist > 0).sum() >= 3  # a spread of rungs
    e0 = sum(kdk.energies(st, ps.mass))
    log = []
    for _ in range(2):
        st = kdk.base_step(st, f, eps, eta, dt, R, log)
    e1 = sum(kdk.energies(st, ps.mass))
    assert abs(e1 - e0) < 2e-3 * abs(e0)
    # force computations follow the schedule: at boundary k the rungs >= l_k
    assert [lo for (_, lo, _) in log[:16]] == [kdk.boundary_rung(k, R) for k in range(1, 17)]
    assert all(cnt == ps.n for (k, lo, cnt) in log if lo == 0)


def test_fixed_rung_rule():
    """Sec. 3.2: the second tree for the rungs below the shallowest rung
    whose particles, with the deeper ones, are fewer than 5 %, at a step
    boundary of the rung above it, with two rungs below the fixed one."""
    R = 4
    r = np.array([0] * 96 + [3] * 4)
    assert kdk.fixed_rung(r, 0, R, 0.05) == 1     # 4 % on rungs >= 1: the whole base step
    assert kdk.fixed_rung(r, 8, R, 0.05) == 2     # mid-step: a boundary of rung 1, not 0
    assert kdk.fixed_rung(r, 4, R, 0.05) == 3
    assert kdk.fixed_rung(r, 6, R, 0.05) is None  # a boundary of rung 3 only
    r = np.array([0] * 50 + [1] * 46 + [3] * 4)
    assert kdk.fixed_rung(r, 0, R, 0.05) == 2     # rungs >= 1 hold half
    assert kdk.fixed_rung(r, 8, R, 0.05) == 2
    assert kdk.fixed_rung(r, 4, R, 0.05) == 3     # a boundary of rung 2 only
    assert kdk.fixed_rung(r, 2, R, 0.05) is None  # of rung 3 only: one rung below
    r = np.array([0] * 50 + [3] * 48 + [4] * 2)
    assert kdk.fixed_rung(r, 0, R, 0.05) is None  # only the deepest rung is small
    assert kdk.fixed_rung(np.zeros(100, np.int64), 0, R, 0.05) is None
    assert kdk.fixed_rung(np.array([0] * 99 + [2]), 0, R, 0.0) is None


def _plummer_512():
    import workloads
    ps = workloads.plummer(512, seed=5, eps=0.05, fp32_positions=False)
    origin, scale = (-60.0, -60.0, -60.0), 120.0 / kdk.TWO32
    rng = np.random.default_rng(2)
    _, pot = oracle.direct_open(ps.pos, ps.mass, ps.eps)
    v = np.sqrt(np.maximum(-pot, 0) / 3.0)[:, None] * rng.normal(size=(ps.n, 3)) * 0.7
    st = kdk.State(kdk.quantize(ps.pos, origin, scale, False), v.astype(np.float32),
                   np.zeros(ps.n, np.int64), None, None, origin, scale, False)
    return ps, st


def _direct3(mass, eps):
    f = _direct(mass, eps)
    return lambda pos, active, group=None: f(pos, active)


def test_fixed_schedule_without_intervals_is_the_plain_step():
    ps, st = _plummer_512()
    f = _direct3(ps.mass, ps.eps)
    st = kdk.start(st, f, ps.eps, 0.2, 0.25, 4)
    a = kdk.base_step(st, f, ps.eps, 0.2, 0.25, 4)
    b = kdk.base_step_fixed(st, f, ps.eps, 0.2, 0.25, 4, 0.0)
    for x, y in ((a.q, b.q), (a.vel, b.vel), (a.rung, b.rung), (a.acc, b.acc)):
        assert np.array_equal(x, y)


def test_fixed_tree_intervals_conserve_energy_and_track_the_plain_step():
    """Plummer 512 with rungs 0..4, 3 % on rung 3: intervals of rung 2 with
    the fixed particles at their midpoint.  The fixed particles end each
    interval where substep drifts put them (to a few grid steps, the
    rounding of 2 drifts against 4), the very active ones stay within the
    midpoint approximation of the plain trajectories, and energy is
    conserved as with the plain schedule."""
    ps, st0 = _plummer_512()
    f = _direct3(ps.mass, ps.eps)
    R, dt = 4, 0.25
    st0 = kdk.start(st0, f, ps.eps, 0.2, dt, R)
    e0 = sum(kdk.energies(st0, ps.mass))
    log = []
    a = kdk.base_step_fixed(st0, f, ps.eps, 0.2, dt, R, 0.05, log)
    b = kdk.base_step(st0, f, ps.eps, 0.2, dt, R)
    used = [k for (k, lo, cnt, g) in log if g]
    assert used, "no interval opened"
    assert all(lo >= 3 for (k, lo, cnt, g) in log if g)
    assert [lo for (_, lo, _, _) in log] == [kdk.boundary_rung(k, R) for k in range(1, 17)]
    fixed = st0.rung < 3  # rungs are shallower than 3 at the start: fixed in every interval
    dq = np.abs(a.q - b.q)
    assert dq[~fixed].max() > 0  # the approximation changes the very active orbits ...
    x_a = kdk.decode(a.q, a.origin, a.scale)
    x_b = kdk.decode(b.q, b.origin, b.scale)
    assert np.abs(x_a - x_b).max() < 1e-3  # ... a little
    e1 = sum(kdk.energies(a, ps.mass))
    assert abs(e1 - e0) < 2e-3 * abs(e0)
