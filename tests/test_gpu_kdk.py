"""The particle store (Sec. 3.4) and the hierarchical KDK integrator with
individual time steps (Sec. 3.2) on the device, against oracle/kdk.py.

Store kernels are compared bit for bit with the oracle's grid arithmetic
on the same inputs.  The integrator runs the same schedule on both sides
with each side's own forces (device: float PP + PC on its tree and lists;
oracle: FP64 on its own), so trajectories agree to the force error; rungs
and the schedule (active counts per substep, dual-tree substeps) must be
identical.  Every test prints its case before the first device call."""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads
from oracle import kdk

try:  # imported at collection so its one-off start-up cost is not a test's
    import torch
except ImportError:  # pragma: no cover
    torch = None

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"\n[gpu case] {msg}", flush=True)


@pytest.fixture(scope="module")
def mg_ctx():
    if torch is None or not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_08621_amd as mg
    ctx = mg.Context(0)
    yield mg, ctx
    ctx.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(torch.device("cuda", 0))


def _q64(st):
    return st.q.cpu().numpy().astype(np.int64) & 0xffffffff


@pytest.mark.parametrize("periodic", [True, False])
def test_store_kernels_match_the_oracle_grid(mg_ctx, periodic):
    mg, ctx = mg_ctx
    rng = np.random.default_rng(8)
    n = 5000
    if periodic:
        pos = rng.uniform(0, 1, (n, 3))
        pos[:7] = [[0.5 / 2 ** 32, 1.5 / 2 ** 32, 2.5 / 2 ** 32]] * 7  # ties to even
        pos[7] = [1 - 0.3 / 2 ** 32, 0.25, 0.75]                       # rounds up to 2^32: wraps
        origin, scale = (0.0, 0.0, 0.0), 1.0 / 2 ** 32
    else:
        pos = rng.normal(0, 3, (n, 3))
        origin, scale = (-60.0, -60.0, -60.0), 120.0 / 2 ** 32
    vel = rng.normal(0, 1, (n, 3)).astype(np.float32)
    _case(f"store encode/decode/permute/drift/kick periodic={periodic}")
    st = ctx.store_alloc(n, origin, scale)
    ctx.store_encode(st, _dev(pos), _dev(vel), periodic)
    q_or = kdk.quantize(pos, origin, scale, periodic)
    assert np.array_equal(_q64(st), q_or)
    x = ctx.store_decode(st).cpu().numpy()
    assert np.abs(x - kdk.decode(q_or, origin, scale)).max() <= 2 * np.spacing(60.0)
    assert np.array_equal(st.vel.cpu().numpy(), vel)
    perm = rng.permutation(n)
    st2 = ctx.store_permute(st, _dev(perm))
    assert np.array_equal(_q64(st2), q_or[perm])
    dt = 3e-3 * (1.0 if periodic else 40.0)
    ctx.store_drift(st2, dt, periodic)
    assert np.array_equal(_q64(st2), kdk.drift(q_or[perm], vel[perm], dt, scale, periodic))
    acc = rng.normal(0, 2, (3, n)).astype(np.float32)
    rung = rng.integers(0, 5, n)
    st2.aux.copy_(_dev(rung.astype(np.int32)))
    ctx.store_kick(st2, _dev(acc.ravel()), 0.1, 2)
    want = kdk.half_kick(vel[perm], acc.T.astype(np.float64), rung, 0.1, rung >= 2)
    assert np.array_equal(st2.vel.cpu().numpy(), want)
    ctx.store_rungs(st2, _dev(acc.ravel()), 0.01, 0.2, 0.1, 1, 1, 6)
    amag = np.linalg.norm(acc.T.astype(np.float64), axis=1)
    want_r = rung.copy()
    sel = rung >= 1
    want_r[sel] = kdk.rung_of(amag[sel], 0.01, 0.2, 0.1, 1, 6)
    assert np.array_equal(st2.rung.cpu().numpy(), want_r)
    act = ctx.store_active(st2, 3).cpu().numpy()
    assert np.array_equal(act, (want_r >= 3).astype(np.uint8))


def _oracle_forces(mass, eps, theta, L, dual_below):
    parts = 7 if L > 0 else 3

    def forces(pos, active):
        n = pos.shape[0]
        n_act = int(active.sum())
        acc, pot = np.zeros((n, 3)), np.zeros(n)
        if n_act == 0:
            return acc, pot
        if n_act < dual_below * n:
            t = oracle.build_forest(pos, mass, L, active.astype(np.uint8))
            sinks = np.flatnonzero(t.bucket_cell >= t.roots[1])
            lists = oracle.build_lists(t, theta, eps, sinks=sinks)
            t = dataclasses.replace(t, bucket_cell=np.ascontiguousarray(t.bucket_cell[sinks]))
        else:
            t = oracle.build_tree(pos, mass, L, 16)
            lists = oracle.build_lists(t, theta, eps)
        a_t, p_t = oracle.evaluate(t, lists, pos[t.perm], mass[t.perm], eps, parts)
        acc[t.perm] = a_t
        pot[t.perm] = p_t
        return acc, pot
    return forces


def _run_both(mg, ctx, pos, vel, mass, eps, theta, L, dt, R, steps, origin, scale, label):
    from paper_1609_08621_amd.kdk import Integrator
    _case(f"kdk {label}: device, {steps} base steps of 2^{R} substeps")
    it = Integrator(ctx, _dev(pos), _dev(vel), mass[0], eps, theta, L, dt, R, origin=origin,
                    scale=scale)
    it.start()
    e_dev = [sum(it.energies())]
    for _ in range(steps):
        it.base_step()
        e_dev.append(sum(it.energies()))
    _case(f"kdk {label}: oracle")
    periodic = L > 0
    f = _oracle_forces(mass, eps, theta, L, it.dual_below)
    so = kdk.State(kdk.quantize(pos, origin, scale, periodic), vel.astype(np.float32),
                   np.zeros(len(mass), np.int64), None, None, origin, scale, periodic)
    so = kdk.start(so, f, eps, 0.2, dt, R)
    e_or = [sum(kdk.energies(so, mass))]
    log = []
    for _ in range(steps):
        so = kdk.base_step(so, f, eps, 0.2, dt, R, log)
        e_or.append(sum(kdk.energies(so, mass)))
    return it, so, e_dev, e_or, log


def test_kdk_plummer_matches_the_oracle_and_conserves_energy(mg_ctx):
    """Open Plummer sphere, 2048 particles, four rungs below the base step:
    the device integrator against the oracle's, two base steps."""
    mg, ctx = mg_ctx
    ps = workloads.plummer(2048, seed=31, eps=0.01, fp32_positions=False)
    rng = np.random.default_rng(4)
    _, pot = oracle.direct_open(ps.pos, ps.mass, ps.eps)
    vel = (np.sqrt(np.maximum(-pot, 0) / 3.0)[:, None] * rng.normal(size=(ps.n, 3)) * 0.7)
    origin, scale = (-60.0, -60.0, -60.0), 120.0 / 2 ** 32
    it, so, e_dev, e_or, log = _run_both(mg, ctx, ps.pos, vel.astype(np.float32), ps.mass,
                                         ps.eps, 0.7, 0.0, 0.125, 4, 2, origin, scale,
                                         "plummer_2048")
    pos_d, vel_d, rung_d, acc_d, pot_d = [t.cpu().numpy() for t in it.state()]
    print(f"  rungs {np.bincount(rung_d, minlength=5)}; substeps (k, lo, active, dual): "
          f"{it.log[:8]}", flush=True)
    assert [(k, lo, n) for (k, lo, n, _) in it.log] == [(k, lo, n) for (k, lo, n) in log]
    assert any(d for (*_, d) in it.log), "no substep used the very active tree"
    assert np.array_equal(rung_d, so.rung)
    x_or = kdk.decode(so.q, origin, scale)
    dx = np.abs(pos_d - x_or).max()
    dv = np.abs(vel_d - so.vel).max() / np.sqrt(np.mean(so.vel.astype(np.float64) ** 2))
    print(f"  max |dx| {dx:.3e}, max |dv|/v_rms {dv:.3e}; energy device {e_dev} "
          f"oracle {e_or}", flush=True)
    assert dx < 1e-5 and dv < 1e-4
    for e in (e_dev, e_or):
        assert abs(e[-1] - e[0]) < 2e-3 * abs(e[0])


def test_kdk_periodic_lattice_matches_the_oracle(mg_ctx):
    """Periodic perturbed lattice 12^3 (exact Ewald), small random
    velocities, one base step of four substeps: wrapping on the integer
    grid and the periodic force path inside the integrator."""
    mg, ctx = mg_ctx
    ps = workloads.perturbed_lattice(12, 0.3, seed=41)
    rng = np.random.default_rng(6)
    vel = rng.normal(0, 0.05, (ps.n, 3)).astype(np.float32)
    it, so, e_dev, e_or, log = _run_both(mg, ctx, ps.pos, vel, ps.mass, ps.eps, 0.7, 1.0,
                                         0.02, 2, 1, (0.0, 0.0, 0.0), 1.0 / 2 ** 32,
                                         "lattice_12")
    pos_d, vel_d, rung_d, _, _ = [t.cpu().numpy() for t in it.state()]
    assert [(k, lo, n) for (k, lo, n, _) in it.log] == [(k, lo, n) for (k, lo, n) in log]
    assert np.array_equal(rung_d, so.rung)
    x_or = kdk.decode(so.q, (0.0, 0.0, 0.0), 1.0 / 2 ** 32)
    d = np.abs(pos_d - x_or)
    d = np.minimum(d, 1.0 - d)  # periodic images
    dv = np.abs(vel_d - so.vel).max() / np.sqrt(np.mean(so.vel.astype(np.float64) ** 2))
    print(f"  max |dx| {d.max():.3e}, max |dv|/v_rms {dv:.3e}", flush=True)
    assert d.max() < 1e-6 and dv < 1e-4


def test_kdk_fixed_tree_matches_the_oracle(mg_ctx):
    """Sec. 3.2 with the fixed tree kept: clustered 12^3 (periodic, exact
    Ewald) from rest, rungs 0..4 with 3 % on rung 3, so that intervals of
    rung 2 open; the device (fixed tree built once per interval, very
    active tree rebuilt behind it) against oracle/kdk.base_step_fixed
    with the oracle's forest, one base step."""
    mg, ctx = mg_ctx
    from paper_1609_08621_amd.kdk import Integrator
    ps = workloads.make(3, scale_n1d=12)
    t = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    a, _ = oracle.evaluate(t, oracle.build_lists(t, 0.7, ps.eps), ps.pos[t.perm],
                           ps.mass[t.perm], ps.eps, 7)
    am = np.zeros(ps.n)
    am[t.perm] = np.linalg.norm(a, axis=1)
    R = 4
    dt = float(np.quantile(0.2 * np.sqrt(ps.eps / am), 0.03)) * 4 * 1.0001
    origin, scale = (0.0, 0.0, 0.0), 1.0 / 2 ** 32
    vel = np.zeros((ps.n, 3), np.float32)
    _case(f"kdk fixed tree clustered_12: device, 1 base step of 2^{R} substeps, dt {dt:.4g}")
    it = Integrator(ctx, _dev(ps.pos), _dev(vel), ps.mass[0], ps.eps, 0.7, 1.0, dt, R,
                    origin=origin, scale=scale, dual_mode="fixed")
    it.start()
    it.base_step()
    _case("kdk fixed tree clustered_12: oracle")
    f0 = _oracle_forces(ps.mass, ps.eps, 0.7, 1.0, it.dual_below)

    def f(pos, active, group=None):
        if group is None:
            return f0(pos, active)
        tr = oracle.build_forest(pos, ps.mass, 1.0, group.astype(np.uint8))
        sinks = np.flatnonzero(tr.bucket_cell >= tr.roots[1])
        lists = oracle.build_lists(tr, 0.7, ps.eps, sinks=sinks)
        tr = dataclasses.replace(tr, bucket_cell=np.ascontiguousarray(tr.bucket_cell[sinks]))
        a_t, p_t = oracle.evaluate(tr, lists, pos[tr.perm], ps.mass[tr.perm], ps.eps, 7)
        acc, pot = np.zeros((len(ps.mass), 3)), np.zeros(len(ps.mass))
        acc[tr.perm] = a_t
        pot[tr.perm] = p_t
        return acc, pot
    so = kdk.State(kdk.quantize(ps.pos, origin, scale, True), vel, np.zeros(ps.n, np.int64),
                   None, None, origin, scale, True)
    so = kdk.start(so, f, ps.eps, 0.2, dt, R)
    log = []
    so = kdk.base_step_fixed(so, f, ps.eps, 0.2, dt, R, it.dual_below, log)
    pos_d, vel_d, rung_d, _, _ = [x.cpu().numpy() for x in it.state()]
    print(f"  rungs {np.bincount(rung_d, minlength=R + 1)}; kept-tree substeps {it.kept}; "
          f"log {it.log}", flush=True)
    assert [(k, lo, n) for (k, lo, n, _) in it.log] == [(k, lo, n) for (k, lo, n, _) in log]
    assert it.kept and it.kept == [k for (k, _, _, g) in log if g]
    assert np.array_equal(rung_d, so.rung)
    x_or = kdk.decode(so.q, origin, scale)
    d = np.abs(pos_d - x_or)
    d = np.minimum(d, 1.0 - d)
    dv = np.abs(vel_d - so.vel).max() / np.sqrt(np.mean(so.vel.astype(np.float64) ** 2))
    print(f"  max |dx| {d.max():.3e}, max |dv|/v_rms {dv:.3e}", flush=True)
    assert d.max() < 1e-6 and dv < 1e-4


def test_store_positions_give_identical_forces(mg_ctx):
    """The 64^3 lattice on the 2^32 grid of the unit box: the evaluation
    reading positions from the store (12 bytes, equal masses without an
    array) gives the same bits as reading the decoded doubles."""
    mg, ctx = mg_ctx
    ps = workloads.make(2)
    origin, scale = (0.0, 0.0, 0.0), 1.0 / 2 ** 32
    _case(f"store positions vs doubles, lattice_64 n={ps.n}")
    st = ctx.store_alloc(ps.n, origin, scale)
    ctx.store_encode(st, _dev(ps.pos), None, True)
    pos = ctx.store_decode(st)
    mass = torch.full((ps.n,), ps.mass[0], dtype=torch.float64, device=pos.device)
    td = ctx.tree_build(pos, mass, 1.0, 16)
    dl = ctx.lists_build(td, 0.7, ps.eps)
    st = ctx.store_permute(st, td.perm)
    out = []
    for use_store in (False, True):
        keep, p = ctx.problem_device(td, dl, ps.eps, 0.7)
        if use_store:
            p.pos, p.pos_q, p.q_scale = None, st.q.data_ptr(), scale
            p.mass, p.mass_uniform = None, float(ps.mass[0])
            keep["q"] = st.q
        ctx.bind(p, keep)
        acc, pot = ctx.outputs()
        ctx.compute(acc, pot)
        ctx.wait(120)
        out.append((acc.cpu().numpy(), pot.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
