"""The fast-multipole form on the device (CC / CP interactions into 5th
order local expansions, Sec. 3.1) against the oracle: every bucket's
expansion coefficient by coefficient (both sides in double), and the whole
force (PP and PC of the FMM lists in float, the expansions in double, the
Ewald correction) particle by particle.  Every test prints its case before
the first device call."""
import numpy as np
import pytest

import oracle
import workloads

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


def _packed_from_full(L364):
    """The 56 coefficients (order <= 5; decreasing x, then y exponent) of a
    full-tensor expansion (364 values: orders 0..5, 3^n each)."""
    off = [0, 1, 4, 13, 40, 121]
    out = []
    for n in range(6):
        for x in range(n, -1, -1):
            for y in range(n - x, -1, -1):
                z = n - x - y
                axes = [0] * x + [1] * y + [2] * z
                flat = 0
                for a in axes:
                    flat = 3 * flat + a
                out.append(L364[..., off[n] + flat])
    return np.stack(out, axis=-1)


SETS = {
    "plummer_4096_open": lambda: workloads.plummer(4096, seed=23),
    "clustered_16": lambda: workloads.make(3, scale_n1d=16),
    "lattice_16": lambda: workloads.perturbed_lattice(16, 0.2, seed=29),
}


@pytest.mark.parametrize("name", list(SETS))
def test_fmm_matches_the_oracle(mg_ctx, name):
    mg, ctx = mg_ctx
    ps = SETS[name]()
    dev = torch.device("cuda", 0)
    t = mg.tree_build(ps.pos, ps.mass, ps.box_L, 16)
    pt, mt = ps.pos[t.perm], ps.mass[t.perm]
    fl = mg.fmm_lists_build(t, pt, 0.7, ps.eps)
    _case(f"fmm {name} n={ps.n}: pp={fl.pp_src.size} pc={fl.pc_src.size} cc+cp={fl.cc_src.size}")
    keep, p = ctx.upload(pt, mt, t, fl, ps.eps, 0.7)
    ctx.bind(p, keep)
    acc, pot = ctx.outputs()
    ctx.compute(acc, pot)
    st = ctx.wait(120)
    fl_dev = {k: torch.from_numpy(np.ascontiguousarray(getattr(fl, k) if getattr(fl, k).size
                                                        else np.zeros(1, getattr(fl, k).dtype))
                                  ).to(dev) for k in ("cc_off", "cc_src", "cc_img")}
    _case(f"fmm {name}: local expansions")
    local = ctx.fmm_apply(keep["pos"], keep["mass"], keep, fl_dev, ps.eps, ps.box_L, acc, pot,
                          want_local=True)
    ag = acc.cpu().numpy().reshape(3, -1).T
    pg = pot.cpu().numpy()
    Ld = local.cpu().numpy()
    to = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    lo = oracle.build_fmm_lists(to, pt, 0.7, ps.eps)
    Lo = oracle.fmm_local(to, lo, pt, mt, ps.eps)
    Lob = _packed_from_full(Lo[to.bucket_cell])
    # each coefficient against the largest of its order over all buckets
    order = np.array([n for n in range(6) for _ in range((n + 1) * (n + 2) // 2)])
    scale = np.array([np.abs(Lob[:, order == n]).max() for n in range(6)])[order]
    dl = np.abs(Ld - Lob) / scale
    parts = 7 if ps.box_L > 0 else 3
    ao, po = oracle.fmm_evaluate(to, lo, pt, mt, ps.eps, parts | 8, local=Lo)
    _, p_tree = oracle.fmm_evaluate(to, lo, pt, mt, ps.eps, 3 | 8, local=Lo)
    rel = np.sqrt(np.sum((ag - ao) ** 2, 1) / np.sum(ao ** 2, 1))
    perr = np.sqrt(np.sum((pg - po) ** 2) / np.sum(p_tree ** 2))
    print(f"  expansions max rel {dl.max():.3e}; acc rms {np.sqrt(np.mean(rel ** 2)):.3e} max "
          f"{rel.max():.3e}; pot {perr:.3e}; pp={st.n_pp_interactions} "
          f"pc={st.n_pc_interactions}", flush=True)
    assert dl.max() < 1e-9
    assert np.sqrt(np.mean(rel ** 2)) < 1e-4
    assert perr < 1e-5


def test_fmm_active_subset(mg_ctx):
    """With an active mask only active particles get the expansion part,
    bitwise as in the full run; the others keep their values."""
    mg, ctx = mg_ctx
    ps = workloads.make(3, scale_n1d=16)
    dev = torch.device("cuda", 0)
    t = mg.tree_build(ps.pos, ps.mass, ps.box_L, 16)
    pt, mt = ps.pos[t.perm], ps.mass[t.perm]
    fl = mg.fmm_lists_build(t, pt, 0.7, ps.eps)
    _case("fmm clustered_16: active subset")
    keep, p = ctx.upload(pt, mt, t, fl, ps.eps, 0.7)
    fl_dev = {k: torch.from_numpy(getattr(fl, k)).to(dev) for k in ("cc_off", "cc_src", "cc_img")}
    ctx.bind(p, keep)
    acc, pot = ctx.outputs()
    ctx.compute(acc, pot)
    ctx.wait(120)
    ctx.fmm_apply(keep["pos"], keep["mass"], keep, fl_dev, ps.eps, ps.box_L, acc, pot)
    a_full, p_full = acc.cpu().numpy().copy(), pot.cpu().numpy().copy()
    act = (np.random.default_rng(3).uniform(size=ps.n) < 0.1).astype(np.uint8)
    act_d = torch.from_numpy(act).to(dev)
    ctx.set_active(act_d)
    acc2 = torch.full_like(acc, -9.0)
    pot2 = torch.full_like(pot, -9.0)
    ctx.compute(acc2, pot2)
    ctx.wait(120)
    ctx.fmm_apply(keep["pos"], keep["mass"], keep, fl_dev, ps.eps, ps.box_L, acc2, pot2,
                  active_dev=act_d)
    ctx.set_active(None)
    a2, p2 = acc2.cpu().numpy(), pot2.cpu().numpy()
    on = act.astype(bool)
    A, A2 = a_full.reshape(3, -1), a2.reshape(3, -1)
    assert np.array_equal(A2[:, on], A[:, on]) and np.array_equal(p2[on], p_full[on])
    assert np.all(A2[:, ~on] == -9.0) and np.all(p2[~on] == -9.0)
