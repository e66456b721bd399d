"""The device tree build and checklist walk against the oracle's.

What is unique is compared exactly: the tree's structure (particle order,
cell ranges, children, buckets) and bounding boxes, the buckets' centres of
mass, b_max and moments (the device repeats the oracle's operations in its
order), and the interaction lists.  A parent's centre of mass is summed
from its children on the device, in particle order by the oracle, so it
may differ in the last bits; its b_max follows, and its moments are the
children's shifted to it: those are compared within a tolerance.

Every test prints its case before the first device call."""
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


def _dev(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else a.astype(dtype))
    return torch.from_numpy(a).to(torch.device("cuda", 0))


def _coincident():
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 1, (600, 3))
    pos[100:140] = pos[7]          # 40 copies of one point: index halves below depth 64
    pos[300:320] = [0.5, 0.5, 0.5]
    return workloads.ParticleSet(pos, np.full(600, 1 / 600), 1e-3, 1.0, "coincident")


SETS = {
    "plummer_3000_open": lambda: workloads.plummer(3000, seed=21),
    "lattice_12": lambda: workloads.perturbed_lattice(12, 0.2, seed=22),
    "clustered_16": lambda: workloads.make(3, scale_n1d=16),
    "coincident_600": _coincident,
    "tiny_5_open": lambda: workloads.plummer(5, seed=4),
    "lattice_box2.5": lambda: (lambda b: workloads.ParticleSet(b.pos * 2.5, b.mass, b.eps * 2.5,
                                                               2.5))(
        workloads.perturbed_lattice(10, 0.2, seed=37)),
}


def compare_trees(mg, td, to, label):
    th = td.to_host()
    for f in ("perm", "cell_first", "cell_count", "child", "bucket_cell"):
        assert np.array_equal(getattr(th, f), getattr(to, f)), f"{label}: {f}"
    assert np.array_equal(th.bbox, to.bbox), f"{label}: bbox"
    leaf = to.child[:, 0] < 0
    assert np.array_equal(th.com[leaf], to.com[leaf]), f"{label}: bucket com"
    assert np.array_equal(th.bmax[leaf], to.bmax[leaf]), f"{label}: bucket bmax"
    assert np.array_equal(th.mom[leaf], to.mom[leaf]), f"{label}: bucket moments"
    # parents: centre of mass and b_max within 1e-10 of b_max plus 64 ulps
    # of the position (cells of coincident points have b_max ~ 0); moments
    # relative to M b_max^k, b_max floored at 1e-8 of the root's extent
    ulps = 64 * np.spacing(np.abs(to.com).max(1))
    dcom = np.maximum(np.abs(th.com - to.com).max(1) - ulps, 0) / np.maximum(to.bmax, 1e-300)
    assert dcom.max() < 1e-10, f"{label}: com {dcom.max()}"
    dbm = np.maximum(np.abs(th.bmax - to.bmax) - ulps, 0) / np.maximum(to.bmax, 1e-300)
    assert dbm.max() < 1e-10, f"{label}: bmax {dbm.max()}"
    extent = (to.bbox[to.roots[0], 3:] - to.bbox[to.roots[0], :3]).max()
    size = np.maximum(to.bmax, 1e-8 * extent)
    order = np.array([0] + [2] * 6 + [3] * 10 + [4] * 15)
    scale = to.mom[:, :1] * size[:, None] ** order[None, :]
    dm = np.abs(th.mom - to.mom) / scale
    assert dm.max() < 1e-9, f"{label}: moments {dm.max()}"
    print(f"  cells={to.n_cell} buckets={to.n_bucket} parent com {dcom.max():.2e} "
          f"moments {dm.max():.2e}", flush=True)


@pytest.mark.parametrize("name", list(SETS))
def test_device_tree_and_lists_equal_oracle(mg_ctx, name):
    mg, ctx = mg_ctx
    ps = SETS[name]()
    _case(f"device tree {name} n={ps.n} L={ps.box_L}")
    td = ctx.tree_build(_dev(ps.pos, np.float64), _dev(ps.mass, np.float64), ps.box_L, 16)
    to = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    compare_trees(mg, td, to, name)
    assert np.array_equal(td.pos.cpu().numpy(), ps.pos[to.perm])
    assert np.array_equal(td.mass.cpu().numpy(), ps.mass[to.perm])
    _case(f"device lists {name}")
    dl = ctx.lists_build(td, 0.7, ps.eps)
    lo = oracle.build_lists(to, 0.7, ps.eps)
    lh = dl.to_host()
    for f in ("pp_off", "pp_src", "pp_img", "pc_off", "pc_src", "pc_img"):
        assert np.array_equal(getattr(lh, f), getattr(lo, f)), f"{name}: {f}"
    print(f"  pp={lo.pp_src.size} pc={lo.pc_src.size}", flush=True)


def test_device_tree_feeds_the_evaluation(mg_ctx):
    """Device tree and lists bound as they are (no host copy): every part
    against the oracle on the oracle's tree and lists."""
    mg, ctx = mg_ctx
    ps = workloads.make(3, scale_n1d=24)
    _case(f"device tree + lists -> compute, clustered_24 n={ps.n}")
    td = ctx.tree_build(_dev(ps.pos, np.float64), _dev(ps.mass, np.float64), ps.box_L, 16)
    dl = ctx.lists_build(td, 0.7, ps.eps)
    keep, p = ctx.problem_device(td, dl, ps.eps, 0.7)
    ctx.bind(p, keep)
    acc, pot = ctx.outputs()
    ctx.compute(acc, pot)
    st = ctx.wait(120)
    ag = acc.cpu().numpy().reshape(3, -1).T
    to = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    lo = oracle.build_lists(to, 0.7, ps.eps)
    ao, po = oracle.evaluate(to, lo, ps.pos[to.perm], ps.mass[to.perm], ps.eps, 7)
    err = np.sqrt(np.mean(np.sum((ag - ao) ** 2, 1) / np.sum(ao ** 2, 1)))
    print(f"  pp={st.n_pp_interactions} pc={st.n_pc_interactions} rms {err:.3e}", flush=True)
    assert err < 1e-4


@pytest.mark.parametrize("name,frac", [("clustered_16", 0.1), ("plummer_3000_open", 0.2),
                                       ("lattice_12", 0.03)])
def test_device_forest_equals_oracle_forest(mg_ctx, name, frac):
    """The fixed and very active trees of Sec. 3.2 as one forest, and the
    lists of the very active buckets walked over both."""
    mg, ctx = mg_ctx
    ps = SETS[name]()
    rng = np.random.default_rng(17)
    g = np.zeros(ps.n, np.uint8)
    g[rng.choice(ps.n, max(1, int(frac * ps.n)), replace=False)] = 1
    _case(f"device forest {name} n={ps.n} active={int(g.sum())}")
    td = ctx.tree_build(_dev(ps.pos, np.float64), _dev(ps.mass, np.float64), ps.box_L, 16,
                        group_dev=_dev(g))
    fo = oracle.build_forest(ps.pos, ps.mass, ps.box_L, g)
    assert td.roots == fo.roots
    compare_trees(mg, td, fo, name + " forest")
    _case(f"device forest lists {name}")
    dl = ctx.lists_build(td, 0.7, ps.eps, sinks="second")
    sinks = np.arange(td.n_bucket_first, fo.n_bucket)
    assert np.all(fo.bucket_cell[sinks] >= fo.roots[1])
    lo = oracle.build_lists(fo, 0.7, ps.eps, sinks=sinks)
    lh = dl.to_host()
    assert np.all(lh.pp_off[:td.n_bucket_first + 1] == 0)
    for f in ("pp_off", "pc_off"):
        assert np.array_equal(getattr(lh, f)[td.n_bucket_first:], getattr(lo, f)), f
    for f in ("pp_src", "pp_img", "pc_src", "pc_img"):
        assert np.array_equal(getattr(lh, f), getattr(lo, f)), f
    # the forest evaluated with the active mask: forces on the very active
    # particles against the oracle's forest evaluation
    _case(f"device forest compute {name}")
    keep, p = ctx.problem_device(td, dl, ps.eps, 0.7)
    ctx.bind(p, keep)
    n0 = int(td.cell_count[0].item())  # particles of the fixed tree
    act = np.zeros(ps.n, np.uint8)
    act[n0:] = 1
    ctx.set_active(_dev(act))
    acc = torch.full((3 * ps.n,), -7.0, dtype=torch.float32, device=torch.device("cuda", 0))
    pot = torch.full((ps.n,), -7.0, dtype=torch.float32, device=torch.device("cuda", 0))
    ctx.compute(acc, pot)
    ctx.wait(120)
    ctx.set_active(None)
    ag = acc.cpu().numpy().reshape(3, -1).T
    import dataclasses
    sub = dataclasses.replace(fo, bucket_cell=np.ascontiguousarray(fo.bucket_cell[sinks]))
    ao, _ = oracle.evaluate(sub, lo, ps.pos[fo.perm], ps.mass[fo.perm], ps.eps, 7)
    err = np.sqrt(np.mean(np.sum((ag[n0:] - ao[n0:]) ** 2, 1) / np.sum(ao[n0:] ** 2, 1)))
    print(f"  active={ps.n - n0} rms {err:.3e}", flush=True)
    assert err < 1e-4
    assert np.all(ag[:n0] == -7.0)


@pytest.mark.parametrize("name,frac", [("clustered_16", 0.1), ("lattice_12", 0.03)])
def test_kept_fixed_tree_equals_one_call_forest(mg_ctx, name, frac):
    """Sec. 3.2: the fixed tree built once and the very active tree rebuilt
    alone behind it give, array for array, the forest of one call; again
    after the very active particles have moved (the fixed ones kept)."""
    mg, ctx = mg_ctx
    ps = SETS[name]()
    rng = np.random.default_rng(29)
    g = np.zeros(ps.n, np.uint8)
    g[rng.choice(ps.n, max(2, int(frac * ps.n)), replace=False)] = 1
    pos = ps.pos.copy()
    fields = ("perm", "pos", "mass", "cell_first", "cell_count", "child", "com", "bmax", "bbox",
              "mom", "bucket_cell")
    _case(f"kept fixed tree {name} n={ps.n} very active={int(g.sum())}")
    kf = ctx.forest_keep(_dev(pos, np.float64), _dev(ps.mass, np.float64), ps.box_L, _dev(g))
    for step in range(2):
        if step:  # the very active particles move, the fixed tree stays
            sel = g == 1
            pos[sel] = np.mod(pos[sel] + rng.normal(0, 0.01, (int(sel.sum()), 3)), ps.box_L)
            pos[pos >= ps.box_L] = 0.0
        _case(f"kept fixed tree {name} rebuild {step}")
        tk = ctx.forest_rebuild(kf, _dev(pos, np.float64), _dev(ps.mass, np.float64))
        tf = ctx.tree_build(_dev(pos, np.float64), _dev(ps.mass, np.float64), ps.box_L, 16,
                            group_dev=_dev(g))
        assert tk.n_cell_first == tf.n_cell_first and tk.roots == tf.roots
        for f in fields:
            a, b = getattr(tk, f).cpu().numpy(), getattr(tf, f).cpu().numpy()
            assert a.shape == b.shape and np.array_equal(a, b), f"{f} (rebuild {step})"
        lk = ctx.lists_build(tk, 0.7, ps.eps, sinks="second").to_host()
        lf = ctx.lists_build(tf, 0.7, ps.eps, sinks="second").to_host()
        for f in ("pp_off", "pc_off", "pp_src", "pp_img", "pc_src", "pc_img"):
            assert np.array_equal(getattr(lk, f), getattr(lf, f)), f
    with pytest.raises(ValueError):
        ctx.forest_keep(_dev(pos, np.float64), _dev(ps.mass, np.float64), 0.0, _dev(g))
    _case("tree offset: without ids the subset is a range; fewer ids than particles is rejected")
    t1 = ctx.tree_build(_dev(pos[:100], np.float64), _dev(ps.mass[:100], np.float64), ps.box_L)
    f1 = {f: getattr(t1, f) for f in fields}
    before = {f: v.cpu().numpy().copy() for f, v in f1.items()}
    ctx._tree_offset(f1, t1.cell_first.shape[0], t1.bucket_cell.shape[0], 100, 5, 7, None)
    after = {f: v.cpu().numpy() for f, v in f1.items()}
    assert np.array_equal(after["perm"], before["perm"] + 7)
    assert np.array_equal(after["cell_first"], before["cell_first"] + 7)
    assert np.array_equal(after["bucket_cell"], before["bucket_cell"] + 5)
    assert np.array_equal(after["child"], np.where(before["child"] >= 0, before["child"] + 5, -1))
    with pytest.raises(mg.MgravError) as e:
        ctx._tree_offset(f1, t1.cell_first.shape[0], t1.bucket_cell.shape[0], 100, 0, 0,
                         _dev(np.arange(50, dtype=np.int64)))
    assert e.value.status == mg.ERR_INVALID_ARG


def test_device_tree_errors(mg_ctx):
    mg, ctx = mg_ctx
    ps = workloads.perturbed_lattice(8, 0.2, seed=5)
    _case("device tree: capacity, bad input and an empty group are reported")
    with pytest.raises(mg.MgravError) as e:
        ctx.tree_build(_dev(ps.pos), _dev(ps.mass), ps.box_L, 16, cap=3)
    assert e.value.status == mg.ERR_INVALID_ARG and "capacity" in str(e.value)
    bad = ps.pos.copy()
    bad[5, 2] = 1.0  # on the upper face of the periodic box
    with pytest.raises(mg.MgravError) as e:
        ctx.tree_build(_dev(bad), _dev(ps.mass), ps.box_L, 16)
    assert e.value.status == mg.ERR_INVALID_ARG
    with pytest.raises(mg.MgravError) as e:
        ctx.tree_build(_dev(ps.pos), _dev(ps.mass), ps.box_L, 16,
                       group_dev=_dev(np.zeros(ps.n, np.uint8)))
    assert e.value.status == mg.ERR_INVALID_ARG
    # a later build on the same context works
    td = ctx.tree_build(_dev(ps.pos), _dev(ps.mass), ps.box_L, 16)
    to = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    assert np.array_equal(td.to_host().perm, to.perm)


def test_long_checklists_take_the_overflow_pass(mg_ctx):
    """Clustered 48^3 with 0.2 % of the particles, scattered, in the very
    active tree: its buckets are wide, their checklists among the dense
    fixed cells grow past the walk's LDS ring (1183 entries at the peak on
    the host), and the second pass with the global ring must give the
    oracle's lists all the same."""
    mg, ctx = mg_ctx
    ps = workloads.make(3, scale_n1d=48)
    rng = np.random.default_rng(1)
    g = np.zeros(ps.n, np.uint8)
    g[rng.choice(ps.n, int(0.002 * ps.n), replace=False)] = 1
    _case(f"device forest clustered_48 n={ps.n} active={int(g.sum())} (long checklists)")
    td = ctx.tree_build(_dev(ps.pos, np.float64), _dev(ps.mass, np.float64), ps.box_L, 16,
                        group_dev=_dev(g))
    dl = ctx.lists_build(td, 0.7, ps.eps, sinks="second")
    fo = oracle.build_forest(ps.pos, ps.mass, ps.box_L, g)
    sinks = np.arange(td.n_bucket_first, fo.n_bucket)
    lo = oracle.build_lists(fo, 0.7, ps.eps, sinks=sinks)
    lh = dl.to_host()
    for f in ("pp_off", "pc_off"):
        assert np.array_equal(getattr(lh, f)[td.n_bucket_first:], getattr(lo, f)), f
    for f in ("pp_src", "pp_img", "pc_src", "pc_img"):
        assert np.array_equal(getattr(lh, f), getattr(lo, f)), f
    print(f"  sinks={sinks.size} pp={lo.pp_src.size} pc={lo.pc_src.size}", flush=True)
