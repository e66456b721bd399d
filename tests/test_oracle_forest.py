"""Pins of the oracle's tree geometry and of the two-tree forest of
Sec. 3.2 (the fixed tree and the very active tree, built over the same
root box and walked together).  CPU only."""
import dataclasses

import numpy as np
import pytest

import oracle
import workloads


def _morton(pos, L, bits=21):
    """Interleaved key of the bisection sequence of a cube of side L:
    x first, then y, then z, most significant level first."""
    k = np.floor(pos / L * (1 << bits)).astype(np.int64)
    key = np.zeros(pos.shape[0], np.int64)
    for b in range(bits - 1, -1, -1):
        for a in range(3):
            key = (key << 1) | ((k[:, a] >> b) & 1)
    return key


def _check_bucket_order(tree, pos, L, first, count):
    """Buckets of a tree over a cube cover disjoint dyadic key ranges in
    increasing order, and keep input order inside."""
    key = _morton(pos[tree.perm], L)
    cells = [c for c in tree.bucket_cell if first <= tree.cell_first[c] < first + count]
    prev_max = -1
    for c in cells:
        f, k = tree.cell_first[c], tree.cell_count[c]
        kk = key[f:f + k]
        assert kk.min() > prev_max
        prev_max = kk.max()
        assert np.all(np.diff(tree.perm[f:f + k]) > 0)


@pytest.mark.parametrize("which", [0, 1])
def test_tree_order_follows_the_bisection_key(which):
    """The equal-volume longest-axis bisection of the unit cube cuts x, y,
    z in turn at dyadic planes, so the tree order of a periodic set is the
    order of the interleaved (Morton) key, level by level."""
    ps = [workloads.perturbed_lattice(8, 0.2, seed=12), workloads.make(3, scale_n1d=12)][which]
    t = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    _check_bucket_order(t, ps.pos, ps.box_L, 0, ps.n)


def _groups(n, frac, seed):
    rng = np.random.default_rng(seed)
    g = np.zeros(n, np.uint8)
    g[rng.choice(n, int(frac * n), replace=False)] = 1
    return g


@pytest.fixture(scope="module")
def forests():
    out = []
    for ps, frac in ((workloads.make(3, scale_n1d=12), 0.1), (workloads.plummer(1500, seed=11), 0.2)):
        g = _groups(ps.n, frac, 5)
        out.append((ps, g, oracle.build_forest(ps.pos, ps.mass, ps.box_L, g)))
    return out


@pytest.mark.parametrize("k", [0, 1])
def test_forest_structure(forests, k):
    ps, g, f = forests[k]
    n0 = int((g == 0).sum())
    assert np.array_equal(np.sort(f.perm), np.arange(ps.n))
    assert np.all(g[f.perm[:n0]] == 0) and np.all(g[f.perm[n0:]] == 1)
    r0, r1 = f.roots
    assert r0 == 0 and f.cell_first[r0] == 0 and f.cell_count[r0] == n0
    assert f.cell_first[r1] == n0 and f.cell_count[r1] == ps.n - n0
    fixed = np.arange(f.n_cell) < r1
    assert np.all(f.cell_first[fixed] + f.cell_count[fixed] <= n0)
    assert np.all(f.cell_first[~fixed] >= n0)
    inner = f.child[:, 0] >= 0
    assert np.all((f.child[fixed & inner] < r1)) and np.all(f.child[~fixed & inner] >= r1)
    assert np.all(f.cell_count[f.bucket_cell] <= 16)
    # each tree is the plain tree of its group over the common root box
    box = (np.array([0, 0, 0, 1.0, 1.0, 1.0]) * ps.box_L if ps.box_L > 0 else
           np.concatenate([ps.pos.min(0), ps.pos.max(0)]))
    t1 = oracle.build_tree(ps.pos[g == 1], ps.mass[g == 1], ps.box_L, 16, box)
    assert np.array_equal(f.cell_count[r1:], t1.cell_count)
    assert np.array_equal(f.com[r1:], t1.com)
    if ps.box_L > 0:
        # the same geometric planes: both trees follow the bisection key
        _check_bucket_order(f, ps.pos, ps.box_L, 0, n0)
        _check_bucket_order(f, ps.pos, ps.box_L, n0, ps.n - n0)
        t1d = oracle.build_tree(ps.pos[g == 1], ps.mass[g == 1], ps.box_L, 16)
        assert np.array_equal(t1d.perm, t1.perm)


def _active_sinks(f):
    return np.flatnonzero(f.bucket_cell >= f.roots[1])


@pytest.mark.parametrize("k", [0, 1])
def test_forest_lists_cover_every_particle_image_once(forests, k):
    ps, g, f = forests[k]
    sinks = _active_sinks(f)
    ls = oracle.build_lists(f, 0.7, ps.eps, sinks=sinks)
    nimg = ls.n_images
    allpairs = sorted((j, i) for j in range(ps.n) for i in range(nimg))
    for b in range(0, sinks.size, 5):
        pp = slice(ls.pp_off[b], ls.pp_off[b + 1])
        pc = slice(ls.pc_off[b], ls.pc_off[b + 1])
        got = []
        for cells, imgs in ((ls.pp_src[pp], ls.pp_img[pp]), (ls.pc_src[pc], ls.pc_img[pc])):
            for c, i in zip(cells, imgs):
                got.extend((j, int(i)) for j in range(f.cell_first[c],
                                                       f.cell_first[c] + f.cell_count[c]))
        assert sorted(got) == allpairs
        assert np.any((ls.pp_src[pp] == f.bucket_cell[sinks[b]]) & (ls.pp_img[pp] == 0))
        # sources from both trees
        assert np.any(ls.pp_src[pp] < f.roots[1]) or np.any(ls.pc_src[pc] < f.roots[1])


def test_forest_forces_reach_the_direct_sum():
    """Open Plummer set: with theta -> 0 every source is a PP pair and the
    forest gives the direct sum on the active particles; at theta = 0.7 it
    is within the method's error of it."""
    ps = workloads.plummer(1500, seed=11)
    g = _groups(ps.n, 0.2, 9)
    f = oracle.build_forest(ps.pos, ps.mass, 0.0, g)
    sinks = _active_sinks(f)
    sub = dataclasses.replace(f, bucket_cell=np.ascontiguousarray(f.bucket_cell[sinks]))
    pos_t, m_t = ps.pos[f.perm], ps.mass[f.perm]
    a_dir, p_dir = oracle.direct_open(ps.pos, ps.mass, ps.eps)
    n0 = f.cell_first[f.roots[1]]
    act = f.perm[n0:]
    for theta, tol in ((1e-3, 1e-13), (0.7, 3e-3)):
        ls = oracle.build_lists(sub, theta, ps.eps)
        a, p = oracle.evaluate(sub, ls, pos_t, m_t, ps.eps, 3)
        a, p = a[n0:], p[n0:]
        ref = a_dir[act]
        err = np.sqrt(np.mean(np.sum((a - ref) ** 2, 1) / np.sum(ref ** 2, 1)))
        assert err < tol, (theta, err)
        if theta < 0.01:
            assert np.allclose(p, p_dir[act], rtol=1e-13, atol=0)
