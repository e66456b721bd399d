"""Pins of the oracle's fast-multipole form (CC / CP interactions into 5th
order local expansions, Sec. 3.1): expansion convergence orders against
exact sums, exactness of the shift, the particle limit of the cell
expansion, exact coverage of every (particle, image) by the lists, the
acceptance rules, and the whole method against direct summation.  CPU
only."""
import numpy as np
import pytest

import oracle
import workloads


def _exact(pos, mass, eps, x):
    """Softened potential and acceleration at x of point masses."""
    r = x[None, :] - pos
    D = np.sum(r * r, 1) + eps * eps
    w = 1.0 / np.sqrt(D)
    return -(mass[:, None] * r * (w ** 3)[:, None]).sum(0), -(mass * w).sum()


def _slope(xs, ys):
    return np.polyfit(np.log(xs), np.log(ys), 1)[0]


def test_particle_expansion_converges_at_order_six():
    """CP: the local expansion of one mass about X_S, evaluated at X_S + h:
    the potential error falls as |h|^6 and the force error as |h|^5 (the
    first dropped terms are of order 6)."""
    XC = np.array([0.0, 0.0, 0.0])
    XS = np.array([1.0, 0.3, -0.2])
    eps = 1e-3
    L = oracle.fmm_m2l_point(None, 0.7, True, XS, XC, eps)
    hs, ep, ea = [], [], []
    for s in (0.02, 0.04, 0.08, 0.16):
        h = s * np.array([0.6, -0.5, 0.62])
        o = oracle.fmm_l2p_point(L, h)
        a, p = _exact(XC[None, :], np.array([0.7]), eps, XS + h)
        hs.append(s)
        ep.append(abs(o[3] - p))
        ea.append(np.linalg.norm(o[:3] - a))
    assert abs(_slope(hs, ep) - 6.0) < 0.3
    assert abs(_slope(hs, ea) - 5.0) < 0.3


def test_cell_expansion_of_one_particle_equals_the_particle_expansion():
    """Moments of orders >= 2 vanish for a single particle: CC = CP."""
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (1, 3))
    m = np.array([0.4])
    mom = oracle.moments(x, m)[1]
    XS = np.array([2.0, -1.0, 0.5])
    a = oracle.fmm_m2l_point(mom, 0.0, False, XS, x[0], 0.01)
    b = oracle.fmm_m2l_point(None, 0.4, True, XS, x[0], 0.01)
    assert np.allclose(a, b, rtol=1e-14, atol=1e-14 * np.abs(b).max())


def test_cell_to_local_converges_at_order_five():
    """CC of a cluster of size s at distance 1, evaluated at offset ~ s
    from X_S: the moments stop at order 4 and the expansion at total order
    5, so potential and force both err at order s^5 (the missing order-5
    moment), one order better than a quadrupole-free truncation at 3."""
    rng = np.random.default_rng(5)
    base = rng.uniform(-1, 1, (12, 3))
    m = rng.uniform(0.5, 1.5, 12)
    XS = np.array([1.0, 0.4, 0.2])
    hdir = np.array([-0.3, 0.5, 0.4])
    ss, ep, ea = [], [], []
    for s in (0.01, 0.02, 0.04, 0.08):
        pos = s * base
        X, mom = oracle.moments(pos, m)
        L = oracle.fmm_m2l_point(mom, 0.0, False, XS, X, 1e-4)
        o = oracle.fmm_l2p_point(L, s * hdir)
        a, p = _exact(pos, m, 1e-4, XS + s * hdir)
        ss.append(s)
        ep.append(abs(o[3] - p))
        ea.append(np.linalg.norm(o[:3] - a))
    assert abs(_slope(ss, ep) - 5.0) < 0.35
    assert abs(_slope(ss, ea) - 5.0) < 0.35


def test_shifting_an_expansion_is_exact():
    """The local expansion is a polynomial of degree 5: shifted by d and
    evaluated at h - d it gives what it gives at h."""
    rng = np.random.default_rng(7)
    L = oracle.fmm_m2l_point(None, 1.3, True, np.array([0.9, 0.2, 0.1]), np.zeros(3), 0.01)
    for _ in range(5):
        d = rng.uniform(-0.1, 0.1, 3)
        h = rng.uniform(-0.1, 0.1, 3)
        a = oracle.fmm_l2p_point(L, h)
        b = oracle.fmm_l2p_point(oracle.fmm_l2l_point(L, d), h - d)
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12 * np.abs(a).max())


@pytest.fixture(scope="module")
def fmm_sets():
    out = []
    for ps in (workloads.plummer(2000, seed=13), workloads.make(3, scale_n1d=12),
               workloads.perturbed_lattice(10, 0.2, seed=9)):
        t = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
        pt = ps.pos[t.perm]
        out.append((ps, t, pt, oracle.build_fmm_lists(t, pt, 0.7, ps.eps)))
    return out


@pytest.mark.parametrize("k", [0, 1, 2])
def test_fmm_lists_cover_every_particle_image_once(fmm_sets, k):
    ps, t, pt, fl = fmm_sets[k]
    nimg = fl.n_images
    parent = np.full(t.n_cell, -1)
    for c in range(t.n_cell):
        if t.child[c, 0] >= 0:
            parent[t.child[c]] = c
    allpairs = sorted((j, i) for j in range(ps.n) for i in range(nimg))
    n_cc = n_cp = 0
    for b in range(0, t.n_bucket, 4):
        got = []
        for e in range(fl.pp_off[b], fl.pp_off[b + 1]):
            c, sub = fl.pp_src[e], fl.pp_sub[e]
            assert t.child[c, 0] < 0
            rng_ = [t.cell_first[c] + sub - 1] if sub else range(t.cell_first[c],
                                                                   t.cell_first[c] + t.cell_count[c])
            got.extend((j, int(fl.pp_img[e])) for j in rng_)
        for e in range(fl.pc_off[b], fl.pc_off[b + 1]):
            c = fl.pc_src[e]
            got.extend((j, int(fl.pc_img[e])) for j in range(t.cell_first[c],
                                                               t.cell_first[c] + t.cell_count[c]))
        a = t.bucket_cell[b]
        while a >= 0:  # the bucket's expansion holds its ancestors' CC / CP sources
            for e in range(fl.cc_off[a], fl.cc_off[a + 1]):
                s = fl.cc_src[e]
                if s < 0:
                    got.append((~s, int(fl.cc_img[e])))
                    n_cp += 1
                else:
                    got.extend((j, int(fl.cc_img[e])) for j in range(t.cell_first[s],
                                                                       t.cell_first[s] + t.cell_count[s]))
                    n_cc += 1
            a = parent[a]
        assert sorted(got) == allpairs
    assert n_cc > 0


def _geom(t, pt, src, img, L):
    sh = oracle.image_shift(img, L)
    if src < 0:
        p = ~src
        X = pt[p] + sh
        return X, X, X, 0.0
    return t.com[src] + sh, t.bbox[src, :3] + sh, t.bbox[src, 3:] + sh, t.bmax[src]


def test_fmm_entries_obey_the_acceptance_rules(fmm_sets):
    ps, t, pt, fl = fmm_sets[1]
    theta, eps, L = 0.7, ps.eps, ps.box_L
    for s in range(0, t.n_cell, 3):
        for e in range(fl.cc_off[s], fl.cc_off[s + 1]):
            X, lo, hi, bm = _geom(t, pt, fl.cc_src[e], fl.cc_img[e], L)
            d = np.linalg.norm(X - t.com[s])
            gap = np.linalg.norm(np.maximum(0, np.maximum(lo - t.bbox[s, 3:], t.bbox[s, :3] - hi)))
            assert d > 1.5 * t.bmax[s] / theta + bm / theta and gap >= 2 * eps


def test_fmm_method_against_direct_summation(fmm_sets):
    """Open Plummer set: theta -> 0 leaves only PP pairs (the direct sum);
    at theta = 0.7 the method's error is in the paper's regime (well below
    1 %) and close to the bucket walk's."""
    ps, t, pt, fl = fmm_sets[0]
    mt = ps.mass[t.perm]
    a_dir, _ = oracle.direct_open(pt, mt, ps.eps)

    def err(a):
        return np.sqrt(np.mean(np.sum((a - a_dir) ** 2, 1) / np.sum(a_dir ** 2, 1)))
    a, _ = oracle.fmm_evaluate(t, fl, pt, mt, ps.eps, 3 | 8)
    e_fmm = err(a)
    lo = oracle.build_lists(t, 0.7, ps.eps)
    a_b, _ = oracle.evaluate(t, lo, pt, mt, ps.eps, 3)
    e_bucket = err(a_b)
    fl0 = oracle.build_fmm_lists(t, pt, 1e-3, ps.eps)
    a0, p0 = oracle.fmm_evaluate(t, fl0, pt, mt, ps.eps, 3 | 8)
    # what is left as CC / CP / PC has zero extent on one side (a bucket of
    # one particle), where the expansions are exact
    for s in np.flatnonzero(np.diff(fl0.cc_off)):
        srcs = fl0.cc_src[fl0.cc_off[s]:fl0.cc_off[s + 1]]
        assert t.bmax[s] == 0 or all(c < 0 or t.bmax[c] == 0 for c in srcs)
    assert err(a0) < 1e-13
    print(f"fmm {e_fmm:.3e} bucket walk {e_bucket:.3e} CC+CP entries {fl.cc_src.size}")
    assert e_fmm < 3e-3 and e_fmm < 3 * e_bucket


def test_fmm_periodic_with_ewald_against_the_bucket_walk(fmm_sets):
    """Periodic lattice: FMM + Ewald and bucket walk + Ewald agree within
    the method's error."""
    ps, t, pt, fl = fmm_sets[2]
    mt = ps.mass[t.perm]
    a, _ = oracle.fmm_evaluate(t, fl, pt, mt, ps.eps, 7 | 8)
    lo = oracle.build_lists(t, 0.7, ps.eps)
    a_b, _ = oracle.evaluate(t, lo, pt, mt, ps.eps, 7)
    scale = np.sqrt(np.mean(np.sum(a_b ** 2, 1)))
    diff = np.sqrt(np.mean(np.sum((a - a_b) ** 2, 1)))
    assert diff < 2e-2 * scale
