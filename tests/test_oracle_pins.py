"""Pins of the FP64 oracle against mathematics it does not itself encode.

Each test checks the oracle against a closed form, an invariant, a limit,
a literature constant, brute force, or a convergence order, chosen so that
a plausible slip (a dropped term, a wrong sign or index, a transposed
operand) fails one of them.  CPU only.
"""
import math
import os

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].split()
            if len(line) >= 2:
                vals[line[0]] = [float(x) for x in line[1:]]
    return vals


XI = _golden("ewald_constants.txt")["XI"][0]


def _rel_rms(a, ref):
    return float(np.sqrt(np.mean(np.sum((a - ref) ** 2, axis=1) / np.sum(ref ** 2, axis=1))))


# ---------------------------------------------------------------- tree ----

@pytest.fixture(scope="module")
def small_sets():
    return [
        workloads.plummer(1500, seed=11),
        workloads.perturbed_lattice(8, 0.2, seed=12),
        workloads.make(3, scale_n1d=12),
    ]


def test_tree_invariants(small_sets):
    for ps in small_sets:
        t = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
        n = ps.n
        assert np.array_equal(np.sort(t.perm), np.arange(n))
        pos = ps.pos[t.perm]
        m = ps.mass[t.perm]
        # buckets partition [0, n) in order and hold <= 16 particles
        first = t.cell_first[t.bucket_cell]
        cnt = t.cell_count[t.bucket_cell]
        assert first[0] == 0 and np.all(first[1:] == first[:-1] + cnt[:-1])
        assert first[-1] + cnt[-1] == n
        assert cnt.min() >= 1 and cnt.max() <= 16
        for c in range(t.n_cell):
            f, k = t.cell_first[c], t.cell_count[c]
            l, r = t.child[c]
            x = pos[f:f + k]
            mm = m[f:f + k]
            assert np.isclose(t.mom[c, 0], mm.sum(), rtol=1e-14)
            com = (mm[:, None] * x).sum(0) / mm.sum()
            assert np.allclose(t.com[c], com, rtol=0, atol=1e-13)
            d = np.sqrt(((x - t.com[c]) ** 2).sum(1))
            assert abs(t.bmax[c] - d.max()) <= 1e-13
            assert np.all(t.bbox[c, :3] == x.min(0)) and np.all(t.bbox[c, 3:] == x.max(0))
            if l < 0:
                assert r < 0 and k <= 16
                continue
            assert k > 16
            # node-left-right numbering, nested contiguous ranges
            assert l == c + 1
            assert t.cell_first[l] == f and t.cell_first[r] == f + t.cell_count[l]
            assert t.cell_count[l] + t.cell_count[r] == k
            # the two children are separated by an axis-aligned plane
            xl = pos[f:f + t.cell_count[l]]
            xr = pos[t.cell_first[r]:f + k]
            assert any(xl[:, a].max() < xr[:, a].min() for a in range(3))
            # parent mass and centre of mass are the children's mass-weighted ones
            ml, mr = t.mom[l, 0], t.mom[r, 0]
            assert np.isclose(ml + mr, t.mom[c, 0], rtol=1e-14)
            assert np.allclose((ml * t.com[l] + mr * t.com[r]) / (ml + mr), t.com[c], atol=1e-13)


def test_tree_split_is_equal_volume_bisection():
    # Four points at the corners of a unit square's quadrants, bucket 1: the
    # root box [0,1]^2 x [0,1] (periodic) is cut at 1/2 along x first
    # (lowest index on ties), then each half at 1/2 along y.
    pos = np.array([[0.7, 0.2, 0.5], [0.2, 0.7, 0.5], [0.2, 0.2, 0.5], [0.7, 0.7, 0.5]])
    t = oracle.build_tree(pos, np.ones(4), 1.0, 1)
    # node-left-right: root, [x<.5], [x<.5,y<.5], [x<.5,y>=.5], [x>=.5], ...
    leaves = [tuple(pos[t.perm[t.cell_first[c]]][:2]) for c in t.bucket_cell]
    assert leaves == [(0.2, 0.2), (0.2, 0.7), (0.7, 0.2), (0.7, 0.7)]
    # a particle exactly on the plane goes to the upper child
    pos2 = np.array([[0.5, 0.1, 0.1], [0.1, 0.1, 0.1]])
    t2 = oracle.build_tree(pos2, np.ones(2), 1.0, 1)
    assert list(t2.perm) == [1, 0]


def test_tree_coincident_points_terminate():
    pos = np.full((40, 3), 0.25)
    t = oracle.build_tree(pos, np.ones(40), 1.0, 16)
    assert t.cell_count[t.bucket_cell].max() <= 16
    assert t.cell_count[t.bucket_cell].sum() == 40


# --------------------------------------------------------------- lists ----

def _expand(tree, cells, imgs):
    out = []
    for c, i in zip(cells, imgs):
        f, k = tree.cell_first[c], tree.cell_count[c]
        out.extend((j, int(i)) for j in range(f, f + k))
    return out


@pytest.mark.parametrize("which", [0, 1, 2])
def test_lists_cover_every_particle_image_once(small_sets, which):
    ps = small_sets[which]
    t = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    ls = oracle.build_lists(t, 0.7, ps.eps)
    nimg = ls.n_images
    assert nimg == (27 if ps.box_L > 0 else 1)
    allpairs = sorted((j, i) for j in range(ps.n) for i in range(nimg))
    mtot = ps.mass.sum()
    for b in range(0, t.n_bucket, 3):
        pp = slice(ls.pp_off[b], ls.pp_off[b + 1])
        pc = slice(ls.pc_off[b], ls.pc_off[b + 1])
        got = _expand(t, ls.pp_src[pp], ls.pp_img[pp]) + _expand(t, ls.pc_src[pc], ls.pc_img[pc])
        assert sorted(got) == allpairs
        msum = t.mom[ls.pp_src[pp], 0].sum() + t.mom[ls.pc_src[pc], 0].sum()
        assert np.isclose(msum, nimg * mtot, rtol=1e-12)
        # PP sources are leaves; the sink's own bucket is on its PP list at image 0
        assert np.all(t.child[ls.pp_src[pp], 0] < 0)
        own = t.bucket_cell[b]
        assert np.any((ls.pp_src[pp] == own) & (ls.pp_img[pp] == 0))


def _criterion(t, c, img, s, theta, eps, L):
    sh = oracle.image_shift(img, L)
    d = np.sqrt(((t.com[c] + sh - t.com[s]) ** 2).sum())
    clo, chi = t.bbox[c, :3] + sh, t.bbox[c, 3:] + sh
    slo, shi = t.bbox[s, :3], t.bbox[s, 3:]
    gap = np.maximum(0, np.maximum(clo - shi, slo - chi))
    return d > t.bmax[c] / theta + t.bmax[s] and np.sqrt((gap ** 2).sum()) >= 2 * eps


def test_lists_obey_acceptance_rule(small_sets):
    ps = small_sets[2]
    theta = 0.7
    t = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    ls = oracle.build_lists(t, theta, ps.eps)
    parent = np.full(t.n_cell, -1)
    for c in range(t.n_cell):
        if t.child[c, 0] >= 0:
            parent[t.child[c]] = c
    for b in range(0, t.n_bucket, 7):
        s = t.bucket_cell[b]
        for e in range(ls.pc_off[b], ls.pc_off[b + 1]):
            c, i = ls.pc_src[e], ls.pc_img[e]
            assert _criterion(t, c, i, s, theta, ps.eps, ps.box_L)
            if parent[c] >= 0:  # it was reached by opening a cell that failed
                assert not _criterion(t, parent[c], i, s, theta, ps.eps, ps.box_L)
        for e in range(ls.pp_off[b], ls.pp_off[b + 1]):
            c, i = ls.pp_src[e], ls.pp_img[e]
            assert not _criterion(t, c, i, s, theta, ps.eps, ps.box_L)


# ------------------------------------------------------------------ PP ----

def test_pp_two_body_closed_form():
    eps = 0.05
    pos = np.array([[0.1, -0.2, 0.3], [0.4, 0.5, -0.6]])
    m = np.array([0.3, 0.7])
    acc, pot = oracle.direct_open(pos, m, eps)
    r = pos[0] - pos[1]
    D = r @ r + eps * eps
    assert np.allclose(acc[0], -m[1] * r / D ** 1.5, rtol=1e-15, atol=0)
    assert np.allclose(acc[1], m[0] * r / D ** 1.5, rtol=1e-15, atol=0)
    assert np.isclose(pot[0], -m[1] / math.sqrt(D), rtol=1e-15)


def test_direct_sum_conserves_momentum():
    ps = workloads.plummer(1024, seed=3)
    acc, _ = oracle.direct_open(ps.pos, ps.mass, ps.eps)
    ptot = (ps.mass[:, None] * acc).sum(0)
    assert np.abs(ptot).max() < 1e-14 * np.abs(ps.mass[:, None] * acc).sum()


def test_tree_reproduces_direct_sum_as_theta_goes_to_zero():
    ps = workloads.plummer(1024, seed=4)
    tree, lists, acc, pot = oracle.forces(ps, theta=1e-7)
    ad, pd = oracle.direct_open(ps.pos, ps.mass, ps.eps)
    assert np.abs(acc - ad[tree.perm]).max() < 1e-12
    assert np.abs(pot - pd[tree.perm]).max() < 1e-12


# ------------------------------------------------------------------ PC ----

def test_pc_single_particle_cell_equals_pp():
    x0 = np.array([[0.3, -0.1, 0.2]])
    com, mom = oracle.moments(x0, np.array([0.5]))
    assert np.all(mom[1:] == 0.0)
    x = np.array([1.1, 0.4, -0.7])
    eps = 0.02
    out = oracle.pc_point(mom, com, x, eps)
    r = x - x0[0]
    D = r @ r + eps * eps
    assert np.allclose(out[:3], -0.5 * r / D ** 1.5, rtol=1e-14, atol=0)
    assert np.isclose(out[3], -0.5 / math.sqrt(D), rtol=1e-14)


def test_pc_two_particle_axis_closed_form():
    # Two masses m at +-s on the x axis; on the axis at distance R the
    # Newtonian potential is -(2m/R) sum_k (s/R)^(2k); order-4 moments keep
    # k = 0, 1, 2 exactly, and the force is its R-derivative.
    m, s, R = 0.25, 0.1, 0.9
    pos = np.array([[s, 0, 0], [-s, 0, 0]])
    com, mom = oracle.moments(pos, np.array([m, m]))
    out = oracle.pc_point(mom, com, np.array([R, 0, 0]), 0.0)
    u = s / R
    assert np.isclose(out[3], -(2 * m / R) * (1 + u ** 2 + u ** 4), rtol=1e-14)
    assert np.isclose(out[0], -(2 * m / R ** 2) * (1 + 3 * u ** 2 + 5 * u ** 4), rtol=1e-14)
    assert abs(out[1]) < 1e-16 and abs(out[2]) < 1e-16


def test_pc_error_decays_as_fifth_power():
    # Order-4 moments: the first neglected term is order 5, so the relative
    # error of both force and potential falls as (b/R)^5.
    rng = np.random.default_rng(7)
    pts = rng.normal(size=(25, 3)) * 0.1
    m = rng.uniform(0.5, 1.5, size=25)
    com, mom = oracle.moments(pts, m)
    direction = np.array([0.48, -0.6, 0.64])
    Rs = np.array([1.0, 1.4, 2.0, 2.8, 4.0])
    ea, ep = [], []
    for R in Rs:
        x = com + R * direction
        out = oracle.pc_point(mom, com, x, 1e-6)
        r = x - pts
        D = (r ** 2).sum(1) + 1e-12
        a_ex = -(m[:, None] * r / D[:, None] ** 1.5).sum(0)
        p_ex = -(m / np.sqrt(D)).sum()
        ea.append(np.linalg.norm(out[:3] - a_ex) / np.linalg.norm(a_ex))
        ep.append(abs(out[3] - p_ex) / abs(p_ex))
    sa = np.polyfit(np.log(Rs), np.log(ea), 1)[0]
    sp = np.polyfit(np.log(Rs), np.log(ep), 1)[0]
    assert -5.3 < sa < -4.7, sa
    assert -5.3 < sp < -4.7, sp


def test_pc_translation_and_rotation():
    rng = np.random.default_rng(8)
    pts = rng.normal(size=(10, 3)) * 0.1
    m = rng.uniform(0.5, 1.5, size=10)
    x = np.array([0.7, -0.5, 0.9])
    com, mom = oracle.moments(pts, m)
    ref = oracle.pc_point(mom, com, x, 0.01)
    shift = np.array([3.0, -2.0, 5.0])
    com2, mom2 = oracle.moments(pts + shift, m)
    out2 = oracle.pc_point(mom2, com2, x + shift, 0.01)
    assert np.allclose(out2, ref, rtol=1e-10, atol=1e-14)
    # 90-degree rotation about z: (x, y, z) -> (-y, x, z)
    rot = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], float)
    com3, mom3 = oracle.moments(pts @ rot.T, m)
    out3 = oracle.pc_point(mom3, com3, rot @ x, 0.01)
    assert np.allclose(out3[:3], rot @ ref[:3], rtol=1e-12, atol=1e-15)
    assert np.isclose(out3[3], ref[3], rtol=1e-12)


# ------------------------------------------------- method vs direct sum ----

def test_method_error_decreases_with_theta_and_meets_accuracy_regime():
    ps = workloads.plummer(2048, seed=1)
    ad, _ = oracle.direct_open(ps.pos, ps.mass, ps.eps)
    errs = []
    for th in (0.9, 0.7, 0.5, 0.3):
        tree, _, acc, _ = oracle.forces(ps, theta=th)
        errs.append(_rel_rms(acc, ad[tree.perm]))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    # Sec. 3.1 / 4.2: theta = 0.7 with order-4 moments is in the
    # "better than 0.1% RMS" regime.
    assert errs[1] < 2e-3, errs


def test_plummer_radial_acceleration_matches_enclosed_mass():
    ps = workloads.plummer(8192)
    tree, _, acc, _ = oracle.forces(ps, theta=0.5)
    pos = ps.pos[tree.perm]
    r = np.sqrt((pos ** 2).sum(1))
    ar = -(acc * pos).sum(1) / r
    ftrunc = workloads.PLUMMER_TRUNC_FRAC
    for lo, hi in [(0.3, 0.45), (0.6, 0.8), (1.0, 1.3), (1.8, 2.4)]:
        sel = (r > lo) & (r < hi)
        rc = np.sqrt(lo * hi)
        menc = rc ** 3 / (1 + rc ** 2) ** 1.5 / ftrunc
        ncount = menc * ps.n
        model = np.mean(((r[sel] ** 3 / (1 + r[sel] ** 2) ** 1.5) / ftrunc) / r[sel] ** 2)
        got = np.mean(ar[sel])
        assert abs(got / model - 1) < 3.0 / math.sqrt(ncount) + 0.01, (lo, got, model)


# --------------------------------------------------------------- Ewald ----

def test_ewald_psi_at_origin_is_lattice_constant():
    psi0 = XI + 6 + 12 / math.sqrt(2) + 8 / math.sqrt(3)
    for alpha, rmax, h2 in [(1.5, 3, 40), (2.0, 3, 48), (2.6, 3, 80)]:
        d = oracle.ewald_derivs(np.zeros(3), alpha, rmax, h2, 1)
        assert abs(d[0] - psi0) < 1e-11
        assert np.abs(d[1]).max() < 1e-14


def test_ewald_alpha_independence():
    for r in ([0.1, 0.2, 0.3], [0.45, -0.3, 0.05], [0.8, 0.7, -0.6]):
        v = [oracle.ewald_derivs(np.array(r), a, 3, 80, 3) for a in (1.6, 2.2, 2.8)]
        for k in range(4):
            ref = np.asarray(v[0][k])
            for w in v[1:]:
                assert np.abs(np.asarray(w[k]) - ref).max() < 1e-9 * (1 + np.abs(ref).max())


def test_ewald_laplacian_and_finite_differences():
    rng = np.random.default_rng(5)
    for _ in range(3):
        r = rng.uniform(-0.6, 0.6, size=3)
        d = oracle.ewald_derivs(r, 2.0, 3, 48, 5)
        # the 27 near images are harmonic; the rest carries the background
        assert abs(np.trace(d[2]) + 4 * math.pi) < 1e-10
        h = 1e-4
        for b in range(3):
            e = np.zeros(3)
            e[b] = h
            dp = oracle.ewald_derivs(r + e, 2.0, 3, 48, 5)
            dm = oracle.ewald_derivs(r - e, 2.0, 3, 48, 5)
            for k in range(5):
                fd = (np.asarray(dp[k]) - np.asarray(dm[k])) / (2 * h)
                an = np.asarray(d[k + 1])[..., b]
                assert np.abs(fd - an).max() < 1e-5 * (1 + np.abs(an).max()), (k, b)


def test_ewald_symmetries():
    r = np.array([0.31, -0.17, 0.44])
    base = oracle.ewald_derivs(r, 2.0, 3, 48, 1)
    for flip in ([-1, 1, 1], [1, -1, 1], [1, 1, -1]):
        f = np.array(flip, float)
        d = oracle.ewald_derivs(r * f, 2.0, 3, 48, 1)
        assert abs(d[0] - base[0]) < 1e-12
        assert np.allclose(d[1], base[1] * f, atol=1e-12)
    d = oracle.ewald_derivs(r[[2, 0, 1]], 2.0, 3, 48, 1)
    assert abs(d[0] - base[0]) < 1e-12
    assert np.allclose(d[1], base[1][[2, 0, 1]], atol=1e-12)


def test_periodic_force_vanishes_on_half_box_plane():
    # Full periodic potential of one mass: phi_per = psi - sum_{N1} 1/|r - n|.
    # By the mirror symmetry about x = 1/2 its x-derivative is zero there.
    for y, z in [(0.1, 0.3), (-0.4, 0.2)]:
        r = np.array([0.5, y, z])
        d = oracle.ewald_derivs(r, 2.0, 3, 48, 1)
        gx = d[1][0]
        for ix in (-1, 0, 1):
            for iy in (-1, 0, 1):
                for iz in (-1, 0, 1):
                    v = r - np.array([ix, iy, iz])
                    gx += v[0] / np.linalg.norm(v) ** 3
        assert abs(gx) < 1e-11


def test_ewald_quadrature_converged():
    r = np.array([0.2, -0.35, 0.4])
    oracle.set_quadrature(128)
    a = oracle.ewald_derivs(r, 2.6, 2, 10, 5)
    oracle.set_quadrature(256)
    b = oracle.ewald_derivs(r, 2.6, 2, 10, 5)
    oracle.set_quadrature(128)
    for k in range(6):
        assert np.abs(np.asarray(a[k]) - np.asarray(b[k])).max() < 1e-11 * (
            1 + np.abs(np.asarray(b[k])).max())


def test_direct_periodic_sum_on_cubic_lattice_gives_lattice_constant():
    # n^3 equal masses 1/n^3 on a cubic lattice form a simple-cubic lattice of
    # spacing 1/n: by scaling, each feels zero force and the potential
    # (self singularity excluded) XI * m / spacing = XI / n^2.
    n1d = 3
    ps = workloads.perturbed_lattice(n1d, 0.0, eps=1e-9)
    acc, pot = oracle.direct_periodic(ps.pos, ps.mass, ps.eps, 1.0)
    assert np.abs(acc).max() < 1e-11
    assert np.allclose(pot, XI / n1d ** 2, rtol=0, atol=1e-10)


def test_ewald_root_expansion_converges_as_fifth_power():
    # Root-multipole Ewald correction of a compact two-mass source vs the
    # pairwise kernel: order-4 moments leave an O(s^5) remainder.
    x = np.array([0.23, -0.11, 0.37])
    errs, ss = [], np.array([0.05, 0.07, 0.1, 0.14])
    for s in ss:
        pts = np.array([[s, 0.3 * s, -0.2 * s], [-0.6 * s, -0.2 * s, 0.5 * s], [0.1 * s, -s, 0.2 * s]])
        m = np.array([1.0, 1.5, 0.7])
        com, mom = oracle.moments(pts, m)
        out = oracle.ewald_root_point(mom, com, x, 1.0, 2.0, 3, 48)
        ex = np.zeros(3)
        for j in range(3):
            d = oracle.ewald_derivs(x - pts[j], 2.0, 3, 48, 1)
            ex -= m[j] * d[1]
        errs.append(np.linalg.norm(out[:3] - ex) / np.linalg.norm(ex))
    slope = np.polyfit(np.log(ss), np.log(errs), 1)[0]
    assert 4.6 < slope < 5.4, (slope, errs)


def test_periodic_tree_matches_direct_sum_within_expansion_error():
    ps = workloads.perturbed_lattice(4, 0.2, seed=9)
    ad, pd = oracle.direct_periodic(ps.pos, ps.mass, ps.eps, 1.0)
    tree, _, acc, pot = oracle.forces(ps, theta=1e-7, ewald=oracle.CONVERGED_EWALD)
    # theta -> 0 leaves only the root-expansion error of the Ewald term
    assert _rel_rms(acc, ad[tree.perm]) < 3e-3
    momentum = (ps.mass[tree.perm, None] * acc).sum(0)
    assert np.abs(momentum).max() < 1e-3 * np.abs(acc).mean()


# ------------------------------------------- softened PC, orders >= 2 ----

@pytest.mark.parametrize("eps_over_R", [0.5, 1.0])
def test_softened_pc_error_decays_as_fifth_power_of_cell_size(eps_over_R):
    # Sec. 3.1 expands the softened Green's function about the cell's centre
    # of mass.  With the softening comparable to the distance (eps = 0.5 R
    # and eps = R), shrinking the cell at fixed R and eps must leave an
    # order-5 remainder against the direct softened sum: the relative error
    # falls as b^5.  If eps^2 were missing from the radial derivatives of any
    # order >= 2, the expansion would approximate a different function and
    # the error would stall at O(b^2) instead.
    rng = np.random.default_rng(71)
    base = rng.normal(size=(25, 3))
    m = rng.uniform(0.5, 1.5, size=25)
    R, eps = 1.0, eps_over_R * 1.0
    direction = np.array([0.48, -0.6, 0.64])
    # small enough that the order-6 remainder is a few per cent of the
    # order-5 one (the potential's order-5 term is the smaller at eps = R)
    bs = np.array([0.01, 0.014, 0.02, 0.028, 0.04])
    ea, ep = [], []
    for b in bs:
        pts = b * base
        com, mom = oracle.moments(pts, m)
        x = com + R * direction
        out = oracle.pc_point(mom, com, x, eps)
        r = x - pts
        D = (r ** 2).sum(1) + eps * eps
        a_ex = -(m[:, None] * r / D[:, None] ** 1.5).sum(0)
        p_ex = -(m / np.sqrt(D)).sum()
        ea.append(np.linalg.norm(out[:3] - a_ex) / np.linalg.norm(a_ex))
        ep.append(abs(out[3] - p_ex) / abs(p_ex))
    sa = np.polyfit(np.log(bs), np.log(ea), 1)[0]
    sp = np.polyfit(np.log(bs), np.log(ep), 1)[0]
    assert 4.7 < sa < 5.3, (sa, ea)
    assert 4.7 < sp < 5.3, (sp, ep)


def test_softened_pc_quadrupole_closed_form():
    # Two masses m at +-s on the x axis seen from (0, R, 0) with Plummer
    # softening: the exact potential is -2m (R^2 + s^2 + eps^2)^(-1/2);
    # expanded in s^2 its first two terms are -2m/S (1 - s^2/(2 S^2)),
    # S^2 = R^2 + eps^2.  The order-4 moments reproduce the expansion
    # through s^4: -2m/S (1 - s^2/(2S^2) + 3 s^4/(8 S^4)).
    m, s, R, eps = 0.25, 0.05, 0.6, 0.45
    pos = np.array([[s, 0, 0], [-s, 0, 0]])
    com, mom = oracle.moments(pos, np.array([m, m]))
    out = oracle.pc_point(mom, com, np.array([0.0, R, 0.0]), eps)
    S2 = R * R + eps * eps
    u = s * s / S2
    expect_phi = -2 * m / math.sqrt(S2) * (1 - u / 2 + 3 * u * u / 8)
    # d/dR of -2m (S^2 + s^2)^(-1/2) is 2m R (S^2+s^2)^(-3/2); its series
    # through s^4 is 2m R / S^3 (1 - 3u/2 + 15 u^2/8), and acc = -grad phi
    expect_ay = -2 * m * R / S2 ** 1.5 * (1 - 1.5 * u + 15 * u * u / 8)
    assert np.isclose(out[3], expect_phi, rtol=1e-13)
    assert np.isclose(out[1], expect_ay, rtol=1e-13)
    assert abs(out[0]) < 1e-16 and abs(out[2]) < 1e-16


# ------------------------------------------------------ box side L != 1 ----

def _scaled_lattice(L):
    ps = workloads.perturbed_lattice(4, 0.2, seed=9)
    return ps.pos * L, ps.mass, ps.eps * L


def test_direct_periodic_sum_scales_with_box_side():
    # Gravity has no intrinsic length: scaling positions, softening and the
    # box by L leaves the masses' field self-similar, with accelerations
    # times 1/L^2 and potentials times 1/L.
    L = 2.5
    p1, m, e1 = _scaled_lattice(1.0)
    pL, _, eL = _scaled_lattice(L)
    a1, q1 = oracle.direct_periodic(p1, m, e1, 1.0)
    aL, qL = oracle.direct_periodic(pL, m, eL, L)
    assert np.allclose(aL * L * L, a1, rtol=1e-11, atol=1e-11 * np.abs(a1).max())
    assert np.allclose(qL * L, q1, rtol=1e-11, atol=1e-11 * np.abs(q1).max())


def test_tree_method_with_ewald_scales_with_box_side():
    # The same scaling through the whole oracle path: tree, lists (the
    # acceptance rule compares lengths only), PP, PC and the root-multipole
    # Ewald correction with its powers of L.
    L = 2.5
    p1, m, e1 = _scaled_lattice(1.0)
    pL, _, eL = _scaled_lattice(L)
    t1 = oracle.build_tree(p1, m, 1.0, 16)
    tL = oracle.build_tree(pL, m, L, 16)
    assert np.array_equal(t1.perm, tL.perm) and np.array_equal(t1.child, tL.child)
    l1 = oracle.build_lists(t1, 0.7, e1)
    lL = oracle.build_lists(tL, 0.7, eL)
    for f in ("pp_off", "pp_src", "pp_img", "pc_off", "pc_src", "pc_img"):
        assert np.array_equal(getattr(l1, f), getattr(lL, f)), f
    assert np.allclose(tL.mom[:, 1:7] / L ** 2, t1.mom[:, 1:7], rtol=1e-12, atol=1e-18)
    a1, q1 = oracle.evaluate(t1, l1, p1[t1.perm], m[t1.perm], e1, 7)
    aL, qL = oracle.evaluate(tL, lL, pL[tL.perm], m[tL.perm], eL, 7)
    assert np.allclose(aL * L * L, a1, rtol=1e-10, atol=1e-10 * np.abs(a1).max())
    assert np.allclose(qL * L, q1, rtol=1e-10, atol=1e-10 * np.abs(q1).max())
    # the Ewald part alone, where the powers L^-(1+k) and L^-(2+k) act
    e1a, e1q = oracle.evaluate(t1, l1, p1[t1.perm], m[t1.perm], e1, 4)
    eLa, eLq = oracle.evaluate(tL, lL, pL[tL.perm], m[tL.perm], eL, 4)
    assert np.allclose(eLa * L * L, e1a, rtol=1e-10, atol=1e-12 * np.abs(e1a).max())
    assert np.allclose(eLq * L, e1q, rtol=1e-10)


def test_ewald_root_point_scales_with_box_side():
    # one compact source of order-4 moments, seen at the same scaled offset
    rng = np.random.default_rng(72)
    pts = rng.normal(size=(6, 3)) * 0.08
    m = rng.uniform(0.5, 1.5, size=6)
    x = np.array([0.23, -0.11, 0.37])
    com, mom = oracle.moments(pts, m)
    ref = oracle.ewald_root_point(mom, com, x, 1.0, 2.6, 1, 10)
    for L in (0.4, 2.5, 7.0):
        comL, momL = oracle.moments(pts * L, m)
        out = oracle.ewald_root_point(momL, comL, x * L, L, 2.6, 1, 10)
        assert np.allclose(out[:3] * L * L, ref[:3], rtol=1e-11, atol=1e-13)
        assert np.isclose(out[3] * L, ref[3], rtol=1e-11)
