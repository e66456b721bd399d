"""Pins of the seeded input generators (workloads/): the sizes, ranges and
distributions the benchmark configurations state.  CPU only."""
import numpy as np

import workloads


def test_perturbed_lattice_recipe():
    ps0 = workloads.perturbed_lattice(8, 0.0)
    h = 1.0 / 8
    g = (np.arange(8) + 0.5) * h
    assert ps0.n == 512 and np.allclose(np.unique(ps0.pos[:, 0]), g)  # cell centres
    ps = workloads.perturbed_lattice(32, 0.2, seed=3)
    assert ps.n == 32 ** 3 and ps.box_L == 1.0
    assert np.all((ps.pos >= 0) & (ps.pos < 1))
    assert np.isclose(ps.mass.sum(), 1.0) and np.all(ps.mass == ps.mass[0])
    assert np.isclose(ps.eps, 1.0 / (50 * 32))
    # displacement from the nearest cell centre: Gaussian with sigma 0.2 h per axis
    h = 1.0 / 32
    d = ps.pos - ((np.floor(ps.pos / h) + 0.5) * h)
    sd = np.std(d)
    assert abs(sd - 0.2 * h) < 0.03 * 0.2 * h


def test_halo_mass_function():
    rng = np.random.default_rng(7)
    counts, masses = workloads.halo_counts(1_000_000, 32000, rng)
    assert counts.sum() == 1_000_000 and np.all(counts >= 0)
    assert masses.min() >= 1.0 and masses.max() <= 100.0
    # dN/dM ~ M^-1.9 over two decades: P(M < 10) = (10^-0.9 - 1) / (100^-0.9 - 1)
    want = (10 ** -0.9 - 1) / (100 ** -0.9 - 1)
    assert abs(np.mean(masses < 10.0) - want) < 0.01
    # counts proportional to mass (largest remainder: within one particle)
    share = masses / masses.sum() * 1_000_000
    assert np.all(np.abs(counts - share) < 1.0)


def test_clustered_recipe():
    ps = workloads.clustered(24, 40, seed=5)
    n = 24 ** 3
    assert ps.n == n and ps.box_L == 1.0 and np.isclose(ps.eps, 1.0 / (50 * 24))
    assert np.all((ps.pos >= 0) & (ps.pos < 1)) and np.isclose(ps.mass.sum(), 1.0)
    # 30 % uniform background, 70 % in haloes: the densest 1 % of 32^3 grid
    # cells hold far more than 1 % of the particles
    k = np.floor(ps.pos * 32).astype(int)
    occ = np.bincount((k[:, 0] * 32 + k[:, 1]) * 32 + k[:, 2], minlength=32 ** 3)
    top = np.sort(occ)[::-1][: 32 ** 3 // 100].sum() / n
    assert top > 0.3
    # the same seed gives the same set
    assert np.array_equal(workloads.clustered(24, 40, seed=5).pos, ps.pos)


def test_config_shapes_and_active_sets():
    assert workloads.make(3, scale_n1d=16).n == 16 ** 3
    assert workloads.make(5, scale_n1d=16).n == 16 ** 3
    a = np.array([3.0, 1.0, 3.0, 2.0, 0.5, 3.0])
    m = workloads.active_by_acceleration(a, 0.5)
    assert m.dtype == np.uint8 and m.sum() == 3
    assert set(np.flatnonzero(m)) == {0, 2, 5}  # the largest |a|
    assert workloads.active_by_acceleration(a, 0.0).sum() == 0
    assert workloads.active_by_acceleration(a, 1.0).sum() == 6


def test_plummer_recipe():
    ps = workloads.make(1)
    assert ps.n == 8192 and ps.box_L == 0.0 and ps.eps == 0.01
    assert np.allclose(ps.mass, 1.0 / 8192)
    # positions are float32 values
    assert np.array_equal(ps.pos, ps.pos.astype(np.float32).astype(np.float64))
    r = np.linalg.norm(ps.pos, axis=1)
    assert r.max() <= 10.0 * (1 + 1e-6)
    # enclosed-mass fraction of a Plummer sphere truncated at 10 a:
    # M(<r) = r^3 / (1 + r^2)^(3/2), normalised by M(<10)
    m10 = 1000.0 / 101.0 ** 1.5
    for rr in (0.5, 1.0, 2.0, 5.0):
        want = rr ** 3 / (1 + rr * rr) ** 1.5 / m10
        assert abs(np.mean(r < rr) - want) < 0.02
    # isotropic: centre of mass near the origin, equal second moments
    assert np.all(np.abs(ps.pos.mean(0)) < 0.1)
    m2 = (ps.pos ** 2).mean(0)
    assert np.all(np.abs(m2 / m2.mean() - 1) < 0.15)


def test_clustered_halo_radii_scale_with_config():
    # the 512^3 recipe has haloes a quarter the size of the 128^3 one: the
    # same scaled-down set is more concentrated
    a = workloads.clustered(24, 40, seed=5)
    b = workloads.clustered(24, 40, seed=5, a_max=0.005 / 4.0)
    def top_share(ps):
        k = np.floor(ps.pos * 64).astype(int)
        occ = np.bincount((k[:, 0] * 64 + k[:, 1]) * 64 + k[:, 2], minlength=64 ** 3)
        return np.sort(occ)[::-1][:64 ** 3 // 1000].sum() / ps.n
    assert top_share(b) > top_share(a)
