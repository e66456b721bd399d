"""Seeded synthetic particle sets for the five benchmark configurations.

This module only draws random numbers and lays out particle arrays: it
holds none of the gravity method's arithmetic (no forces, no tree, no
multipoles).  Both the oracle-based tests and the GPU path consume these
arrays, so nothing here may depend on either of them.

The paper measures on cosmological LCDM initial conditions and snapshots
(its Sections 4.2-4.7); those are not available, so the generators below
stand in for them with the shapes the configurations fix:

* ``plummer``            -- isotropic Plummer sphere (open boundary),
* ``perturbed_lattice``  -- a unit periodic box of lattice points with
                            Gaussian displacements (early, near-homogeneous
                            universe),
* ``clustered``          -- uniform background plus Plummer haloes with a
                            power-law mass function (late, clustered
                            universe).

Softening follows Section 3.1: one fiftieth of the mean inter-particle
separation, eps = L / (50 N^(1/3)).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

BASE_SEED = 20160928

# Mass fraction of an untruncated Plummer sphere inside 10 scale radii:
# M(<r)/M = r^3 / (1 + r^2)^(3/2) at r = 10.
PLUMMER_TRUNC_FRAC = 1000.0 / 101.0 ** 1.5


@dataclasses.dataclass
class ParticleSet:
    """Particles in input order.

    pos   : float64 [n, 3]   positions (periodic sets wrapped into [0, L))
    mass  : float64 [n]
    eps   : Plummer softening length
    box_L : periodic box side, 0.0 for open boundaries
    """

    pos: np.ndarray
    mass: np.ndarray
    eps: float
    box_L: float
    name: str = ""
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _plummer_radii(rng: np.random.Generator, count: int, a: float,
                   rmax_over_a: float = 10.0) -> np.ndarray:
    """Radii distributed as a Plummer sphere truncated at ``rmax_over_a * a``.

    Inverse CDF of the enclosed-mass fraction u = r^3/(1+r^2)^(3/2) (r in
    units of a): r^2 = u^(2/3) / (1 - u^(2/3)).
    """
    umax = rmax_over_a ** 3 / (1.0 + rmax_over_a ** 2) ** 1.5
    u = rng.uniform(0.0, umax, size=count)
    u23 = u ** (2.0 / 3.0)
    return a * np.sqrt(u23 / (1.0 - u23))


def _isotropic(rng: np.random.Generator, count: int) -> np.ndarray:
    cz = rng.uniform(-1.0, 1.0, size=count)
    ph = rng.uniform(0.0, 2.0 * math.pi, size=count)
    sz = np.sqrt(np.maximum(0.0, 1.0 - cz * cz))
    return np.stack([sz * np.cos(ph), sz * np.sin(ph), cz], axis=1)


def plummer(n: int = 8192, seed: int = BASE_SEED + 1, a: float = 1.0,
            eps: float = 0.01, fp32_positions: bool = True) -> ParticleSet:
    """Plummer sphere of total mass 1 (masses 1/n), open boundary.

    With ``fp32_positions`` the positions are rounded to float32 and then
    widened back to float64, so every consumer sees exactly the same values.
    """
    rng = np.random.default_rng(seed)
    r = _plummer_radii(rng, n, a)
    pos = r[:, None] * _isotropic(rng, n)
    if fp32_positions:
        pos = pos.astype(np.float32).astype(np.float64)
    mass = np.full(n, 1.0 / n)
    return ParticleSet(pos, mass, eps, 0.0, "plummer", seed)


def perturbed_lattice(n1d: int = 64, sigma_frac: float = 0.2,
                      seed: int = BASE_SEED + 2, L: float = 1.0,
                      eps: Optional[float] = None) -> ParticleSet:
    """n1d^3 lattice in a periodic box of side L, cell-centred points plus
    Gaussian displacements of ``sigma_frac`` lattice spacings per axis,
    wrapped into [0, L).  ``sigma_frac = 0`` gives the unperturbed lattice,
    on which the exact periodic force vanishes by symmetry."""
    rng = np.random.default_rng(seed)
    h = L / n1d
    g = (np.arange(n1d) + 0.5) * h
    gx, gy, gz = np.meshgrid(g, g, g, indexing="ij")
    pos = np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)
    if sigma_frac > 0:
        pos = pos + rng.normal(0.0, sigma_frac * h, size=pos.shape)
    pos = np.mod(pos, L)
    pos[pos >= L] = 0.0  # mod can return L for tiny negative inputs
    n = pos.shape[0]
    mass = np.full(n, 1.0 / n)
    if eps is None:
        eps = L / (50.0 * n1d)
    return ParticleSet(pos, mass, eps, L, "lattice", seed)


def halo_counts(n_halo_particles: int, n_halos: int, rng: np.random.Generator,
                slope: float = -1.9, decades: float = 2.0):
    """Particle counts per halo: masses drawn from dN/dM ~ M^slope over
    [1, 10^decades] by inverse CDF, counts proportional to mass with the
    largest-remainder rule so they sum exactly to ``n_halo_particles``."""
    k = slope + 1.0
    u = rng.uniform(0.0, 1.0, size=n_halos)
    lo, hi = 1.0, 10.0 ** decades
    masses = (lo ** k + u * (hi ** k - lo ** k)) ** (1.0 / k)
    share = masses / masses.sum() * n_halo_particles
    counts = np.floor(share).astype(np.int64)
    rem = n_halo_particles - int(counts.sum())
    order = np.argsort(-(share - counts), kind="stable")
    counts[order[:rem]] += 1
    return counts, masses


def clustered(n1d: int = 128, n_halos: int = 500, seed: int = BASE_SEED + 3,
              L: float = 1.0, background_frac: float = 0.3,
              a_max: float = 0.005, eps: Optional[float] = None) -> ParticleSet:
    """Uniform background (``background_frac`` of the particles) plus Plummer
    haloes: masses from a M^-1.9 power law over two decades, radii
    a_h = a_max * L * (M_h / M_max)^(1/3), truncated at 10 a_h, centres
    uniform in the box, everything wrapped into [0, L)."""
    rng = np.random.default_rng(seed)
    n = n1d ** 3
    n_bg = int(round(background_frac * n))
    n_h = n - n_bg
    counts, masses = halo_counts(n_h, n_halos, rng)
    bg = rng.uniform(0.0, L, size=(n_bg, 3))
    centres = rng.uniform(0.0, L, size=(n_halos, 3))
    a_h = a_max * L * (masses / masses.max()) ** (1.0 / 3.0)
    parts = [bg]
    for h in range(n_halos):
        c = int(counts[h])
        if c == 0:
            continue
        r = _plummer_radii(rng, c, a_h[h])
        parts.append(centres[h] + r[:, None] * _isotropic(rng, c))
    pos = np.mod(np.concatenate(parts, axis=0), L)
    pos[pos >= L] = 0.0
    mass = np.full(n, 1.0 / n)
    if eps is None:
        eps = L / (50.0 * n1d)
    return ParticleSet(pos, mass, eps, L, "clustered", seed)


def active_by_acceleration(acc_mag: np.ndarray, fraction: float) -> np.ndarray:
    """Active mask for an individual-time-step substep.

    With the time-step criterion dt_i = 0.2 sqrt(eps / |a_i|) (Section 3.2)
    the deepest rungs hold the particles with the largest |a_i|; the active
    set of a substep that touches a ``fraction`` of the particles is taken as
    that many particles with the largest |a_i| (ties broken by index).
    Returns uint8 [n]."""
    n = acc_mag.shape[0]
    k = int(round(fraction * n))
    mask = np.zeros(n, dtype=np.uint8)
    if k >= n:
        mask[:] = 1
        return mask
    if k <= 0:
        return mask
    order = np.argsort(-acc_mag, kind="stable")
    mask[order[:k]] = 1
    return mask


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    theta: float
    bucket: int
    ewald: str  # "none" | "exact" | "surrogate"


CONFIGS = {
    1: Config("plummer_8192_open", 0.7, 16, "none"),
    2: Config("lattice_64cubed_periodic", 0.7, 16, "exact"),
    3: Config("clustered_128cubed_periodic", 0.7, 16, "exact"),
    4: Config("lattice_256cubed_periodic", 0.7, 16, "surrogate"),
    5: Config("clustered_512cubed_periodic", 0.7, 16, "surrogate"),
}


def make(config: int, scale_n1d: Optional[int] = None) -> ParticleSet:
    """Particle set of a benchmark configuration.  ``scale_n1d`` shrinks the
    periodic configurations to scale_n1d^3 particles (same recipe, softening
    rescaled with the mean separation) for tests that must stay small."""
    if config == 1:
        return plummer(8192 if scale_n1d is None else scale_n1d ** 3)
    if config == 2:
        return perturbed_lattice(64 if scale_n1d is None else scale_n1d, 0.2,
                                 BASE_SEED + 2)
    if config == 3:
        n1d = 128 if scale_n1d is None else scale_n1d
        halos = 500 if scale_n1d is None else max(4, 500 * n1d ** 3 // 128 ** 3)
        return clustered(n1d, halos, BASE_SEED + 3)
    if config == 4:
        return perturbed_lattice(256 if scale_n1d is None else scale_n1d, 0.3,
                                 BASE_SEED + 4)
    if config == 5:
        n1d = 512 if scale_n1d is None else scale_n1d
        halos = 32000 if scale_n1d is None else max(4, 32000 * n1d ** 3 // 512 ** 3)
        return clustered(n1d, halos, BASE_SEED + 5, a_max=0.005 / 4.0)
    raise ValueError(f"unknown configuration {config}")


# Layer shapes of the Ewald-surrogate network (3 -> 128 -> 128 -> 128 -> 4),
# in the order of its flat parameter vector.
MLP_SHAPES = [(128, 3), (128,), (128, 128), (128,), (128, 128), (128,), (4, 128), (4,)]


def mlp_init(seed: int = BASE_SEED + 10) -> np.ndarray:
    """Initial parameters of the surrogate network (float64, flat): weights
    uniform in +-1/sqrt(fan_in), biases zero.  Drawn here so the GPU
    trainer and its reference start from the same numbers."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in MLP_SHAPES:
        if len(shp) == 2:
            b = 1.0 / math.sqrt(shp[1])
            parts.append(rng.uniform(-b, b, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts)


def octant_points(n: int, seed: int = BASE_SEED + 11) -> np.ndarray:
    """Uniform sample points u in the fundamental octant [0, 1)^3 of the
    unit box, where the Ewald surrogate is trained (float64 [n, 3])."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, size=(n, 3))
