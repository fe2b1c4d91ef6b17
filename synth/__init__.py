"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws inputs: particle positions, masses, smoothing lengths and
ray positions.  It contains none of the lensing arithmetic (no deflection, no
tree), so the GPU path and the CPU oracle can both consume its arrays without
sharing any computation.

The workloads follow the paper's synthetic lenses: random point masses in a
region (Sec. 5.1), smoothed simulation particles whose smoothing length is the
distance to the N_sph-th neighbour (Sec. 3.1), and stars with a mass function
implanted near an image (Sec. 3.5).  All draws use numpy's PCG64 generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 11281312


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# --------------------------------------------------------------------------
# ray sets
# --------------------------------------------------------------------------
def ray_grid(n: int, lo: float = -0.5, hi: float = 0.5):
    """n x n cell-centred grid over [lo, hi]^2, row-major with x fastest."""
    h = (hi - lo) / n
    c = lo + (np.arange(n, dtype=np.float64) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="xy")
    return X.ravel().copy(), Y.ravel().copy()


def ray_grid_tiled(n: int, lo: float = -0.5, hi: float = 0.5):
    """The same n x n cell-centred grid, listed in Z (Morton) order of the grid
    indices -- a storage order in which every 64 consecutive rays form an 8x8
    tile (n a power of two)."""
    i = np.arange(n, dtype=np.uint64)
    def spread(v):
        v = v & np.uint64(0xFFFF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x00FF00FF)
        v = (v | (v << np.uint64(4))) & np.uint64(0x0F0F0F0F)
        v = (v | (v << np.uint64(2))) & np.uint64(0x33333333)
        v = (v | (v << np.uint64(1))) & np.uint64(0x55555555)
        return v
    IX, IY = np.meshgrid(i, i, indexing="xy")
    z = spread(IX.ravel()) | (spread(IY.ravel()) << np.uint64(1))
    order = np.argsort(z, kind="stable")
    x, y = ray_grid(n, lo, hi)
    return x[order].copy(), y[order].copy()


def uniform_points(n: int, seed: int, lo: float = -0.5, hi: float = 0.5):
    g = rng(seed)
    return g.uniform(lo, hi, n), g.uniform(lo, hi, n)


# --------------------------------------------------------------------------
# particle sets
# --------------------------------------------------------------------------
def nfw_projected(n: int, seed: int, c: float = 5.0, r200: float = 1.0):
    """Projected positions of n particles drawn from a 3D NFW profile
    (nfw_3d without its z coordinate)."""
    x, y, _ = nfw_3d(n, seed, c, r200)
    return x, y


def nfw_3d(n: int, seed: int, c: float = 5.0, r200: float = 1.0):
    """3D positions (x, y, z) of n particles drawn from an NFW profile.

    Radii follow the enclosed-mass fraction mu(x) = ln(1+x) - x/(1+x) on
    x = r/r_s in [0, c] (truncated at r200 = c r_s), inverted through the
    principal branch of the Lambert W function; directions are isotropic.
    """
    from scipy.special import lambertw

    g = rng(seed)
    rs = r200 / c
    mu_c = math.log1p(c) - c / (1.0 + c)
    t = g.uniform(0.0, 1.0, n) * mu_c
    w = lambertw(-np.exp(-1.0 - t), 0).real
    x = -1.0 / w - 1.0
    r = np.clip(x, 0.0, c) * rs
    cost = g.uniform(-1.0, 1.0, n)
    phi = g.uniform(0.0, 2.0 * math.pi, n)
    sint = np.sqrt(np.maximum(0.0, 1.0 - cost * cost))
    return r * sint * np.cos(phi), r * sint * np.sin(phi), r * cost


def knn_smoothing(x, y, k: int = 32):
    """2D distance from each particle to its k-th nearest neighbour (self excluded)."""
    from scipy.spatial import cKDTree

    pts = np.column_stack([x, y])
    tree = cKDTree(pts)
    d, _ = tree.query(pts, k=k + 1, workers=-1)
    return np.ascontiguousarray(d[:, k])


def salpeter_masses(n: int, seed: int, lo: float = 0.1, hi: float = 1.0, slope: float = 2.35):
    """Masses with dN/dm proportional to m^-slope on [lo, hi] (inverse CDF)."""
    g = rng(seed)
    a = 1.0 - slope
    u = g.uniform(0.0, 1.0, n)
    return (lo ** a + u * (hi ** a - lo ** a)) ** (1.0 / a)


@dataclass
class Lens:
    """Particles of one lens plane (code units: a point mass deflects m d/|d|^2)."""

    x: np.ndarray
    y: np.ndarray
    m: np.ndarray
    s: np.ndarray  # smoothing length; 0 marks a point mass
    q: float = 3.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def point_masses(n: int, seed: int, m: float = 1e-3, half: float = 0.5) -> Lens:
    """n equal point masses uniform in the square [-half, half]^2."""
    g = rng(seed)
    x = g.uniform(-half, half, n)
    y = g.uniform(-half, half, n)
    return Lens(x, y, np.full(n, m), np.zeros(n), meta={"kind": "point_masses"})


def point_masses_disk(n: int, seed: int, m: float = 1.0, radius: float = 1.0) -> Lens:
    """n equal point masses uniform in a disk (the paper's tree convergence test)."""
    g = rng(seed)
    r = radius * np.sqrt(g.uniform(0.0, 1.0, n))
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    return Lens(r * np.cos(ph), r * np.sin(ph), np.full(n, m), np.zeros(n),
                meta={"kind": "point_masses_disk"})


def nfw_halo(n: int, seed: int, k: int = 32, q: float = 3.0, total_mass: float = 1.0) -> Lens:
    """Smoothed NFW halo: equal masses summing to total_mass, kNN smoothing."""
    x, y = nfw_projected(n, seed)
    s = knn_smoothing(x, y, k) if n > k else np.full(n, 0.05)
    return Lens(x, y, np.full(n, total_mass / n), s, q=q, meta={"kind": "nfw", "k": k})


def star_patch(n: int, seed: int, center=(0.25, 0.0), side: float = 0.01,
               kappa_star: float = 0.3) -> Lens:
    """n point-mass stars uniform in a square patch, Salpeter masses scaled so
    that the mean stellar convergence over the patch equals kappa_star."""
    g = rng(seed)
    x = center[0] + g.uniform(-side / 2, side / 2, n)
    y = center[1] + g.uniform(-side / 2, side / 2, n)
    m = salpeter_masses(n, seed + 1)
    # kappa = (sum m) * pi / area in code units (m already divided by pi Sigma_crit)
    m *= kappa_star * side * side / math.pi / m.sum()
    return Lens(x, y, m, np.zeros(n), meta={"kind": "stars"})


def gaussian_blobs(n: int, seed: int, s_lo: float = 0.01, s_hi: float = 0.1,
                   half: float = 0.5, q: float = 3.0) -> Lens:
    """Smoothed particles with random positions, masses and smoothing lengths."""
    g = rng(seed)
    x = g.uniform(-half, half, n)
    y = g.uniform(-half, half, n)
    m = g.uniform(0.1, 1.0, n) / n
    s = np.exp(g.uniform(math.log(s_lo), math.log(s_hi), n))
    return Lens(x, y, m, s, q=q, meta={"kind": "blobs"})


def nfw_halo_field(n: int, seed: int, rmax: float = 0.3, c: float = 3.0, mmin: float = 1e-3,
                   mmax: float = 1.0, radius: float = 1.0):
    """The paper's halo convergence test (Sec. 5.1): n truncated NFW halos
    uniform in a disk, sizes uniform up to rmax, masses dN/dm ~ m^-2 on
    [mmin, mmax], all of concentration c.  Returns (Lens with s = sizes, c)."""
    g = rng(seed)
    r = radius * np.sqrt(g.uniform(0.0, 1.0, n))
    ph = g.uniform(0.0, 2.0 * math.pi, n)
    size = g.uniform(0.0, rmax, n)
    u = g.uniform(0.0, 1.0, n)
    m = 1.0 / (1.0 / mmin - u * (1.0 / mmin - 1.0 / mmax))
    return Lens(r * np.cos(ph), r * np.sin(ph), m, size, q=c, meta={"kind": "nfw_halos", "c": c}), c


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def workload_point_masses_1k():
    """1,000 point masses of m=1e-3 in [-0.5,0.5]^2; 64x64 ray grid."""
    lens = point_masses(1000, BASE_SEED + 1)
    rx, ry = ray_grid(64)
    return lens, rx, ry


def workload_nfw(n: int = 1_000_000, grid: int = 2048, seed: int = BASE_SEED + 2):
    """Smoothed NFW halo (c=5, r200=1) of n particles, kNN32 smoothing, q=3;
    grid x grid ray grid over [-0.5,0.5]^2."""
    lens = nfw_halo(n, seed)
    rx, ry = ray_grid(grid)
    return lens, rx, ry


def workload_microlensing(n_halo: int = 1_000_000, n_stars: int = 100_000, base: int = 256,
                          center=(0.25, 0.0), patch: float = 0.01):
    """The smoothed NFW halo plus n_stars point-mass stars in a patch x patch
    square around an image position (Salpeter masses, mean stellar convergence
    0.3 over the patch), and a base x base grid of square cells over the patch
    (centres and sides)."""
    halo = nfw_halo(n_halo, BASE_SEED + 2)
    stars = star_patch(n_stars, BASE_SEED + 20, center=center, side=patch)
    lens = Lens(np.concatenate([halo.x, stars.x]), np.concatenate([halo.y, stars.y]),
                np.concatenate([halo.m, stars.m]), np.concatenate([halo.s, stars.s]), q=halo.q,
                meta={"kind": "halo+stars", "n_stars": n_stars})
    cx, cy = ray_grid(base, -patch / 2, patch / 2)
    return lens, cx + center[0], cy + center[1], np.full(base * base, patch / base)


def workload_batched_lenses(nlens: int = 64, seed: int = BASE_SEED + 30, scale: float = 1.0):
    """nlens independent smoothed NFW lenses: particle counts log-uniform in
    [1e3, 1e5], ray grids n x n with n log-uniform in [256, 1024] over
    [-0.5, 0.5]^2 (scale < 1 shrinks both for quick runs)."""
    g = rng(seed)
    out = []
    for l in range(nlens):
        n = int(round(10 ** g.uniform(3, 5) * scale))
        side = int(round(2 ** g.uniform(8, 10) * math.sqrt(scale)))
        lens = nfw_halo(max(n, 40), seed + 1000 + l)
        rx, ry = ray_grid(max(side, 8))
        out.append((lens, rx, ry))
    return out


def sample_rays(rx, ry, k: int, seed: int):
    """Seeded subset of k ray indices (sorted)."""
    g = rng(seed)
    k = min(k, rx.shape[0])
    return np.sort(g.choice(rx.shape[0], size=k, replace=False))
