"""Seeded synthetic inputs for the image-plane chi^2 workloads.

This module only draws random numbers and lays them out; it holds none of the
lensing arithmetic (no deflection, no cosmology, no image finding).  Both the
CPU oracle's tests and the GPU path's tests and benchmark take their inputs
from here, so the two sides always see identical bytes.

Parameter layout (structure of arrays, as in Sec. 2.3 of Rexroth et al. 2019):
a float64 array of shape [7, P] whose rows are

    0 x        centre, arcsec
    1 y        centre, arcsec
    2 eps      pseudo-ellipticity of the potential, 0 <= eps < 1 (Sec. 2.2.2)
    3 phi      position angle, radians, counter-clockwise from the theta_1 axis
    4 r_core   core radius a, arcsec (0 for a singular profile)
    5 r_cut    cut radius s, arcsec (+inf for an uncut profile)
    6 sigma_v  velocity dispersion, km/s

The workloads below follow the five benchmark configurations; every choice they
leave open (centred halo, uniform core/cut radii, source disk radius, ...) is
marked "reading" where it is made.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PARAM_ROWS = ("x", "y", "eps", "phi", "r_core", "r_cut", "sigma_v")
N_PARAM = 7

SEED_BASE = 190203252  # arXiv id of the paper; config k uses SEED_BASE * 10 + k
Z_LENS = 0.3           # lens redshift of the paper's benchmark cluster (Sec. 4)
OBS_SIGMA = 0.1        # arcsec, positional error of every observed image


@dataclasses.dataclass(frozen=True)
class Grid:
    """Regular image-plane grid of nodes: node (i, j) = (x0 + i*h, y0 + j*h)."""
    x0: float
    y0: float
    h: float
    nx: int
    ny: int

    @property
    def n_triangles(self) -> int:
        return 2 * (self.nx - 1) * (self.ny - 1)


def square_grid(n: int, half_width: float) -> Grid:
    """N x N nodes spanning [-L, L] in both axes, end points included (reading)."""
    h = 2.0 * half_width / (n - 1)
    return Grid(-half_width, -half_width, h, n, n)


def rng(config: int, stream: int = 0) -> np.random.Generator:
    """Independent PCG64 stream per (config, purpose)."""
    return np.random.Generator(np.random.PCG64([SEED_BASE * 10 + config, stream]))


# --------------------------------------------------------------------------
# potentials
# --------------------------------------------------------------------------

def _empty(p: int) -> np.ndarray:
    return np.zeros((N_PARAM, p), dtype=np.float64)


def config1_potentials() -> np.ndarray:
    """One cored/cut isothermal potential at the origin (reading: centred)."""
    prm = _empty(1)
    prm[:, 0] = (0.0, 0.0, 0.2, math.radians(30.0), 0.5, 300.0, 800.0)
    return prm


CLUSTER_HALO = (0.0, 0.0, 0.05, 0.0, 5.0, 1000.0, 1000.0)  # reading: centred, eps of Sec. 4's first halo


def draw_galaxies(g: np.random.Generator, n: int, pos_half_width: float = 60.0) -> np.ndarray:
    """Galaxy-scale potentials: uniform positions, log-uniform sigma_v on [100, 300] km/s,
    r_core ~ U[0.05, 0.3]", r_cut ~ U[20, 80]", eps ~ U[0, 0.5], phi ~ U[0, pi)."""
    prm = _empty(n)
    prm[0] = g.uniform(-pos_half_width, pos_half_width, n)
    prm[1] = g.uniform(-pos_half_width, pos_half_width, n)
    prm[2] = g.uniform(0.0, 0.5, n)
    prm[3] = g.uniform(0.0, math.pi, n)
    prm[4] = g.uniform(0.05, 0.3, n)
    prm[5] = g.uniform(20.0, 80.0, n)
    prm[6] = np.exp(g.uniform(math.log(100.0), math.log(300.0), n))
    return prm


def cluster_potentials(n_galaxies: int, config: int) -> np.ndarray:
    """One cluster halo followed by n_galaxies galaxy-scale potentials."""
    prm = _empty(1 + n_galaxies)
    prm[:, 0] = CLUSTER_HALO
    prm[:, 1:] = draw_galaxies(rng(config, 1), n_galaxies)
    return prm


def sie_potentials(n: int, seed: int = 0, half_width: float = 50.0) -> np.ndarray:
    """Singular (r_core = 0) uncut (r_cut = inf) pseudo-elliptical isothermal
    potentials: the exact model of Algorithm 1."""
    g = np.random.Generator(np.random.PCG64([SEED_BASE, 100 + seed]))
    prm = _empty(n)
    prm[0] = g.uniform(-half_width, half_width, n)
    prm[1] = g.uniform(-half_width, half_width, n)
    prm[2] = g.uniform(0.0, 0.3, n)
    prm[3] = g.uniform(0.0, math.pi, n)
    prm[4] = 0.0
    prm[5] = np.inf
    prm[6] = g.uniform(50.0, 400.0, n)
    return prm


# --------------------------------------------------------------------------
# sources and observations (raw draws only)
# --------------------------------------------------------------------------

def disk_points(g: np.random.Generator, n: int, radius: float) -> np.ndarray:
    """Area-uniform points in a disk of the given radius, shape [n, 2]."""
    r = radius * np.sqrt(g.uniform(0.0, 1.0, n))
    t = g.uniform(0.0, 2.0 * math.pi, n)
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def source_redshifts(g: np.random.Generator, n: int, lo: float = 1.0, hi: float = 6.0) -> np.ndarray:
    return g.uniform(lo, hi, n)


def position_noise(g: np.random.Generator, n: int, sigma: float = OBS_SIGMA) -> np.ndarray:
    """Gaussian positional noise for n observed images, shape [n, 2]."""
    return g.normal(0.0, sigma, (n, 2))


# --------------------------------------------------------------------------
# workload descriptions
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n_galaxies: int       # -1 for the single-potential config
    n: int                # grid nodes per side
    half_width: float     # grid spans [-L, L]
    n_sources: int
    source_radius: float  # area-uniform source draw radius, arcsec
    z_sources: tuple = () # fixed source redshifts (config 1); empty => U[1, 6]
    min_images: int = 2
    max_images: int = 5

    @property
    def grid(self) -> Grid:
        return square_grid(self.n, self.half_width)


WORKLOADS = {
    1: Workload("tiny: 1 cored/cut isothermal potential, 128^2 grid, 2 sources",
                -1, 128, 40.0, 2, 2.0, (2.0, 3.0), 1, 5),
    2: Workload("cluster: 1 halo + 49 galaxies, 1024^2 grid, 20 sources",
                49, 1024, 80.0, 20, 15.0),
    3: Workload("large: 1 halo + 199 galaxies, 4096^2 grid, 100 sources",
                199, 4096, 100.0, 100, 15.0),
    5: Workload("differentiation: 50 potentials, 512^2 grid, config-2 systems",
                49, 512, 80.0, 20, 15.0),
}


def potentials(config: int) -> np.ndarray:
    if config == 1:
        return config1_potentials()
    if config == 5:  # reading: the config-2 potentials themselves
        return cluster_potentials(WORKLOADS[2].n_galaxies, 2)
    return cluster_potentials(WORKLOADS[config].n_galaxies, config)


# --------------------------------------------------------------------------
# batched samples (config 4)
# --------------------------------------------------------------------------

BATCH_GRID_SIZES = (256, 512, 1024, 2048)
BATCH_HALF_WIDTH = 80.0


def batch_samples(n_samples: int = 1024, base: np.ndarray | None = None, seed_stream: int = 4,
                  p_min: int = 10, p_max: int = 200, grid_sizes=BATCH_GRID_SIZES,
                  scale: float = 0.05):
    """Lens-parameter samples as a sampler proposes them (reading of the batched workload):
    P_s ~ U{p_min..p_max}; grid side N_s uniform over grid_sizes; parameters are the
    config-2 halo plus its first min(P_s-1, 49) galaxies, extra galaxies drawn fresh,
    then every parameter multiplied by (1 + scale * N(0,1)).  r_cut > r_core is kept,
    eps is clipped to [0, 0.5] and phi taken mod pi.

    Returns (params [7, sum P_s] float64, pot_off [n+1] int32, grids list[Grid])."""
    if base is None:
        base = potentials(2)
    g = rng(4, seed_stream)
    counts = g.integers(p_min, p_max + 1, n_samples)
    sides = g.choice(np.asarray(grid_sizes), n_samples)
    blocks = []
    for s in range(n_samples):
        p = int(counts[s])
        keep = min(p, base.shape[1])
        prm = np.empty((N_PARAM, p))
        prm[:, :keep] = base[:, :keep]
        if p > keep:
            prm[:, keep:] = draw_galaxies(g, p - keep)
        prm = prm * (1.0 + scale * g.normal(0.0, 1.0, prm.shape))
        prm[2] = np.clip(prm[2], 0.0, 0.5)
        prm[3] = np.mod(prm[3], math.pi)
        prm[4] = np.abs(prm[4])
        bad = prm[5] <= prm[4]
        prm[5, bad] = prm[4, bad] * 2.0 + 1.0
        prm[6] = np.abs(prm[6])
        blocks.append(prm)
    params = np.concatenate(blocks, axis=1)
    pot_off = np.zeros(n_samples + 1, dtype=np.int32)
    pot_off[1:] = np.cumsum(counts)
    grids = [square_grid(int(n), BATCH_HALF_WIDTH) for n in sides]
    return params, pot_off, grids


def cotangent(n_nodes: int, seed_stream: int = 5) -> np.ndarray:
    """Seeded N(0,1) cotangent for the deflection-field backward pass, shape [2, n_nodes]."""
    return rng(5, seed_stream).normal(0.0, 1.0, (2, n_nodes))


# --------------------------------------------------------------------------
# the paper's benchmark lens (Sec. 4): SIE halos on an HST ACS-like image
# --------------------------------------------------------------------------

PAPER_PIXEL = 0.03  # arcsec per pixel (Sec. 3.2, Sec. 4)
PAPER_SIDE = 6730   # pixels per side (Sec. 4)
PAPER_GALAXIES = 700


def paper_grid(n: int = PAPER_SIDE, h: float = PAPER_PIXEL, ny: int | None = None) -> Grid:
    """n x ny nodes of spacing h centred on the origin (reading: one node per pixel)."""
    ny = n if ny is None else ny
    return Grid(-0.5 * (n - 1) * h, -0.5 * (ny - 1) * h, h, n, ny)


def paper_sie_cluster(grid: Grid, n_galaxies: int = PAPER_GALAXIES, seed: int = 0) -> np.ndarray:
    """Two cluster-scale SIE halos (sigma_v 1000 and 700 km/s, eps 0.05 and
    0.04) followed by n_galaxies galaxy-scale SIE halos (sigma_v ~ U[10, 15]
    km/s, eps ~ U[0, 0.15]), Sec. 4.  Readings (the paper gives no positions
    or angles): the two halos at (-0.2, -0.1) and (0.25, 0.15) times the grid's
    half widths, at position angles 0.5 and 2.0 rad; galaxies uniform over the
    grid with phi ~ U[0, pi)."""
    g = np.random.Generator(np.random.PCG64([SEED_BASE, 200 + seed]))
    lx, ly = 0.5 * (grid.nx - 1) * grid.h, 0.5 * (grid.ny - 1) * grid.h
    cx, cy = grid.x0 + lx, grid.y0 + ly
    prm = _empty(2 + n_galaxies)
    prm[:, 0] = (cx - 0.2 * lx, cy - 0.1 * ly, 0.05, 0.5, 0.0, np.inf, 1000.0)
    prm[:, 1] = (cx + 0.25 * lx, cy + 0.15 * ly, 0.04, 2.0, 0.0, np.inf, 700.0)
    n = n_galaxies
    prm[0, 2:] = g.uniform(cx - lx, cx + lx, n)
    prm[1, 2:] = g.uniform(cy - ly, cy + ly, n)
    prm[2, 2:] = g.uniform(0.0, 0.15, n)
    prm[3, 2:] = g.uniform(0.0, math.pi, n)
    prm[4, 2:] = 0.0
    prm[5, 2:] = np.inf
    prm[6, 2:] = g.uniform(10.0, 15.0, n)
    return prm


# --------------------------------------------------------------------------
# pseudo-elliptical NFW halos (parameter table [6, P]: x, y, eps, phi, r_s, kappa_s)
# --------------------------------------------------------------------------

NFW_ROWS = ("x", "y", "eps", "phi", "r_s", "kappa_s")


def nfw_cluster(grid: Grid, n_galaxies: int = PAPER_GALAXIES, seed: int = 0) -> np.ndarray:
    """The benchmark cluster of paper_sie_cluster with NFW halos instead of
    SIEs (reading; the paper only names the profile): two cluster-scale halos
    at the same places (r_s 40" and 30", kappa_s 0.25 and 0.2, eps 0.05 and
    0.04) and galaxy-scale halos with r_s ~ U[1, 4]", kappa_s ~ U[0.01, 0.05],
    eps ~ U[0, 0.15], uniform over the grid."""
    g = np.random.Generator(np.random.PCG64([SEED_BASE, 300 + seed]))
    lx, ly = 0.5 * (grid.nx - 1) * grid.h, 0.5 * (grid.ny - 1) * grid.h
    cx, cy = grid.x0 + lx, grid.y0 + ly
    prm = np.zeros((6, 2 + n_galaxies))
    prm[:, 0] = (cx - 0.2 * lx, cy - 0.1 * ly, 0.05, 0.5, 40.0, 0.25)
    prm[:, 1] = (cx + 0.25 * lx, cy + 0.15 * ly, 0.04, 2.0, 30.0, 0.2)
    n = n_galaxies
    prm[0, 2:] = g.uniform(cx - lx, cx + lx, n)
    prm[1, 2:] = g.uniform(cy - ly, cy + ly, n)
    prm[2, 2:] = g.uniform(0.0, 0.15, n)
    prm[3, 2:] = g.uniform(0.0, math.pi, n)
    prm[4, 2:] = g.uniform(1.0, 4.0, n)
    prm[5, 2:] = g.uniform(0.01, 0.05, n)
    return prm
