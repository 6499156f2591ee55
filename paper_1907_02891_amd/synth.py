"""Seeded synthetic inputs: radiance maps, point-spread matrices, site lists.

This module holds input generation only -- no convolution, transform or any
other step of the method -- so that the HIP path and the FP64 oracle can both
be fed from it.  All randomness comes from numpy's PCG64 (`default_rng(seed)`)
with a fixed draw order; maps are accumulated in FP64 and rounded to FP32 once.

The paper's own inputs (a reprojected VIIRS 2016 composite of Iberia at
404.4 m, and the LPTRAN point-spread function) are not available; these
"city-cluster" maps stand in for them: a sparse lognormal background of dim
lit pixels plus Gaussian city blobs with lognormal peaks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Mean distance from the centre of a unit square to a point drawn uniformly in
# it: (sqrt(2) + asinh(1)) / 6.  Used for the centre pixel of a kernel that
# diverges at d = 0 (d^-2.5 is not integrable over a 2-D cell, so a true
# cell average does not exist).
MEAN_CELL_DISTANCE = (math.sqrt(2.0) + math.asinh(1.0)) / 6.0


def radiance_map(ny, nx, n_blobs, bg_frac, sigma_px, rng, *,
                 bg_mu=-4.0, bg_sigma=1.0, peak_mu=3.0, peak_sigma=1.0,
                 truncate=5.0, centres=None):
    """City-cluster radiance grid, FP32 ny x nx.

    Draw order: background mask (Bernoulli(bg_frac) per pixel), background
    values lognormal(bg_mu, bg_sigma), then blob centres (uniform over the
    grid), widths (uniform in sigma_px), peaks lognormal(peak_mu, peak_sigma).
    Each blob is a Gaussian truncated at `truncate` sigma.  If `centres` is a
    list, the blob centres (row, column arrays, in pixels) are appended to it.
    """
    R = np.zeros((ny, nx), np.float64)
    if bg_frac > 0:
        mask = rng.random((ny, nx), dtype=np.float32) < bg_frac
        nbg = int(mask.sum())
        R[mask] = rng.lognormal(bg_mu, bg_sigma, nbg)
    cy = rng.uniform(0.0, ny, n_blobs)
    cx = rng.uniform(0.0, nx, n_blobs)
    sig = rng.uniform(sigma_px[0], sigma_px[1], n_blobs)
    peak = rng.lognormal(peak_mu, peak_sigma, n_blobs)
    if centres is not None:
        centres.append((cy.copy(), cx.copy()))
    for y0, x0, s, pk in zip(cy, cx, sig, peak):
        h = int(math.ceil(truncate * s))
        i0, i1 = max(0, int(y0) - h), min(ny, int(y0) + h + 1)
        j0, j1 = max(0, int(x0) - h), min(nx, int(x0) + h + 1)
        if i0 >= i1 or j0 >= j1:
            continue
        dy = np.arange(i0, i1) + 0.5 - y0
        dx = np.arange(j0, j1) + 0.5 - x0
        gy = np.exp(-0.5 * (dy / s) ** 2)
        gx = np.exp(-0.5 * (dx / s) ** 2)
        gy[np.abs(dy) > truncate * s] = 0.0
        gx[np.abs(dx) > truncate * s] = 0.0
        R[i0:i1, j0:j1] += pk * np.outer(gy, gx)
    return R.astype(np.float32)


def _distance_grid(half_y, half_x, pitch_km):
    di = np.arange(-half_y, half_y + 1, dtype=np.float64)
    dj = np.arange(-half_x, half_x + 1, dtype=np.float64)
    return pitch_km * np.sqrt(di[:, None] ** 2 + dj[None, :] ** 2)


def psf_powexp(half, exponent, scale_km, pitch_km, radius_km=None):
    """Radially symmetric K(d) = d^-exponent * exp(-d / scale_km), FP64.

    (2*half+1)^2 grid at `pitch_km`, distance d from the centre pixel in km.
    The centre pixel, where the formula diverges, takes K at the mean
    cell distance pitch * (sqrt(2) + asinh(1)) / 6.  With `radius_km` the
    kernel is cut to a disk: K = 0 where d > radius_km.
    """
    d = _distance_grid(half, half, pitch_km)
    d[half, half] = pitch_km * MEAN_CELL_DISTANCE
    K = d ** (-exponent) * np.exp(-d / scale_km)
    if radius_km is not None:
        K[_distance_grid(half, half, pitch_km) > radius_km] = 0.0
    return K


ALR_C = 1.0 / 562.72


def psf_alr(half, pitch_km, radius_km=300.0):
    """Duriscoe all-sky light-pollution-ratio kernel (Sec. 3, Eqs. 12-13).

    K(d) = c d^-alpha(d), alpha(d) = 2.3 (d/350)^0.28, c = 1/562.72, d in km;
    finite at d -> 0 (alpha -> 0, K -> c), valid to 300 km.
    """
    d = _distance_grid(half, half, pitch_km)
    with np.errstate(divide="ignore"):
        alpha = 2.3 * (d / 350.0) ** 0.28
        K = ALR_C * np.exp(-alpha * np.log(np.where(d > 0, d, 1.0)))
    K[half, half] = ALR_C
    if radius_km is not None:
        K[d > radius_km] = 0.0
    return K


def psf_random(ky, kx, rng, positive=True):
    """Unstructured kernel (no symmetry) for the general complex-spectrum path."""
    K = rng.random((ky, kx))
    if not positive:
        K -= 0.5
    return K


def psf_separable(ky, kx, rng):
    """Separable positive kernel K = outer(u, v); returns (u, v)."""
    cy, cx = (ky - 1) // 2, (kx - 1) // 2
    u = np.exp(-np.abs(np.arange(ky) - cy) / max(1.0, ky / 6.0)) * (0.5 + rng.random(ky))
    v = np.exp(-np.abs(np.arange(kx) - cx) / max(1.0, kx / 6.0)) * (0.5 + rng.random(kx))
    return u, v


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    ny: int
    nx: int
    ky: int
    kx: int
    py: int
    px: int
    pitch_km: float
    seed: int


SMALL = Workload("small-256x256-psf101-p512", 256, 256, 101, 101, 512, 512, 0.5, 1000)
COUNTRY = Workload("country-4096x4096-psf1201-p5400", 4096, 4096, 1201, 1201, 5400, 5400, 0.5, 1001)
CONTINENTAL = Workload("continental-16384x16384-psf2001-p18432", 16384, 16384, 2001, 2001,
                       18432, 18432, 0.5, 1002)
ADJOINT = Workload("adjoint-2048x2048-psf801-p2880", 2048, 2048, 801, 801, 2880, 2880, 0.5, 1004)
# longer than one LDS tile per column: the four-step column stage; 27000 =
# 5 x 5400 (>= n + k - 1 = 26000) lets the middle transforms use the 5400-point
# register kernels (26244, the smallest 5-smooth size, has no specialised divisor)
LARGE = Workload("large-24000x24000-psf2001-p27000", 24000, 24000, 2001, 2001, 27000, 27000, 0.5, 1006)
# the grid of the paper's own maps (Sec. 3: 11920 x 11804 pixels of 404.4 m)
# with the all-sky light-pollution-ratio kernel of Eqs. 12-13 out to its
# 300 km validity range (742 px at 404.4 m: 1485 x 1485)
PAPER = Workload("paper-11920x11804-alr1485-p13500", 11920, 11804, 1485, 1485, 13500, 13500, 0.4044, 1008)
BATCHED_SEED = 1003
CLASSES = Workload("classes-3x4096x4096-psf1201-p5400", 4096, 4096, 1201, 1201, 5400, 5400, 0.5, 1005)

WORKLOADS = {w.name: w for w in (SMALL, COUNTRY, CONTINENTAL, ADJOINT, CLASSES, LARGE, PAPER)}


def small_inputs(seed=SMALL.seed):
    """256x256 map, 5% background, 6 blobs (sigma 2-8 px); 101x101 kernel
    K = d^-2.5 exp(-d/80 km) on the full square (no radial cut)."""
    rng = np.random.default_rng(seed)
    R = radiance_map(256, 256, 6, 0.05, (2.0, 8.0), rng)
    K = psf_powexp(50, 2.5, 80.0, 0.5)
    return R, K


def country_inputs(seed=COUNTRY.seed, n=4096):
    """4096x4096 map, 5% background, 400 blobs (sigma 2-40 px); 1201x1201
    kernel d^-2.5 exp(-d/80 km) cut to a 300 km disk."""
    rng = np.random.default_rng(seed)
    R = radiance_map(n, n, 400, 0.05, (2.0, 40.0), rng)
    K = psf_powexp(600, 2.5, 80.0, 0.5, radius_km=300.0)
    return R, K


def continental_inputs(seed=CONTINENTAL.seed, n=16384, centres=None):
    """16384x16384 map, 20% background, 6000 blobs (sigma 2-40 px); 2001x2001
    kernel d^-2.5 exp(-d/80 km) cut to a 500 km disk.  `centres`: as in
    radiance_map."""
    rng = np.random.default_rng(seed)
    R = radiance_map(n, n, 6000, 0.20, (2.0, 40.0), rng, centres=centres)
    K = psf_powexp(1000, 2.5, 80.0, 0.5, radius_km=500.0)
    return R, K


def paper_inputs(seed=PAPER.seed, centres=None):
    """The paper's map grid (Sec. 3), 11920 x 11804 pixels of 404.4 m, filled
    with the city-cluster generator at the continental density (20%
    background, 3150 blobs, sigma 2-40 px); the ALR kernel of Eqs. 12-13
    cut at its 300 km validity range, 1485 x 1485.  `centres`: as in
    radiance_map."""
    rng = np.random.default_rng(seed)
    R = radiance_map(PAPER.ny, PAPER.nx, 3150, 0.20, (2.0, 40.0), rng, centres=centres)
    K = psf_alr(PAPER.ky // 2, PAPER.pitch_km, radius_km=300.0)
    return R, K


def large_inputs(seed=LARGE.seed, n=24000):
    """24000x24000 map at the continental density (20% background, 12875
    blobs, sigma 2-40 px); the continental 2001x2001 kernel (500 km disk)."""
    rng = np.random.default_rng(seed)
    R = radiance_map(n, n, 12875, 0.20, (2.0, 40.0), rng)
    K = psf_powexp(1000, 2.5, 80.0, 0.5, radius_km=500.0)
    return R, K


def adjoint_inputs(seed=ADJOINT.seed, n=2048, n_sites=2000):
    """2048x2048 map (100 blobs, sigma 2-40 px, 5% background); 801x801 kernel
    d^-2.5 exp(-d/80 km) cut to a 200 km disk; 2000 distinct site pixels; a
    perturbed ground truth R_true = R0 * exp(0.2 N(0,1)) and per-site noise
    draws eps ~ N(0,1) (measurements are m_i = S[R_true](x_i) (1 + 0.05 eps_i),
    weights w_i = 1/m_i^2; forming S is the caller's job)."""
    rng = np.random.default_rng(seed)
    R0 = radiance_map(n, n, 100, 0.05, (2.0, 40.0), rng)
    K = psf_powexp(400, 2.5, 80.0, 0.5, radius_km=200.0)
    sites = rng.choice(n * n, n_sites, replace=False).astype(np.int64)
    R_true = (R0.astype(np.float64) * np.exp(0.2 * rng.standard_normal((n, n)))).astype(np.float32)
    eps = rng.standard_normal(n_sites)
    return R0, K, sites, R_true, eps


BATCHED_PSFS = ((40.0, 2.2), (80.0, 2.4), (120.0, 2.6), (160.0, 2.8))
BAND_RATIOS = (1.0, 0.8, 0.5)


def batched_inputs(seed=BATCHED_SEED, n_tiles=64, side=(512, 3072), half=600):
    """64 tiles with sides drawn uniformly from [512, 3072] per axis, city
    blobs at 400 per 4096^2 (sigma 2-40 px, 5% background); each tile is
    paired with one of 4 kernels (scale, exponent) = (40 km, 2.2), (80, 2.4),
    (120, 2.6), (160, 2.8), cut to a 300 km disk, and split into 3 bands with
    ratios 1 : 0.8 : 0.5 times a per-tile, per-band lognormal(0, 0.1) jitter.

    Returns (tiles, psf_ids, psfs): tiles is a list of FP32 arrays of shape
    (3, ny, nx)."""
    rng = np.random.default_rng(seed)
    shapes = rng.integers(side[0], side[1] + 1, size=(n_tiles, 2))
    psf_ids = rng.integers(0, len(BATCHED_PSFS), size=n_tiles)
    tiles = []
    for t in range(n_tiles):
        ny, nx = int(shapes[t, 0]), int(shapes[t, 1])
        n_blobs = max(1, int(round(400 * ny * nx / 4096.0 ** 2)))
        base = radiance_map(ny, nx, n_blobs, 0.05, (2.0, 40.0), rng).astype(np.float64)
        jit = np.exp(0.1 * rng.standard_normal(3))
        bands = np.stack([base * (BAND_RATIOS[b] * jit[b]) for b in range(3)]).astype(np.float32)
        tiles.append(bands)
    psfs = [psf_powexp(half, e, s, 0.5, radius_km=300.0) for (s, e) in BATCHED_PSFS]
    return tiles, psf_ids.astype(np.int32), psfs


# (scale km, exponent) of the three source classes' kernels
CLASS_PSFS = ((60.0, 2.3), (80.0, 2.5), (110.0, 2.7))


def classes_inputs(seed=CLASSES.seed, n=4096, half=600):
    """Three source classes (Eq. 4) over the country-sized grid: each class
    is its own city-cluster map (400 blobs, sigma 2-40 px, 5% background,
    own seed stream) with its own kernel d^-a exp(-d/s), (s, a) from
    CLASS_PSFS, cut to a 300 km disk.  Returns (maps, kernels)."""
    rng = np.random.default_rng(seed)
    maps = [radiance_map(n, n, 400, 0.05, (2.0, 40.0), rng) for _ in CLASS_PSFS]
    kernels = [psf_powexp(half, a, s_km, 0.5, radius_km=300.0) for (s_km, a) in CLASS_PSFS]
    return maps, kernels


def sample_pixels(R, n, rng, *, n_bright=None, K=None):
    """Flat pixel indices for sampled parity: half uniform, a quarter at the
    brightest input pixels, a quarter uniform over the dim remainder."""
    ny, nx = R.shape
    n_bright = n // 4 if n_bright is None else n_bright
    n_uni = n - 2 * n_bright
    uni = rng.choice(ny * nx, n_uni, replace=False)
    flat = R.ravel()
    top = np.argpartition(flat, -n_bright)[-n_bright:]
    dim_pool = np.flatnonzero(flat <= np.quantile(flat, 0.5))
    dim = rng.choice(dim_pool, min(n_bright, dim_pool.size), replace=False)
    return np.unique(np.concatenate([uni, top, dim]).astype(np.int64))


def sample_pixels_c12(R, centres, rng, n_uniform=2048, n_bright=1024, n_far=1024, min_dist=200.0):
    """Sample of output pixels for the continental map: n_uniform drawn
    uniformly, the n_bright brightest input pixels, and n_far drawn uniformly
    among the pixels at least min_dist pixels from every blob centre (the
    dark countryside, where FP32 transform error is largest relative to the
    value).  centres: (row, column) arrays of the blob centres.  Flat indices,
    sorted, without repeats."""
    from scipy.spatial import cKDTree
    ny, nx = R.shape
    uni = rng.choice(ny * nx, n_uniform, replace=False)
    flat = R.ravel()
    top = np.argpartition(flat, -n_bright)[-n_bright:]
    tree = cKDTree(np.stack([centres[0], centres[1]], axis=1))
    far = []
    while len(far) < n_far:
        cand = rng.choice(ny * nx, 8 * n_far, replace=False)
        pts = np.stack([cand // nx + 0.5, cand % nx + 0.5], axis=1)
        d, _ = tree.query(pts)
        far.extend(cand[d >= min_dist].tolist())
    far = np.asarray(far[:n_far], np.int64)
    return np.unique(np.concatenate([uni, top, far]).astype(np.int64))
