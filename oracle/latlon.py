"""FP64 oracle for the preprocessing steps either side of the convolution
(test infrastructure only; see the package docstring).

Sec. 2.4: the radiance composite comes on a uniform longitude-latitude grid
(plate carree) whose ground scale varies with latitude; the convolution needs
a grid of uniform scale, so the map is reprojected onto a transverse
Mercator (UTM) grid by nearest-neighbour resampling.  Eq. 11 gives the point
scale factor of that projection, k = k0 cosh(x / (k0 R)), from Snyder's
spherical transverse Mercator (the paper's reference for Eq. 11).  The
inverse of that projection, which a gather needs (the latitude and longitude
of a projected point), is Snyder's spherical inverse:
    D = y / (k0 R) + phi0,
    phi = asin(sin D / cosh(x / (k0 R))),
    lambda = lambda0 + atan2(sinh(x / (k0 R)), cos D),
and the forward projection, used here only to pin the inverse, is
    B = cos(phi) sin(lambda - lambda0),
    x = k0 R atanh(B),  y = k0 R (atan2(tan phi, cos(lambda - lambda0)) - phi0).

Sec. 4 (an alternative the paper outlines but does not develop): convolve in
the native longitude-latitude grid with a kernel held constant within narrow
latitude bands.  On that grid one pixel step is R dphi north-south and
R cos(phi) dlambda east-west, so the band's kernel samples the radial PSF at
d = sqrt((R dphi a)^2 + (R cos(phi_b) dlambda b)^2) with phi_b the band's
centre latitude.

Grid conventions shared with the library: source row r has latitude
lat_first - r dlat (rows run southward), column c longitude lon_first +
c dlon; projected row i has northing y_first - i pitch, column j easting
x_first + j pitch (km from the central meridian, no false easting).
"""
from __future__ import annotations

import numpy as np

from . import conv_same_pixels

DEG = np.pi / 180.0


def tm_forward(lat_deg, lon_deg, lon0_deg, k0, R_km, lat0_deg=0.0):
    """Spherical transverse Mercator, (lat, lon) in degrees -> (x, y) in km."""
    phi = np.asarray(lat_deg, np.float64) * DEG
    dl = (np.asarray(lon_deg, np.float64) - lon0_deg) * DEG
    B = np.cos(phi) * np.sin(dl)
    x = k0 * R_km * np.arctanh(B)
    y = k0 * R_km * (np.arctan2(np.tan(phi), np.cos(dl)) - lat0_deg * DEG)
    return x, y


def tm_inverse(x_km, y_km, lon0_deg, k0, R_km, lat0_deg=0.0):
    """Spherical inverse transverse Mercator, (x, y) in km -> (lat, lon) in degrees."""
    xs = np.asarray(x_km, np.float64) / (k0 * R_km)
    D = np.asarray(y_km, np.float64) / (k0 * R_km) + lat0_deg * DEG
    phi = np.arcsin(np.sin(D) / np.cosh(xs))
    lam = lon0_deg * DEG + np.arctan2(np.sinh(xs), np.cos(D))
    return phi / DEG, lam / DEG


def scale_factor(x_km, k0, R_km):
    """Eq. 11: point scale factor of the transverse Mercator at easting x."""
    return k0 * np.cosh(np.asarray(x_km, np.float64) / (k0 * R_km))


def reproject_indices(ny, nx, x_first, y_first, pitch, lon0_deg, k0, R_km,
                      lat_first, lon_first, dlat, dlon):
    """Continuous source (row, column) of every projected pixel centre."""
    x = x_first + pitch * np.arange(nx, dtype=np.float64)
    y = y_first - pitch * np.arange(ny, dtype=np.float64)
    X, Y = np.meshgrid(x, y)
    lat, lon = tm_inverse(X, Y, lon0_deg, k0, R_km)
    return (lat_first - lat) / dlat, (lon - lon_first) / dlon, X


def reproject_nn(src, lat_first, lon_first, dlat, dlon, ny, nx, x_first, y_first, pitch,
                 lon0_deg, k0, R_km, ground_area=False):
    """Nearest-neighbour gather of a plate-carree map onto the projected grid
    (Sec. 2.4): each projected pixel takes the source pixel whose centre is
    nearest in (row, column) index space, rounding halves to even; 0 where
    that pixel lies outside the source grid.  ground_area multiplies by
    1 / k^2 (Eq. 11; the projection is conformal, so a projected cell of
    pitch^2 covers pitch^2 / k^2 of ground).  Returns (map, rowf, colf)."""
    src = np.asarray(src)
    rowf, colf, X = reproject_indices(ny, nx, x_first, y_first, pitch, lon0_deg, k0, R_km,
                                      lat_first, lon_first, dlat, dlon)
    r = np.rint(rowf)
    c = np.rint(colf)
    ok = (r >= 0) & (r < src.shape[0]) & (c >= 0) & (c < src.shape[1])
    out = np.zeros((ny, nx), np.float64)
    out[ok] = src[r[ok].astype(np.int64), c[ok].astype(np.int64)]
    if ground_area:
        out *= 1.0 / scale_factor(X, k0, R_km) ** 2
    return out, rowf, colf


def band_kernel(radial, lat_c_deg, dlat_deg, dlon_deg, half_y, half_x, R_km):
    """Kernel of one latitude band on the longitude-latitude grid (Sec. 4):
    (2 half_y + 1) x (2 half_x + 1) samples of the radial PSF at the ground
    distance of each pixel offset, east-west steps shortened by cos(phi_c)."""
    a = np.arange(-half_y, half_y + 1, dtype=np.float64)[:, None]
    b = np.arange(-half_x, half_x + 1, dtype=np.float64)[None, :]
    dy = R_km * dlat_deg * DEG * a
    dx = R_km * np.cos(lat_c_deg * DEG) * dlon_deg * DEG * b
    return radial(np.sqrt(dx * dx + dy * dy))


def conv_latitude_bands_pixels(L, band_edges, kernels, idx):
    """Sky brightness at flat pixel indices idx when output row i uses the
    kernel of the band that contains it (band t covers rows
    [band_edges[t], band_edges[t+1])), each a direct FP64 "same" sum over the
    whole map (Eq. 7 with the band's kernel)."""
    idx = np.asarray(idx, np.int64)
    rows = idx // L.shape[1]
    out = np.empty(idx.shape[0], np.float64)
    for t, K in enumerate(kernels):
        sel = (rows >= band_edges[t]) & (rows < band_edges[t + 1])
        if sel.any():
            out[sel] = conv_same_pixels(L, K, idx[sel])
    return out
