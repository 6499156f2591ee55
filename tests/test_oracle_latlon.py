"""Pins of the oracle's preprocessing steps (Sec. 2.4 reprojection with the
scale factor of Eq. 11; Sec. 4 latitude-band kernels; the ALR kernel of
Eqs. 12-13), on the CPU."""
import os

import numpy as np
import pytest

from oracle import latlon
from paper_1907_02891_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
K0, R = 0.9996, 6367.0


def test_eq11_values_printed_in_the_paper():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "eq11_utm_scale.txt"))
            if l.strip() and not l.startswith("#")]
    for x, k, dec in rows:
        assert round(float(latlon.scale_factor(float(x), K0, R)), int(dec)) == float(k)
    # surface scale error at 800 km: k^2 - 1 rounds to 1.5%
    assert round(float(latlon.scale_factor(800.0, K0, R)) ** 2 - 1.0, 3) == 0.015


def test_inverse_undoes_forward():
    lat, lon = np.meshgrid(np.linspace(-70, 70, 29), np.linspace(-9, 5, 15), indexing="ij")
    x, y = latlon.tm_forward(lat, lon, -3.0, K0, R)
    la, lo = latlon.tm_inverse(x, y, -3.0, K0, R)
    np.testing.assert_allclose(la, lat, atol=1e-9)
    np.testing.assert_allclose(lo, lon, atol=1e-9)
    x2, y2 = latlon.tm_forward(la, lo, -3.0, K0, R)
    np.testing.assert_allclose(x2, x, atol=1e-7)
    np.testing.assert_allclose(y2, y, atol=1e-7)


def test_central_meridian_closed_form():
    y = np.linspace(-6000, 6000, 13)
    la, lo = latlon.tm_inverse(np.zeros_like(y), y, 7.5, K0, R)
    np.testing.assert_allclose(lo, 7.5, atol=1e-12)
    np.testing.assert_allclose(la, y / (K0 * R) / latlon.DEG, atol=1e-9)


def test_eq11_is_the_local_scale_of_the_projection():
    """Conformal: the scale along a meridian, |d(x, y)/dphi| / R, equals the
    k of Eq. 11 at that easting."""
    for lat, lon in [(40.0, -3.0), (40.0, 1.0), (55.0, 3.5), (-20.0, -7.0)]:
        h = 1e-6
        x0, y0 = latlon.tm_forward(lat - h, lon, -3.0, K0, R)
        x1, y1 = latlon.tm_forward(lat + h, lon, -3.0, K0, R)
        scale = np.hypot(x1 - x0, y1 - y0) / (2 * h * latlon.DEG * R)
        xm, _ = latlon.tm_forward(lat, lon, -3.0, K0, R)
        assert scale == pytest.approx(float(latlon.scale_factor(xm, K0, R)), rel=1e-8)


def test_nearest_neighbour_matches_brute_force_search():
    rng = np.random.default_rng(3)
    nlat, nlon, dlat, dlon = 60, 80, 0.01, 0.012
    lat_first, lon_first = 41.0, -3.45
    src = rng.random((nlat, nlon))
    ny, nx, pitch = 25, 30, 1.7
    x_first, y_first = -22.0, 4555.0
    out, rowf, colf = latlon.reproject_nn(src, lat_first, lon_first, dlat, dlon, ny, nx,
                                          x_first, y_first, pitch, -3.0, K0, R)
    lat_c = lat_first - dlat * np.arange(nlat)
    lon_c = lon_first + dlon * np.arange(nlon)
    inside = 0
    for i in range(ny):
        for j in range(nx):
            la, lo = latlon.tm_inverse(x_first + j * pitch, y_first - i * pitch, -3.0, K0, R)
            r = int(np.argmin(np.abs(lat_c - la)))
            c = int(np.argmin(np.abs(lon_c - lo)))
            in_grid = (abs(lat_c[r] - la) <= dlat / 2) and (abs(lon_c[c] - lo) <= dlon / 2)
            if in_grid:
                inside += 1
                assert out[i, j] == src[r, c]
            else:
                assert out[i, j] == 0.0
    assert inside > ny * nx // 2


def test_ground_area_factor():
    src = np.ones((400, 400))
    out, _, _ = latlon.reproject_nn(src, 45.0, -5.0, 0.01, 0.01, 5, 5, 100.0, 4900.0, 1.0,
                                    -3.0, K0, R, ground_area=True)
    x = 100.0 + np.arange(5)
    np.testing.assert_allclose(out, np.broadcast_to(1.0 / latlon.scale_factor(x, K0, R) ** 2, (5, 5)))


def test_band_kernel_geometry():
    radial = lambda d: np.exp(-d / 50.0)
    K0_eq = latlon.band_kernel(radial, 0.0, 0.01, 0.01, 3, 4, R)
    a = np.arange(-3, 4)[:, None]
    b = np.arange(-4, 5)[None, :]
    step = R * 0.01 * latlon.DEG
    np.testing.assert_allclose(K0_eq, np.exp(-step * np.sqrt(a * a + b * b) / 50.0), rtol=1e-14)
    K60 = latlon.band_kernel(radial, 60.0, 0.01, 0.01, 3, 4, R)
    # at 60 degrees an east-west step is half as long: column 2b of K60 ... row 0 matches column b of the equator kernel with half steps
    np.testing.assert_allclose(K60[3, 4 + 2], K0_eq[3, 4 + 1], rtol=1e-12)
    np.testing.assert_allclose(K60[:, 4], K0_eq[:, 4], rtol=1e-14)


def _alr_constants():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "eq12_13_alr.txt"))
            if l.strip() and not l.startswith("#")]
    return {k: float(v) for k, v in rows}


def test_alr_kernel_eq12_13():
    """Eqs. 12-13 at the points where they reduce to closed forms, with the
    constants printed in the paper (fixture): d = 1 km, where ln d = 0 so
    K = c whatever alpha is; d = d0 = 350 km, where alpha = 2.3 exactly; the
    d -> 0 limit (alpha -> 0, K -> c); the cut at the 300 km validity range."""
    g = _alr_constants()
    c = 1.0 / g["c_denominator"]
    assert synth.ALR_C == c
    pitch = 0.5
    half = int(round(g["d0_km"] / pitch))          # the grid reaches d = 350 km on each axis
    K = synth.psf_alr(half, pitch, radius_km=None)
    assert K.shape == (2 * half + 1, 2 * half + 1)
    assert K[half, half] == c                      # finite limit at d -> 0
    one_km = int(round(1.0 / pitch))
    for a, b in ((0, one_km), (one_km, 0), (0, -one_km), (-one_km, 0)):
        assert K[half + a, half + b] == pytest.approx(c, rel=1e-15)   # d = 1 km: d^-alpha = 1
    k350 = c * g["d0_km"] ** -g["a0"]                                 # alpha(d0) = a0
    for a, b in ((0, half), (half, 0), (0, -half), (-half, 0)):
        assert K[half + a, half + b] == pytest.approx(k350, rel=1e-13)
    # alpha(d) < a0 below d0, so K(d) > c d^-a0 there, and the reverse above
    d = pitch * np.arange(3, half)
    row = K[half, half + 3:2 * half]
    assert np.all(row > c * d ** -g["a0"])
    # decreasing beyond 1 km (below it ln d < 0 and the kernel rises from c)
    full_row = K[half, half:]
    assert np.all(np.diff(full_row[2:]) < 0) and full_row[1] > full_row[0]
    # symmetric in both axes (radial)
    np.testing.assert_array_equal(K, K[::-1, :])
    np.testing.assert_array_equal(K, K.T)
    # the disk cut at the validity range of Eqs. 12-13
    Kc = synth.psf_alr(half, pitch)
    r = pitch * np.hypot(*np.meshgrid(np.arange(-half, half + 1), np.arange(-half, half + 1), indexing="ij"))
    assert np.all(Kc[r > g["valid_to_km"]] == 0.0)
    np.testing.assert_array_equal(Kc[r <= g["valid_to_km"]], K[r <= g["valid_to_km"]])


def _bands_brute_force(L, edges, kernels):
    """Pure-Python sums: output pixel (i, j) takes the kernel of the band that
    holds output row i and sums it over the whole map (Eq. 7, zero outside)."""
    ny, nx = L.shape
    S = np.zeros((ny, nx))
    for i in range(ny):
        t = next(t for t in range(len(kernels)) if edges[t] <= i < edges[t + 1])
        K = kernels[t]
        ky, kx = K.shape
        cy, cx = (ky - 1) // 2, (kx - 1) // 2
        for j in range(nx):
            s = 0.0
            for a in range(ky):
                for b in range(kx):
                    r, q = i + cy - a, j + cx - b
                    if 0 <= r < ny and 0 <= q < nx:
                        s += K[a, b] * float(L[r, q])
            S[i, j] = s
    return S


@pytest.mark.parametrize("edges,shapes", [
    ((0, 3, 7, 12), ((3, 5), (5, 3), (7, 7))),
    ((0, 1, 5, 5, 12), ((3, 3), (4, 6), (5, 5), (1, 9))),   # an empty band, an even kernel
    ((0, 12), ((5, 7),)),
])
def test_latitude_band_dispatch_brute_force(edges, shapes):
    """Sec. 4: each output row uses its own band's kernel over the whole map,
    so rows next to a band edge draw on the neighbouring band's pixels."""
    rng = np.random.default_rng(len(edges))
    L = rng.random((12, 9)).astype(np.float32)
    # kernels of very different magnitude, so a row given its neighbour's kernel fails
    kernels = [rng.random(s) * 10.0 ** t for t, s in enumerate(shapes)]
    want = _bands_brute_force(L, edges, kernels)
    idx = rng.permutation(L.size)
    got = latlon.conv_latitude_bands_pixels(L, list(edges), kernels, idx)
    np.testing.assert_allclose(got, want.ravel()[idx], rtol=1e-13, atol=0)
    # a single band is the plain "same" convolution
    if len(shapes) == 1:
        import oracle
        np.testing.assert_allclose(got, oracle.conv_same(L, kernels[0]).ravel()[idx], rtol=1e-13)
