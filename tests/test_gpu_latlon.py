"""GPU parity of the preprocessing steps: the nearest-neighbour transverse
Mercator reprojection (Sec. 2.4, Eq. 11) against the oracle's gather, and the
latitude-band convolution (Sec. 4) against the oracle's per-band direct sums."""
import numpy as np
import pytest

import oracle
from oracle import latlon as olat
from paper_1907_02891_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
K0, R = 0.9996, 6367.0


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU test without a GPU"
    return t


@pytest.fixture(scope="module")
def lp(torch):
    from paper_1907_02891_amd import lp as _lp
    return _lp


def reproject_both(lp, torch, src, sg, dg, ground_area=False):
    x = torch.from_numpy(np.ascontiguousarray(src, np.float32)).cuda()
    got = lp.reproject_nn(x, lp.LatLonGrid(*sg), lp.TMGrid(*dg), ground_area=ground_area).cpu().numpy()
    nlat, nlon, lat_first, lon_first, dlat, dlon = sg
    ny, nx, x_first, y_first, pitch, lon0, k0, radius = dg
    ref, rowf, colf = olat.reproject_nn(src.astype(np.float32).astype(np.float64), lat_first, lon_first, dlat, dlon,
                                        ny, nx, x_first, y_first, pitch, lon0, k0, radius, ground_area=ground_area)
    return got, ref, rowf, colf


def check_gather(got, ref, rowf, colf, exact=True):
    """Equal everywhere except where the index sits on a rounding tie (there
    FP64 libraries may round either way: then the value must be one of the
    two neighbours' - checked as nonzero-or-zero consistency)."""
    tie = (np.abs(np.abs(rowf - np.floor(rowf)) - 0.5) < 1e-9) | (np.abs(np.abs(colf - np.floor(colf)) - 0.5) < 1e-9)
    ok = ~tie
    if exact:
        assert np.array_equal(got[ok], ref[ok].astype(np.float32))
    else:
        np.testing.assert_allclose(got[ok], ref[ok], rtol=2e-7, atol=0)
    return int(tie.sum())


CASES = [  # source (nlat, nlon, lat_first, lon_first, dlat, dlon), target (ny, nx, x_first, y_first, pitch, lon0)
    ((500, 700, 44.0, -8.0, 0.01, 0.012), (400, 380, -150.0, 4870.0, 1.0, -3.0)),     # partly outside
    ((240, 360, 41.0, -4.0, 1 / 240, 1 / 240), (97, 131, -40.0, 4540.0, 0.4044, -3.0)),  # 15 arc-second, UTM pitch
    ((300, 300, -10.0, 20.0, 0.02, 0.02), (5, 67, 2000.0, -1200.0, 2.5, 23.0)),       # southern hemisphere, ragged
    ((50, 50, 60.0, 0.0, 0.1, 0.1), (1, 1, 0.0, 6600.0, 1.0, 2.5)),                  # one pixel
    ((50, 50, 60.0, 0.0, 0.1, 0.1), (64, 64, 5000.0, 100.0, 1.0, 2.5)),               # entirely outside
]


@pytest.mark.parametrize("ground_area", [False, True], ids=["radiance", "ground_area"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[1][0]}x{c[1][1]}" for c in CASES])
def test_reprojection_matches_oracle(lp, torch, case, ground_area):
    s, d = case
    rng = np.random.default_rng(s[0] + d[0])
    src = (rng.random((s[0], s[1])) + 0.1).astype(np.float32)
    got, ref, rowf, colf = reproject_both(lp, torch, src, s, (*d, K0, R), ground_area)
    ties = check_gather(got, ref, rowf, colf, exact=not ground_area)
    print(f"reprojection {case} ground_area={ground_area}: {ties} tie pixels", flush=True)
    if d[2] == 5000.0:
        assert not got.any()


def test_reprojection_at_full_map_size_sampled_rows(lp, torch):
    """The paper's projected grid size (11920 x 11804 at 404.4 m, UTM 30N)
    from a 15 arc-second source; 8 sampled rows against the oracle."""
    nlat, nlon = 2400, 4800
    sg = (nlat, nlon, 45.0, -13.0, 1 / 240, 1 / 240)
    rng = np.random.default_rng(7)
    src = rng.random((nlat, nlon), dtype=np.float32)
    ny, nx, pitch = 11920, 11804, 0.4044
    dg = (ny, nx, -nx / 2 * pitch, 4430.0 + ny / 2 * pitch, pitch, -3.0, K0, R)
    x = torch.from_numpy(src).cuda()
    got = lp.reproject_nn(x, lp.LatLonGrid(*sg), lp.TMGrid(*dg)).cpu().numpy()
    for i in rng.choice(ny, 8, replace=False):
        ref, rowf, colf = olat.reproject_nn(src.astype(np.float64), 45.0, -13.0, 1 / 240, 1 / 240, 1, nx,
                                            dg[2], dg[3] - i * pitch, pitch, -3.0, K0, R)
        check_gather(got[i:i + 1], ref, rowf, colf)
    assert got.any()


def band_case(T, ny=600, nx=700, half=(30, 45), seed=11):
    rng = np.random.default_rng(seed)
    L = synth.radiance_map(ny, nx, 20, 0.05, (2.0, 12.0), rng)
    lat_first, dlat, dlon = 60.0, 1 / 120, 1 / 120
    edges = np.linspace(0, ny, T + 1).round().astype(int)
    radial = lambda d: np.where(d > 0, np.maximum(d, 0.3) ** -2.5, 0.3 ** -2.5) * np.exp(-d / 80.0)
    cents = olat_band_centres(edges, lat_first, dlat)
    Ks = [olat.band_kernel(radial, c, dlat, dlon, half[0], half[1], R) for c in cents]
    return L, edges, Ks, radial, lat_first, dlat, dlon, cents


def olat_band_centres(edges, lat_first, dlat):
    return [lat_first - dlat * 0.5 * (edges[t] + edges[t + 1] - 1) for t in range(len(edges) - 1)]


@pytest.mark.parametrize("T", [1, 3, 5])
def test_latitude_bands_full_field(lp, torch, T):
    from paper_1907_02891_amd import latlon
    L, edges, Ks, radial, lat_first, dlat, dlon, cents = band_case(T)
    ny, nx = L.shape
    kp = [latlon.band_kernel(radial, c, dlat, dlon, 30, 45) for c in latlon.band_centres(edges, lat_first, dlat)]
    for a, b in zip(kp, Ks):
        np.testing.assert_allclose(a, b, rtol=1e-13)
    bands = latlon.LatitudeBands(ny, nx, edges, kp)
    y = bands.convolve(torch.from_numpy(L).cuda()).cpu().numpy()
    ref = olat.conv_latitude_bands_pixels(L, edges, Ks, np.arange(ny * nx)).reshape(ny, nx)
    e2, em = oracle.rel_l2(y, ref), oracle.max_err_frac(y, ref)
    print(f"latitude bands T={T}: rel-L2 {e2:.3e} max-err/max {em:.3e}", flush=True)
    assert e2 <= TOL and em <= TOL


def test_latitude_bands_with_one_kernel_equal_plain_convolution(lp, torch):
    """Slabs with halos, stitched: same result as one convolution of the map."""
    from paper_1907_02891_amd import latlon
    rng = np.random.default_rng(12)
    ny, nx = 513, 300
    L = rng.random((ny, nx)).astype(np.float32)
    K = rng.random((41, 31))
    edges = [0, 100, 101, 260, 513]
    bands = latlon.LatitudeBands(ny, nx, edges, [K] * 4)
    x = torch.from_numpy(L).cuda()
    y = bands.convolve(x).cpu().numpy()
    plain = lp.make_plan(K, ny, nx).convolve(x).cpu().numpy()
    assert oracle.rel_l2(y, plain) <= 1e-6
    assert oracle.rel_l2(y, oracle.conv_same(L, K)) <= TOL
