"""Pins for the FP64 oracle, checked against things other than itself.

Each test ties the oracle to something the paper or the mathematics fixes:
an independent pure-Python brute force on tiny grids, a library routine for
a special case (scipy's 2-D convolution, numpy's 1-D convolution and FFT),
closed forms (delta source, constant field, sum identity) and invariants
(linearity, shift invariance, transpose identities).  The shapes cover odd
and even kernels, kernels larger than the map and non-square grids, so that a
dropped term, a flipped index or a transposed operand fails at least one.
"""
import itertools

import numpy as np
import pytest
import scipy.signal

import oracle
from oracle import spectrum

SHAPES = [  # (ny, nx, ky, kx)
    (1, 1, 1, 1), (3, 4, 1, 1), (5, 7, 3, 3), (6, 5, 4, 2), (4, 9, 5, 6),
    (3, 3, 7, 5), (2, 8, 6, 7), (9, 4, 2, 3), (7, 7, 7, 7), (12, 5, 4, 4),
]


def brute_full(R, K):
    """Four nested Python loops over Eq. 7 on the grid (no numpy arithmetic)."""
    ny, nx = len(R), len(R[0])
    ky, kx = len(K), len(K[0])
    out = [[0.0] * (nx + kx - 1) for _ in range(ny + ky - 1)]
    for i in range(ny):
        for j in range(nx):
            for a in range(ky):
                for b in range(kx):
                    out[i + a][j + b] += R[i][j] * K[a][b]
    return out


def brute_same(R, K):
    ky, kx = len(K), len(K[0])
    cy, cx = (ky - 1) // 2, (kx - 1) // 2
    full = brute_full(R, K)
    return [row[cx:cx + len(R[0])] for row in full[cy:cy + len(R)]]


def rand_pair(rng, ny, nx, ky, kx, signed=False):
    R = rng.random((ny, nx))
    K = rng.random((ky, kx))
    if signed:
        R -= 0.5
        K -= 0.5
    return R, K


@pytest.mark.parametrize("shape", SHAPES)
def test_full_matches_brute_force(shape):
    rng = np.random.default_rng(1)
    R, K = rand_pair(rng, *shape, signed=True)
    got = oracle.conv_full(R, K)
    ref = np.array(brute_full(R.tolist(), K.tolist()))
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape", SHAPES)
def test_same_matches_brute_force(shape):
    rng = np.random.default_rng(2)
    R, K = rand_pair(rng, *shape, signed=True)
    got = oracle.conv_same(R, K)
    ref = np.array(brute_same(R.tolist(), K.tolist()))
    assert got.shape == R.shape
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("shape", SHAPES + [(40, 33, 11, 9), (17, 64, 16, 15)])
def test_matches_scipy_convolve2d(shape):
    """Library routine: scipy's 'full' and 'same' use the same centre
    convention ((k-1)//2), for odd and even kernels."""
    rng = np.random.default_rng(3)
    R, K = rand_pair(rng, *shape)
    np.testing.assert_allclose(oracle.conv_full(R, K),
                               scipy.signal.convolve2d(R, K, mode="full"),
                               rtol=1e-12, atol=1e-13)
    if shape[0] >= shape[2] and shape[1] >= shape[3]:
        # scipy's 'same' crops to the larger operand; compare only when it
        # is the map.
        np.testing.assert_allclose(oracle.conv_same(R, K),
                                   scipy.signal.convolve2d(R, K, mode="same"),
                                   rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("shape", [(9, 11, 5, 3), (8, 8, 4, 6), (6, 10, 7, 7)])
def test_delta_source_reproduces_kernel(shape):
    """A unit source at (p, q) gives S(i, j) = K(i - p + cy, j - q + cx)."""
    ny, nx, ky, kx = shape
    rng = np.random.default_rng(4)
    K = rng.random((ky, kx))
    cy, cx = (ky - 1) // 2, (kx - 1) // 2
    for p, q in [(0, 0), (ny // 2, nx // 3), (ny - 1, nx - 1)]:
        R = np.zeros((ny, nx))
        R[p, q] = 1.0
        S = oracle.conv_same(R, K)
        ref = np.zeros((ny, nx))
        for i in range(ny):
            for j in range(nx):
                a, b = i - p + cy, j - q + cx
                if 0 <= a < ky and 0 <= b < kx:
                    ref[i, j] = K[a, b]
        np.testing.assert_array_equal(S, ref)
        F = oracle.conv_full(R, K)
        np.testing.assert_array_equal(F[p:p + ky, q:q + kx], K)
        assert F.sum() == pytest.approx(K.sum(), rel=1e-14)


def test_linearity():
    rng = np.random.default_rng(5)
    R1, K = rand_pair(rng, 13, 10, 5, 7)
    R2 = rng.random(R1.shape)
    al, be = 0.7, -2.25
    lhs = oracle.conv_same(al * R1 + be * R2, K)
    rhs = al * oracle.conv_same(R1, K) + be * oracle.conv_same(R2, K)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_shift_invariance():
    """A map shifted by (s, t) inside a zero margin gives a shifted output."""
    rng = np.random.default_rng(6)
    K = rng.random((5, 3))
    R = np.zeros((20, 18))
    R[6:11, 5:9] = rng.random((5, 4))
    S = oracle.conv_same(R, K)
    s, t = 3, -2
    Rs = np.roll(np.roll(R, s, 0), t, 1)
    Ss = oracle.conv_same(Rs, K)
    np.testing.assert_allclose(Ss, np.roll(np.roll(S, s, 0), t, 1), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("shape", SHAPES)
def test_sum_identity_full(shape):
    """sum S_full = sum R * sum K (the zero-frequency term of Eq. 9)."""
    rng = np.random.default_rng(7)
    R, K = rand_pair(rng, *shape)
    assert oracle.conv_full(R, K).sum() == pytest.approx(R.sum() * K.sum(), rel=1e-13)


def test_sum_identity_same_with_margin():
    rng = np.random.default_rng(8)
    K = rng.random((7, 5))
    R = np.zeros((30, 25))
    R[3:27, 2:23] = rng.random((24, 21))
    assert oracle.conv_same(R, K).sum() == pytest.approx(R.sum() * K.sum(), rel=1e-13)


def test_constant_field_interior():
    """R = c gives S = c * sum K wherever the kernel footprint is inside."""
    rng = np.random.default_rng(9)
    K = rng.random((5, 7))
    c = 3.5
    S = oracle.conv_same(np.full((16, 19), c), K)
    cy, cx = 2, 3
    inner = S[cy:16 - (5 - 1 - cy), cx:19 - (7 - 1 - cx)]
    np.testing.assert_allclose(inner, c * K.sum(), rtol=1e-14)
    assert S[0, 0] < c * K.sum()


@pytest.mark.parametrize("shape", [(15, 12, 5, 7), (9, 20, 8, 3), (6, 6, 9, 9)])
def test_separable_matches_numpy_1d(shape):
    """K = outer(u, v): the oracle's 2-D sum, its separable form, and numpy's
    1-D convolution of rows then columns all agree."""
    ny, nx, ky, kx = shape
    rng = np.random.default_rng(10)
    R = rng.random((ny, nx))
    u, v = rng.random(ky), rng.random(kx)
    K = np.outer(u, v)
    cy, cx = (ky - 1) // 2, (kx - 1) // 2
    T = np.stack([np.convolve(R[i], v, mode="full")[cx:cx + nx] for i in range(ny)])
    ref = np.stack([np.convolve(T[:, j], u, mode="full")[cy:cy + ny] for j in range(nx)], 1)
    np.testing.assert_allclose(oracle.conv_same(R, K), ref, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(oracle.conv_same_separable(R, u, v), ref, rtol=1e-12, atol=1e-14)
    idx = np.array([0, 5, ny * nx - 1, (ny // 2) * nx + nx // 2], np.int64)
    np.testing.assert_allclose(oracle.conv_same_separable_pixels(R, u, v, idx),
                               ref.ravel()[idx], rtol=1e-12, atol=1e-14)


def test_pixels_match_full_field():
    rng = np.random.default_rng(11)
    R, K = rand_pair(rng, 14, 17, 6, 5)
    idx = rng.choice(R.size, 40, replace=False)
    np.testing.assert_array_equal(oracle.conv_same_pixels(R, K, idx),
                                  oracle.conv_same(R, K).ravel()[idx])
    G = rng.random(R.shape)
    np.testing.assert_array_equal(oracle.adjoint_same_pixels(G, K, idx),
                                  oracle.adjoint_same(G, K).ravel()[idx])


@pytest.mark.parametrize("shape", [(4, 5, 3, 2), (6, 3, 4, 4), (3, 3, 5, 5)])
def test_adjoint_is_matrix_transpose(shape):
    """Build the "same" operator as an explicit matrix from the brute force
    and check the oracle's adjoint against its transpose."""
    ny, nx, ky, kx = shape
    rng = np.random.default_rng(12)
    K = rng.random((ky, kx)) - 0.5
    n = ny * nx
    M = np.zeros((n, n))
    for col in range(n):
        e = [[0.0] * nx for _ in range(ny)]
        e[col // nx][col % nx] = 1.0
        M[:, col] = np.array(brute_same(e, K.tolist())).ravel()
    G = rng.random((ny, nx)) - 0.5
    np.testing.assert_allclose(oracle.adjoint_same(G, K).ravel(), M.T @ G.ravel(),
                               rtol=1e-13, atol=1e-14)


def test_adjoint_dot_product():
    rng = np.random.default_rng(13)
    R, K = rand_pair(rng, 23, 19, 7, 8, signed=True)
    G = rng.random(R.shape) - 0.5
    lhs = np.vdot(oracle.conv_same(R, K), G)
    rhs = np.vdot(R, oracle.adjoint_same(G, K))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_symmetric_kernel_is_self_adjoint():
    rng = np.random.default_rng(14)
    A = rng.random((5, 7))
    K = A + A[::-1, :] + A[:, ::-1] + A[::-1, ::-1]
    G = rng.random((12, 10))
    np.testing.assert_allclose(oracle.adjoint_same(G, K), oracle.conv_same(G, K),
                               rtol=1e-13, atol=1e-14)


def test_adjoint_sparse_matches_dense():
    rng = np.random.default_rng(15)
    ny, nx = 16, 13
    K = rng.random((5, 6))
    sites = rng.choice(ny * nx, 9, replace=False)
    g = rng.random(9) - 0.5
    G = np.zeros(ny * nx)
    G[sites] = g
    np.testing.assert_allclose(oracle.adjoint_sparse(sites, g, (ny, nx), K),
                               oracle.adjoint_same(G.reshape(ny, nx), K),
                               rtol=1e-13, atol=1e-15)


def test_bad_arguments_raise():
    with pytest.raises(ValueError):
        oracle.conv_same_pixels(np.ones((3, 3)), np.ones((1, 1)), [9])
    with pytest.raises(ValueError):
        oracle.conv_same(np.ones((0, 3)), np.ones((1, 1)))


# ---------------------------------------------------------------- spectrum --

def brute_dft2(x):
    """Eq. 10 as a quadruple Python loop (0-based indices)."""
    import cmath
    N, M = len(x), len(x[0])
    out = [[0j] * M for _ in range(N)]
    for k, l in itertools.product(range(N), range(M)):
        s = 0j
        for n, m in itertools.product(range(N), range(M)):
            s += x[n][m] * cmath.exp(-2j * cmath.pi * (k * n / N + l * m / M))
        out[k][l] = s
    return out


@pytest.mark.parametrize("kshape,P", [((3, 3), (5, 6)), ((4, 2), (6, 5)), ((1, 1), (3, 3)),
                                      ((5, 3), (8, 9))])
def test_spectrum_matches_brute_dft(kshape, P):
    rng = np.random.default_rng(16)
    K = rng.random(kshape) - 0.5
    got = spectrum.kernel_spectrum(K, *P)
    kw = spectrum.wrap_centre(K, *P)
    np.testing.assert_allclose(got, np.array(brute_dft2(kw.tolist())), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kshape,P", [((11, 9), (30, 24)), ((6, 7), (27, 20)), ((21, 21), (64, 60))])
def test_spectrum_matches_numpy_fft(kshape, P):
    rng = np.random.default_rng(17)
    K = rng.random(kshape)
    got = spectrum.kernel_spectrum(K, *P)
    np.testing.assert_allclose(got, np.fft.fft2(spectrum.wrap_centre(K, *P)),
                               rtol=1e-10, atol=1e-11)


def test_wrap_centre_places_centre_at_origin():
    K = np.arange(15, dtype=float).reshape(3, 5)
    kw = spectrum.wrap_centre(K, 6, 8)
    assert kw[0, 0] == K[1, 2]
    assert kw[5, 7] == K[0, 1]
    assert kw[1, 2] == K[2, 4]
    assert kw.sum() == K.sum()


def test_symmetric_kernel_spectrum_is_real_and_even():
    """An even kernel (odd size, mirror-symmetric on both axes) has a real,
    even spectrum."""
    rng = np.random.default_rng(18)
    A = rng.random((9, 7))
    K = A + A[::-1, :] + A[:, ::-1] + A[::-1, ::-1]
    Py, Px = 24, 20
    F = spectrum.kernel_spectrum(K, Py, Px)
    assert np.max(np.abs(F.imag)) <= 1e-12 * np.max(np.abs(F.real))
    u = (-np.arange(Py)) % Py
    v = (-np.arange(Px)) % Px
    np.testing.assert_allclose(F.real, F.real[u][:, v], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("shape,P", [((10, 12, 5, 7), (14, 18)), ((9, 7, 6, 4), (16, 10)),
                                     ((16, 16, 9, 9), (25, 24))])
def test_convolution_theorem_reproduces_same(shape, P):
    """Eq. 9 with zero padding to at least n+k-1 (Sec. 2.5): the inverse
    transform of Khat * DFT(embedded R), cropped to the map at the origin,
    equals the direct "same" sum."""
    ny, nx, ky, kx = shape
    rng = np.random.default_rng(19)
    R, K = rand_pair(rng, ny, nx, ky, kx)
    Py, Px = P
    assert Py >= ny + ky - 1 and Px >= nx + kx - 1
    Rp = np.zeros((Py, Px))
    Rp[:ny, :nx] = R
    Kh = spectrum.kernel_spectrum(K, Py, Px)
    Fr = spectrum.dft_matrix(Py) @ Rp @ spectrum.dft_matrix(Px).T
    S = (spectrum.dft_matrix(Py, +1) @ (Kh * Fr) @ spectrum.dft_matrix(Px, +1).T) / (Py * Px)
    np.testing.assert_allclose(S.real[:ny, :nx], oracle.conv_same(R, K), rtol=1e-11, atol=1e-12)
    # conj(Khat) gives the transposed operator (the adjoint)
    Sa = (spectrum.dft_matrix(Py, +1) @ (np.conj(Kh) * Fr) @ spectrum.dft_matrix(Px, +1).T) / (Py * Px)
    np.testing.assert_allclose(Sa.real[:ny, :nx], oracle.adjoint_same(R, K), rtol=1e-11, atol=1e-12)


def test_site_loss_gradient_by_central_differences():
    """The gradient of L(R) = sum_i w_i (S(x_i) - m_i)^2 is the transposed
    operator applied to 2 w (S - m) at the sites: checked against central
    differences of the FP64 loss (exact for a quadratic loss up to round-off)."""
    rng = np.random.default_rng(20)
    ny, nx = 21, 17
    R = rng.random((ny, nx))
    K = rng.random((7, 5))
    sites = rng.choice(ny * nx, 12, replace=False)
    m = rng.random(12) + 0.5
    w = 1.0 / m ** 2

    def loss(Rx):
        r = oracle.conv_same_pixels(Rx, K, sites) - m
        return float(np.sum(w * r * r))

    g = 2.0 * w * (oracle.conv_same_pixels(R, K, sites) - m)
    grad = oracle.adjoint_sparse(sites, g, (ny, nx), K).ravel()
    h = 0.5
    for p in rng.choice(ny * nx, 30, replace=False):
        Rp = R.copy().ravel()
        Rp[p] += h
        Lp = loss(Rp.reshape(ny, nx))
        Rp[p] -= 2 * h
        Lm = loss(Rp.reshape(ny, nx))
        assert (Lp - Lm) / (2 * h) == pytest.approx(grad[p], rel=1e-9, abs=1e-11)


# ------------------------------------------------- source classes (Eq. 4) --

@pytest.mark.parametrize("shape", [(5, 7, 3, 3), (4, 9, 5, 6), (7, 7, 7, 7)])
def test_class_sum_matches_brute_force(shape):
    """Eq. 4: B = sum over classes of K_t (*) L_1t, against four Python loops
    per class."""
    rng = np.random.default_rng(11)
    Rs, Ks = zip(*[rand_pair(rng, *shape, signed=True) for _ in range(3)])
    got = oracle.conv_same_classes(Rs, Ks)
    ref = sum(np.array(brute_same(R.tolist(), K.tolist())) for R, K in zip(Rs, Ks))
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)


def test_class_sum_with_one_kernel_is_conv_of_summed_maps():
    """Classes sharing a kernel collapse to one class with the summed radiance
    (Eq. 4 reduces to Eq. 3)."""
    rng = np.random.default_rng(12)
    K = rng.random((9, 7))
    Rs = [rng.random((30, 41)) for _ in range(4)]
    got = oracle.conv_same_classes(Rs, [K] * 4)
    np.testing.assert_allclose(got, oracle.conv_same(sum(Rs), K), rtol=1e-12, atol=1e-12)


def test_class_sum_pixels_match_full_field():
    rng = np.random.default_rng(13)
    Rs = [rng.random((25, 19)) for _ in range(3)]
    Ks = [rng.random((5, 8)) for _ in range(3)]
    full = oracle.conv_same_classes(Rs, Ks).ravel()
    idx = rng.choice(full.size, 40, replace=False)
    np.testing.assert_allclose(oracle.conv_same_classes_pixels(Rs, Ks, idx), full[idx], rtol=1e-13)


def _kept_rows_need(ny, ky, k0, k1):
    """Padded length the library uses for kept output rows [k0, k1) (the
    batch's window bound): k1 + cy, and at least ny + ky - 1 - cy - k0 when
    some kept row reaches above row 0."""
    cy = (ky - 1) // 2
    return k1 + cy if k0 + cy - (ky - 1) >= 0 else max(k1 + cy, ny + ky - 1 - cy - k0)


def _same_1d(x, K, cy):
    """Direct "same" convolution along one axis (Eq. 7, zero outside)."""
    n = len(x)
    return np.array([sum(K[a] * x[i + cy - a] for a in range(len(K)) if 0 <= i + cy - a < n) for i in range(n)])


def _circular_1d(x, K, cy, P):
    """The same sums on a circle of P samples holding the first min(n, P)
    input samples (zero-extended when n < P), i.e. what a length-P transform
    of the loaded rows computes (Eq. 9); rows >= P are not loaded.  Outputs
    for i < min(n, P)."""
    xp = np.zeros(P)
    m = min(len(x), P)
    xp[:m] = x[:m]
    return np.array([sum(K[a] * xp[(i + cy - a) % P] for a in range(len(K))) for i in range(m)])


@pytest.mark.parametrize("seed", range(40))
def test_kept_rows_padding_bound_is_exact_and_tight(seed):
    """Brute force on small 1-D cases: with P = the window bound the kept
    rows of the circular convolution equal the linear ones; with P - 1 some
    kept row differs.  The whole window gives n + floor(k/2); whole halos
    give n; a window whose footprint never wraps may need fewer rows than n
    (then only the first P input rows are loaded, and the kept rows reach no
    further)."""
    rng = np.random.default_rng(seed)
    ny = int(rng.integers(3, 40))
    ky = int(rng.integers(1, 2 * ny))
    k0 = int(rng.integers(0, ny))
    k1 = int(rng.integers(k0 + 1, ny + 1))
    x = rng.random(ny) + 0.5
    K = rng.random(ky) + 0.5
    cy = (ky - 1) // 2
    need = _kept_rows_need(ny, ky, k0, k1)
    assert _kept_rows_need(ny, ky, 0, ny) == ny + ky // 2
    ref = _same_1d(x, K, cy)
    got = _circular_1d(x, K, cy, need)
    np.testing.assert_allclose(got[k0:k1], ref[k0:k1], rtol=1e-13, atol=0)
    assert need >= k1
    if need - 1 >= k1:
        bad = _circular_1d(x, K, cy, need - 1)
        assert np.max(np.abs(bad[k0:k1] - ref[k0:k1])) > 1e-6
    if k0 >= ky - 1 - cy and k1 <= ny - cy:
        assert need <= ny
    if k0 == ky - 1 - cy and k1 == ny - cy:
        assert need == ny
