"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerance (from the target statement of the method): relative L2 error
<= 1e-5 and max |error| <= 1e-5 * max |S|, element by element on the same
seeded inputs.  Full fields at sizes the oracle finishes in seconds (spanning
several workgroup tiles and a ragged tail); sampled pixels at full workload
sizes.
"""
import numpy as np
import pytest

import oracle
from oracle import spectrum
from paper_1907_02891_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU test without a GPU"
    return t


@pytest.fixture(scope="module")
def lp(torch):
    from paper_1907_02891_amd import lp as _lp
    return _lp


def gpu_run(lp, torch, R, K, padding=None, adjoint=False):
    plan = lp.make_plan(K, *R.shape, padding=padding)
    x = torch.from_numpy(np.ascontiguousarray(R, np.float32)).cuda()
    y = plan.adjoint(x) if adjoint else plan.convolve(x)
    torch.cuda.synchronize()
    return y.cpu().numpy(), plan


def assert_parity(S, ref, tol=TOL, label=""):
    e2, em = oracle.rel_l2(S, ref), oracle.max_err_frac(S, ref)
    print(f"{label} rel-L2 {e2:.3e} max-err/max|S| {em:.3e}", flush=True)
    assert e2 <= tol and em <= tol, (label, e2, em)
    return e2, em


def sym_kernel(rng, ky, kx):
    """Kernel with K(cy+d, cx+e) = Q(|d|, |e|): bitwise mirror-symmetric on
    both axes when ky and kx are odd."""
    cy, cx = ky // 2, kx // 2
    Q = rng.random((cy + 1, cx + 1))
    return Q[np.abs(np.arange(ky) - cy)][:, np.abs(np.arange(kx) - cx)]


# ------------------------------------------------------------- small config --

def test_small_workload_full_field(lp, torch):
    R, K = synth.small_inputs()
    S, plan = gpu_run(lp, torch, R, K, padding=(512, 512))
    assert plan.form == lp.FORM_REAL_QUADRANT
    assert_parity(S, oracle.conv_same(R, K), label="small 256^2 P=512")


def test_padding_independence(lp, torch):
    R, K = synth.small_inputs()
    S512, _ = gpu_run(lp, torch, R, K, padding=(512, 512))
    S360, p = gpu_run(lp, torch, R, K)
    assert p.padding == (360, 360)
    ref = oracle.conv_same(R, K)
    assert_parity(S360, ref, label="small 256^2 P=360")
    assert oracle.rel_l2(S360, S512) <= 2 * TOL


SHAPES = [  # ny, nx, ky, kx, symmetric kernel
    (37, 53, 9, 7, False), (64, 64, 5, 5, True), (100, 37, 31, 17, False),
    (5, 300, 3, 41, True), (300, 5, 41, 3, False), (17, 13, 25, 31, False),
    (1, 1, 1, 1, True), (2, 3, 2, 2, False), (129, 257, 64, 64, False),
    (250, 250, 101, 101, True), (333, 71, 1, 1, True), (96, 200, 11, 1, False),
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{s[0]}x{s[1]}k{s[2]}x{s[3]}{'s' if s[4] else 'g'}" for s in SHAPES])
def test_ragged_shapes_full_field(lp, torch, shape):
    ny, nx, ky, kx, sym = shape
    rng = np.random.default_rng(100 + ny + 7 * nx + 3 * ky)
    R = synth.radiance_map(ny, nx, 3, 0.05, (1.0, 4.0), rng) + rng.random((ny, nx)).astype(np.float32)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    S, plan = gpu_run(lp, torch, R, K)
    assert plan.form == (lp.FORM_REAL_QUADRANT if sym and ky % 2 and kx % 2 else lp.FORM_COMPLEX)
    assert_parity(S, oracle.conv_same(R, K), label=str(shape))


PADS = [(27, 54), (25, 50), (32, 64), (30, 60), (48, 96), (75, 150), (64, 128), (81, 162),
        (125, 250), (40, 160), (45, 90), (128, 256), (243, 486), (375, 1000), (512, 2)]


@pytest.mark.parametrize("pad", PADS, ids=[f"{a}x{b}" for a, b in PADS])
def test_every_radix_mix(lp, torch, pad):
    """Padded sizes whose factorisations use radix 2, 3, 4, 5 and 8 passes."""
    py, px = pad
    rng = np.random.default_rng(py * 1000 + px)
    ny, nx = max(1, py - 6), max(1, px - 4)
    ky, kx = min(7, py - ny + 1), min(5, px - nx + 1)
    R = rng.random((ny, nx)).astype(np.float32)
    K = rng.random((ky, kx))
    S, plan = gpu_run(lp, torch, R, K, padding=pad)
    assert plan.padding == pad
    assert_parity(S, oracle.conv_same(R, K), label=f"pad {pad}")


# ---------------------------------------------------------------- spectrum --

@pytest.mark.parametrize("case", [(9, 7, 24, 20, False), (11, 11, 30, 40, True),
                                  (6, 5, 27, 50, False), (101, 101, 360, 360, True)])
def test_spectrum_matches_oracle_dft(lp, torch, case):
    ky, kx, py, px, sym = case
    rng = np.random.default_rng(ky * kx + py)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx)) - 0.3
    plan = lp.Plan(py - ky + 1, px - kx + 1, ky, kx, padding=(py, px))
    plan.bind()
    plan.set_kernel(K)
    got = plan.read_spectrum()
    ref = spectrum.kernel_spectrum(K, py, px)[:, : px // 2 + 1] / (py * px)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"spectrum {case}: max err / max {err:.2e}")
    assert err <= 2e-7
    assert plan.form == (lp.FORM_REAL_QUADRANT if sym else lp.FORM_COMPLEX)


# ------------------------------------------------------------------ adjoint --

@pytest.mark.parametrize("shape", [(40, 52, 9, 6, False), (64, 64, 7, 7, True), (33, 90, 12, 21, False)])
def test_adjoint_full_field(lp, torch, shape):
    ny, nx, ky, kx, sym = shape
    rng = np.random.default_rng(ny + nx)
    G = (rng.random((ny, nx)) - 0.5).astype(np.float32)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    A, _ = gpu_run(lp, torch, G, K, adjoint=True)
    assert_parity(A, oracle.adjoint_same(G, K), label=f"adjoint {shape}")


def test_adjoint_dot_product(lp, torch):
    rng = np.random.default_rng(5)
    ny, nx, ky, kx = 70, 45, 13, 8
    K = rng.random((ky, kx))
    R = rng.random((ny, nx)).astype(np.float32)
    G = rng.random((ny, nx)).astype(np.float32)
    plan = lp.make_plan(K, ny, nx)
    CR = plan.convolve(torch.from_numpy(R).cuda()).cpu().numpy().astype(np.float64)
    CtG = plan.adjoint(torch.from_numpy(G).cuda()).cpu().numpy().astype(np.float64)
    lhs, rhs = np.vdot(CR, G), np.vdot(R, CtG)
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


# -------------------------------------------------------------- invariants --

def test_delta_source_reproduces_kernel(lp, torch):
    rng = np.random.default_rng(6)
    ny, nx, ky, kx = 60, 70, 15, 11
    K = rng.random((ky, kx))
    p, q = 20, 33
    R = np.zeros((ny, nx), np.float32)
    R[p, q] = 1.0
    S, _ = gpu_run(lp, torch, R, K)
    cy, cx = (ky - 1) // 2, (kx - 1) // 2
    ref = np.zeros((ny, nx))
    ref[p - cy:p - cy + ky, q - cx:q - cx + kx] = K
    assert np.max(np.abs(S - ref)) <= 1e-6 * K.max()


def test_deterministic_and_in_place(lp, torch):
    R, K = synth.small_inputs()
    plan = lp.make_plan(K, *R.shape, padding=(512, 512))
    x = torch.from_numpy(R).cuda()
    a = plan.convolve(x).cpu().numpy()
    b = plan.convolve(x).cpu().numpy()
    assert np.array_equal(a, b)
    y = x.clone()
    plan.convolve(y, out=y)
    assert np.array_equal(y.cpu().numpy(), a)


def test_side_stream_ordering(lp, torch):
    """A plan bound to the default stream, called under a side stream that
    has just written its input and reads the output right after: the binding
    orders the bound stream after the side stream and back, so the result is
    the oracle's (and the same bits as on the bound stream)."""
    R, K = synth.small_inputs()
    plan = lp.make_plan(K, *R.shape, padding=(512, 512))
    x0 = torch.from_numpy(R).cuda()
    want = plan.convolve(x0).cpu().numpy()
    side = torch.cuda.Stream()
    for _ in range(3):
        with torch.cuda.stream(side):
            # a long chain of queued work that writes the input on the side stream
            x = torch.zeros_like(x0)
            for _ in range(50):
                x.add_(x0)
            x.mul_(1.0 / 50.0)
            y = plan.convolve(x)
            z = y * 2.0          # consumer queued on the side stream
            del x                # freed while the bound stream may still hold it
        side.synchronize()
        torch.cuda.synchronize()
        assert_parity(y.cpu().numpy(), oracle.conv_same(R, K), label="side stream")
        np.testing.assert_array_equal(z.cpu().numpy(), 2.0 * y.cpu().numpy())
    np.testing.assert_allclose(y.cpu().numpy(), want, rtol=1e-6, atol=1e-6 * np.abs(want).max())


def test_linearity_and_sum(lp, torch):
    rng = np.random.default_rng(8)
    ny, nx, ky, kx = 90, 80, 21, 21
    K = sym_kernel(rng, ky, kx)
    R1 = np.zeros((ny, nx), np.float32)
    R1[15:75, 15:65] = rng.random((60, 50))
    R2 = np.zeros((ny, nx), np.float32)
    R2[12:70, 20:60] = rng.random((58, 40))
    plan = lp.make_plan(K, ny, nx)
    f = lambda r: plan.convolve(torch.from_numpy(np.ascontiguousarray(r, np.float32)).cuda()).cpu().numpy().astype(np.float64)
    S1, S2, S12 = f(R1), f(R2), f(2.0 * R1 + 0.5 * R2)
    assert oracle.rel_l2(S12, 2.0 * S1 + 0.5 * S2) <= 1e-6
    # zero margin >= (k-1)/2: the "same" window holds the whole sum
    assert S1.sum() == pytest.approx(R1.astype(np.float64).sum() * K.sum(), rel=1e-5)


# ------------------------------------------- specialised register kernels --

SPEC_CASES = [  # ny, nx, ky, kx, padding, symmetric
    (200, 64, 9, 9, (512, 80), True), (300, 40, 11, 5, (512, 48), False),
    (2870, 30, 11, 7, (2880, 36), True), (1000, 24, 101, 3, (2880, 30), False),
    (4096, 16, 1201, 3, (5400, 18), True), (3500, 12, 801, 1, (5400, 12), False),
]


@pytest.mark.parametrize("case", SPEC_CASES, ids=[f"py{c[4][0]}-{c[0]}x{c[1]}{'s' if c[5] else 'g'}" for c in SPEC_CASES])
def test_specialised_column_kernel(lp, torch, case):
    """Columns of the specialised lengths (512, 2880, 5400) against the oracle
    and against the generic LDS kernel, forward and adjoint."""
    ny, nx, ky, kx, pad, sym = case
    rng = np.random.default_rng(ny * 7 + nx)
    R = rng.random((ny, nx)).astype(np.float32)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    spec = lp.make_plan(K, ny, nx, padding=pad)
    assert spec.kernels == lp.KERNELS_SPECIALISED
    gen = lp.make_plan(K, ny, nx, padding=pad, kernels=lp.KERNELS_GENERIC)
    assert gen.kernels == lp.KERNELS_GENERIC
    x = torch.from_numpy(R).cuda()
    a, b = spec.convolve(x).cpu().numpy(), gen.convolve(x).cpu().numpy()
    assert_parity(a, oracle.conv_same(R, K), label=f"spec {case}")
    assert oracle.rel_l2(a, b) <= 2 * TOL
    g = spec.adjoint(x).cpu().numpy()
    assert_parity(g, oracle.adjoint_same(R, K), label=f"spec adjoint {case}")


ROW_CASES = [  # ny, nx, ky, kx, padding, symmetric
    (9, 4099, 3, 101, (12, 5400), False), (10, 4096, 5, 1201, (15, 5400), True),
    (7, 2048, 3, 801, (9, 2880), True), (6, 2871, 1, 9, (6, 2880), False),
    (33, 257, 5, 101, (40, 512), True), (30, 500, 3, 13, (32, 512), False),
]


@pytest.mark.parametrize("case", ROW_CASES, ids=[f"px{c[4][1]}-{c[0]}x{c[1]}{'s' if c[5] else 'g'}" for c in ROW_CASES])
def test_specialised_row_kernels(lp, torch, case):
    """Rows of the specialised half lengths (256, 1440, 2700), odd and even
    widths, row counts not a multiple of the rows per workgroup."""
    ny, nx, ky, kx, pad, sym = case
    rng = np.random.default_rng(ny * 13 + nx)
    R = rng.random((ny, nx)).astype(np.float32)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    spec = lp.make_plan(K, ny, nx, padding=pad)
    assert spec.kernels == lp.KERNELS_SPECIALISED
    gen = lp.make_plan(K, ny, nx, padding=pad, kernels=lp.KERNELS_GENERIC)
    x = torch.from_numpy(R).cuda()
    a, b = spec.convolve(x).cpu().numpy(), gen.convolve(x).cpu().numpy()
    assert_parity(a, oracle.conv_same(R, K), label=f"rows {case}")
    assert oracle.rel_l2(a, b) <= 2 * TOL
    g = spec.adjoint(x).cpu().numpy()
    assert_parity(g, oracle.adjoint_same(R, K), label=f"rows adjoint {case}")


# ------------------------------------------------------ every tuned variant --

VARIANT_CASES = [  # ny, nx, ky, kx, padding, symmetric
    (37, 4093, 5, 401, (48, 5400), True), (4096, 9, 1201, 3, (5400, 12), False),
    (11, 2049, 3, 801, (16, 2880), False), (2700, 7, 101, 3, (2880, 10), True),
    (29, 255, 9, 3, (40, 512), False), (400, 15, 31, 1, (512, 16), True),
    (1000, 11, 201, 3, (1200, 12), True), (7, 1000, 3, 201, (8, 1200), False),
    (1300, 5, 141, 1, (1440, 6), False), (9, 1300, 3, 141, (10, 1440), True),
    (1500, 6, 101, 3, (1600, 8), True), (5, 1500, 1, 101, (6, 1600), False),
    (1800, 3, 121, 1, (1920, 4), False), (3, 1800, 1, 121, (4, 1920), True),
    (5, 17000, 3, 1201, (8, 18432), False), (17000, 5, 1201, 3, (18432, 8), True),
    (4500, 7, 301, 3, (4800, 8), False), (7, 4500, 3, 301, (8, 4800), True),
    (7, 26990, 3, 21, (8, 27000), False),
    (12001, 5, 1401, 3, (13500, 8), True), (5, 12001, 3, 1401, (8, 13500), False),
    # row lengths of the batched tiles with two, four and eight rows per
    # workgroup (row counts that leave a partial last tile)
    (9, 1700, 3, 101, (10, 1800), True), (10, 1900, 3, 141, (12, 2048), False),
    (11, 2000, 3, 121, (12, 2160), True), (13, 2400, 3, 181, (15, 2592), False),
    (9, 3100, 3, 121, (10, 3240), True), (17, 3400, 3, 181, (18, 3600), False),
    (9, 4100, 3, 201, (10, 4320), True),
]


@pytest.mark.parametrize("case", VARIANT_CASES, ids=[f"p{c[4][0]}x{c[4][1]}" for c in VARIANT_CASES])
def test_every_variant(lp, torch, case):
    """Every compiled variant of every specialised stage, forward and adjoint."""
    ny, nx, ky, kx, pad, sym = case
    rng = np.random.default_rng(ny + 3 * nx)
    R = rng.random((ny, nx)).astype(np.float32)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    ref = oracle.conv_same(R, K)
    refa = oracle.adjoint_same(R, K)
    plan = lp.make_plan(K, ny, nx, padding=pad)
    x = torch.from_numpy(R).cuda()
    nvar = 0
    for stage in (lp.STAGE_ROWS, lp.STAGE_COLUMNS):
        for k in range(plan.variant_count(stage)):
            plan.set_variant(stage, k)
            info = plan.variant_info(stage, k)
            assert_parity(plan.convolve(x).cpu().numpy(), ref, label=f"{case} stage {stage} v{k} {info}")
            assert_parity(plan.adjoint(x).cpu().numpy(), refa, label=f"adj {case} stage {stage} v{k}")
            nvar += 1
        if plan.variant_count(stage):
            plan.set_variant(stage, 0)
    # the two row directions on different variants (separate twiddle tables)
    n = plan.variant_count(lp.STAGE_ROWS)
    for k in range(n if n > 1 else 0):
        plan.set_variant(lp.STAGE_ROWS, k)
        plan.set_variant(lp.STAGE_ROWS_INVERSE, (k + 1) % n)
        assert plan.variant(lp.STAGE_ROWS) == k and plan.variant(lp.STAGE_ROWS_INVERSE) == (k + 1) % n
        assert_parity(plan.convolve(x).cpu().numpy(), ref, label=f"{case} rows fwd v{k} inv v{(k + 1) % n}")
        assert_parity(plan.adjoint(x).cpu().numpy(), refa, label=f"adj {case} rows fwd v{k} inv v{(k + 1) % n}")
    assert nvar >= 1


def test_autotune_picks_a_variant(lp, torch, tmp_path, monkeypatch):
    from paper_1907_02891_amd import tune
    monkeypatch.setenv("LP_TUNE_CACHE", str(tmp_path / "tune.json"))
    R, K = synth.small_inputs()
    plan = lp.make_plan(K, *R.shape, padding=(512, 512))
    x = torch.from_numpy(R).cuda()
    rep = tune.autotune(plan, x, reps=3, warmup=1)
    assert set(rep) == {"rows", "columns"}
    assert_parity(plan.convolve(x).cpu().numpy(), oracle.conv_same(R, K), label="tuned small")
    rep2 = tune.autotune(plan, x, reps=3, warmup=1)
    assert rep2["rows"]["variant"] == rep["rows"]["variant"]


# ----------------------------------------------- input-sized window padding --

WINDOW_CASES = [  # ny, nx, ky, kx, padding (>= n + floor(k/2), 5-smooth, px even), kernels
    (250, 250, 101, 101, (300, 300), "auto"),      # exactly n + floor(k/2)
    (256, 256, 101, 101, (320, 320), "auto"),
    (100, 120, 20, 31, (120, 144), "auto"),        # even kernel rows
    (4096, 16, 1201, 3, (4800, 18), "auto"),       # specialised 4800-point columns
    (9, 4096, 3, 1201, (12, 4800), "auto"),        # specialised 2400-point rows
    (4096, 16, 1201, 3, (4800, 18), "generic"),
]


@pytest.mark.parametrize("case", WINDOW_CASES, ids=[f"{c[0]}x{c[1]}p{c[4][0]}x{c[4][1]}{c[5][0]}" for c in WINDOW_CASES])
def test_window_padding_full_field(lp, torch, case):
    """Padding below n + k - 1 but >= n + floor(k/2): the input-sized window
    is unchanged (a wrapped tap lands in the zero padding)."""
    ny, nx, ky, kx, pad, kern = case
    rng = np.random.default_rng(ny + 3 * nx + ky)
    R = rng.random((ny, nx)).astype(np.float32)
    K = rng.random((ky, kx))
    plan = lp.make_plan(K, ny, nx, padding=pad,
                        kernels=lp.KERNELS_GENERIC if kern == "generic" else lp.KERNELS_AUTO)
    assert plan.padding == pad
    if kern == "auto" and pad[0] == 4800:
        assert plan.kernels == lp.KERNELS_SPECIALISED
    x = torch.from_numpy(R).cuda()
    S = plan.convolve(x).cpu().numpy()
    assert_parity(S, oracle.conv_same(R, K), label=f"window {case}")
    G = (rng.random((ny, nx)) - 0.5).astype(np.float32)
    A = plan.adjoint(torch.from_numpy(G).cuda()).cpu().numpy()
    assert_parity(A, oracle.adjoint_same(G, K), label=f"window adjoint {case}")


# ---------------------------------------------------------- maximum sizes --

MAX_CASES = [  # ny, nx, ky, kx, padding: the longest single-tile column and the longest row
    (19000, 4, 1481, 3, (20480, 6)),     # Py = 20480: one column fills the 160 KB of LDS
    (3, 39000, 3, 1501, (4, 40500)),     # Px = 40500: largest even 5-smooth length <= LP_MAX_PX
    (19500, 4, 1481, 3, None),           # n + k - 1 = 20980 > 20480: the default 21600 takes four-step columns
]
# (the longest four-step column, Py = LP_MAX_PY = 131072, is a case of test_gpu_long.py)


@pytest.mark.parametrize("case", MAX_CASES, ids=["py20480", "px40500", "py-default"])
def test_maximum_sizes_full_field(lp, torch, case):
    ny, nx, ky, kx, pad = case
    rng = np.random.default_rng(ny + nx)
    R = rng.random((ny, nx)).astype(np.float32)
    K = rng.random((ky, kx))
    plan = lp.make_plan(K, ny, nx, padding=pad)
    if pad is not None:
        assert plan.padding == pad
    assert plan.padding[0] <= lp.MAX_PY and plan.padding[1] <= lp.MAX_PX
    if pad is None:
        assert plan.padding[0] == 21600 and plan.column_split[0] > 1
    y = plan.convolve(torch.from_numpy(R).cuda()).cpu().numpy()
    assert_parity(y, oracle.conv_same(R, K), label=f"max size {case} P={plan.padding}")
