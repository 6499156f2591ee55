"""GPU parity of the split-precision transforms: radix-16 passes as dense
32 x 32 real matrix products on the matrix cores, operands split into FP16
hi + lo (power-of-two block scaling) or BF16 x1 + x2 + x3, FP32 accumulation,
in the generic LDS kernels and in the register-resident 9216-point row and
18432-point column kernels.
Same bar as the FP32 path (relative L2 <= 1e-5, max |error| <= 1e-5 max |S|
against the FP64 oracle), plus a tighter check that the error stays at the
FP32 path's level."""
import numpy as np
import pytest

import oracle
from paper_1907_02891_amd import synth

pytestmark = pytest.mark.gpu

TOL = 1e-5
MODES = {"fp16x2": 1, "bf16x3": 2}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU test without a GPU"
    return t


@pytest.fixture(scope="module")
def lp(torch):
    from paper_1907_02891_amd import lp as _lp
    return _lp


def run(lp, torch, R, K, padding, precision, adjoint=False):
    plan = lp.make_plan(K, *R.shape, padding=padding, precision=precision)
    assert plan.precision == precision
    if precision and 18432 not in plan.padding:
        assert plan.kernels == lp.KERNELS_GENERIC
    x = torch.from_numpy(np.ascontiguousarray(R, np.float32)).cuda()
    y = plan.adjoint(x) if adjoint else plan.convolve(x)
    torch.cuda.synchronize()
    return y.cpu().numpy(), plan


def errors(S, ref, label):
    e2, em = oracle.rel_l2(S, ref), oracle.max_err_frac(S, ref)
    print(f"{label}: rel-L2 {e2:.3e} max-err/max {em:.3e}", flush=True)
    return e2, em


def sym_kernel(rng, ky, kx):
    cy, cx = ky // 2, kx // 2
    Q = rng.random((cy + 1, cx + 1))
    return Q[np.abs(np.arange(ky) - cy)][:, np.abs(np.arange(kx) - cx)]


# padded sizes: radix 16 alone, 16 with a 2/4/8 remainder, with 3 and 5, two
# and three radix-16 passes, and no factor 16 at all (no matrix pass)
PADS = [(16, 32), (32, 64), (48, 96), (64, 128), (128, 256), (256, 512), (80, 160),
        (240, 480), (720, 1440), (512, 1024), (4096, 32), (27, 50), (360, 360)]


@pytest.mark.parametrize("mode", MODES.values(), ids=list(MODES))
@pytest.mark.parametrize("pad", PADS, ids=[f"{a}x{b}" for a, b in PADS])
def test_split_radix_mixes(lp, torch, pad, mode):
    py, px = pad
    rng = np.random.default_rng(py * 7 + px)
    ny, nx = max(1, py - 9), max(1, px - 7)
    ky, kx = min(9, py - ny + 1), min(7, px - nx + 1)
    R = rng.random((ny, nx)).astype(np.float32)
    K = rng.random((ky, kx))
    S, plan = run(lp, torch, R, K, pad, mode)
    e2, em = errors(S, oracle.conv_same(R, K), f"split {mode} pad {pad}")
    assert e2 <= TOL and em <= TOL


SHAPES = [  # ny, nx, ky, kx, padding, symmetric kernel
    (200, 240, 57, 33, (256, 288), True), (130, 401, 31, 80, (160, 480), False),
    (500, 300, 101, 101, (640, 400), True), (61, 1000, 20, 21, (80, 1024), False),
]


@pytest.mark.parametrize("mode", MODES.values(), ids=list(MODES))
@pytest.mark.parametrize("case", SHAPES, ids=[f"{c[0]}x{c[1]}k{c[2]}" for c in SHAPES])
def test_split_matches_fp32_level(lp, torch, case, mode):
    """Error of the split path within 3x that of the FP32 path (and 1e-6)."""
    ny, nx, ky, kx, pad, sym = case
    rng = np.random.default_rng(ny * 3 + nx)
    R = synth.radiance_map(ny, nx, 4, 0.05, (2.0, 10.0), rng)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    ref = oracle.conv_same(R, K)
    S32, _ = run(lp, torch, R, K, pad, 0)
    Ssp, plan = run(lp, torch, R, K, pad, mode)
    assert plan.form == (lp.FORM_REAL_QUADRANT if sym else lp.FORM_COMPLEX)
    e32, m32 = errors(S32, ref, f"fp32 {case[:4]}")
    esp, msp = errors(Ssp, ref, f"split {mode} {case[:4]}")
    assert esp <= max(3 * e32, 1e-6) and msp <= max(3 * m32, 1e-6)


# maps whose padded rows are 18432 long (half rows 9216 = 16 x 24 x 24): the
# split forms run the register-resident row kernels with the radix-16 pass
# (the forward's first, the inverse's last) on the matrix cores
MF_ROWS = [  # ny, nx, ky, kx, symmetric kernel
    (37, 18000, 5, 401, True),    # even width, an odd number of rows (ragged last tile)
    (30, 17999, 7, 433, False),   # odd width: the last column pair is cropped to one
]


@pytest.mark.parametrize("mode", MODES.values(), ids=list(MODES))
@pytest.mark.parametrize("case", MF_ROWS, ids=[f"{c[0]}x{c[1]}" for c in MF_ROWS])
def test_split_matrix_core_rows(lp, torch, case, mode):
    ny, nx, ky, kx, sym = case
    rng = np.random.default_rng(ny + nx + mode)
    R = synth.radiance_map(ny, nx, 6, 0.05, (2.0, 10.0), rng)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    G = (rng.random((ny, nx)) - 0.5).astype(np.float32)
    plan = lp.make_plan(K, ny, nx, precision=mode)
    assert plan.padding[1] == 18432 and plan.kernels == lp.KERNELS_SPECIALISED
    x = torch.from_numpy(np.ascontiguousarray(R, np.float32)).cuda()
    g = torch.from_numpy(G).cuda()
    ref, aref = oracle.conv_same(R, K), oracle.adjoint_same(G, K)
    S32, _ = run(lp, torch, R, K, None, 0)
    e32, m32 = errors(S32, ref, f"fp32 {case[:4]}")
    n = plan.variant_count(lp.STAGE_ROWS)
    assert n >= 2  # with and without the staged intermediate
    for k in range(n):
        plan.set_variant(lp.STAGE_ROWS, k)  # both row stages
        for stage in (lp.STAGE_ROWS, lp.STAGE_ROWS_INVERSE):
            info = plan.variant_info(stage, plan.variant(stage))
            assert info["matrix_core"] and info["radices"][0] == 16, info
        S = plan.convolve(x).cpu().numpy()
        A = plan.adjoint(g).cpu().numpy()
        e2, em = errors(S, ref, f"matrix-core rows {mode} {case[:4]} variant {k}")
        assert e2 <= TOL and em <= TOL
        a2, am = errors(A, aref, f"matrix-core rows {mode} {case[:4]} variant {k} adjoint")
        assert a2 <= TOL and am <= TOL
        # and at the FP32 path's error level
        assert e2 <= max(3 * e32, 1e-6) and em <= max(3 * m32, 1e-6)


# maps whose padded columns are 18432 long: the split forms run register-
# resident column kernels with the radix-16 pass (the forward transform's
# first, the inverse's last) on the matrix cores, every variant of them
MF_COLS = [  # ny, nx, ky, kx, symmetric kernel
    (18000, 37, 401, 5, True),    # real quadrant spectrum
    (17999, 30, 433, 7, False),   # complex spectrum, odd height
]


@pytest.mark.parametrize("mode", MODES.values(), ids=list(MODES))
@pytest.mark.parametrize("case", MF_COLS, ids=[f"{c[0]}x{c[1]}" for c in MF_COLS])
def test_split_matrix_core_columns(lp, torch, case, mode):
    ny, nx, ky, kx, sym = case
    rng = np.random.default_rng(ny + nx + 10 * mode)
    R = synth.radiance_map(ny, nx, 6, 0.05, (2.0, 10.0), rng)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    G = (rng.random((ny, nx)) - 0.5).astype(np.float32)
    ref, aref = oracle.conv_same(R, K), oracle.adjoint_same(G, K)
    plan = lp.make_plan(K, ny, nx, precision=mode)
    assert plan.padding[0] == 18432 and plan.kernels == lp.KERNELS_SPECIALISED
    assert plan.form == (lp.FORM_REAL_QUADRANT if sym else lp.FORM_COMPLEX)
    x, g = (torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda() for a in (R, G))
    S32, _ = run(lp, torch, R, K, None, 0)
    e32, m32 = errors(S32, ref, f"fp32 {case[:4]}")
    n = plan.variant_count(lp.STAGE_COLUMNS)
    assert n >= 2
    for k in range(n):
        plan.set_variant(lp.STAGE_COLUMNS, k)
        info = plan.variant_info(lp.STAGE_COLUMNS, k)
        assert info["matrix_core"] and info["radices"][0] == 16, info
        S = plan.convolve(x).cpu().numpy()
        e2, em = errors(S, ref, f"matrix-core columns {mode} {case[:4]} variant {k}")
        assert e2 <= TOL and em <= TOL
        assert e2 <= max(3 * e32, 1e-6) and em <= max(3 * m32, 1e-6)
        A = plan.adjoint(g).cpu().numpy()
        a2, am = errors(A, aref, f"matrix-core columns {mode} {case[:4]} variant {k} adjoint")
        assert a2 <= TOL and am <= TOL


@pytest.mark.parametrize("mode", MODES.values(), ids=list(MODES))
def test_split_matrix_core_columns_class_sum(lp, torch, mode):
    """Eq. 4 with the split column kernels: two classes summed in registers."""
    rng = np.random.default_rng(5 + mode)
    ny, nx, ky, kx = 18100, 21, 301, 9
    Rs = [synth.radiance_map(ny, nx, 4, 0.05, (2.0, 10.0), rng) for _ in range(2)]
    Ks = [rng.random((ky, kx)) for _ in range(2)]
    plan = lp.make_plan_classes(Ks, ny, nx, precision=mode)
    assert plan.padding[0] == 18432 and plan.variant_info(lp.STAGE_COLUMNS, 0)["matrix_core"]
    y = plan.convolve_classes([torch.from_numpy(np.ascontiguousarray(r, np.float32)).cuda() for r in Rs])
    e2, em = errors(y.cpu().numpy(), oracle.conv_same_classes(Rs, Ks), f"matrix-core columns {mode} class sum")
    assert e2 <= TOL and em <= TOL


@pytest.mark.parametrize("mode", MODES.values(), ids=list(MODES))
def test_split_adjoint(lp, torch, mode):
    rng = np.random.default_rng(77)
    ny, nx, ky, kx = 120, 90, 17, 26
    G = (rng.random((ny, nx)) - 0.5).astype(np.float32)
    K = rng.random((ky, kx))
    A, _ = run(lp, torch, G, K, (144, 128), mode, adjoint=True)
    e2, em = errors(A, oracle.adjoint_same(G, K), f"split {mode} adjoint")
    assert e2 <= TOL and em <= TOL


def test_fp16_block_scaling_is_exact_under_power_of_two_scaling(lp, torch):
    """Each butterfly's inputs are scaled by a power of two before the FP16
    split, so S(2^s R) = 2^s S(R) exactly, far outside FP16's range."""
    rng = np.random.default_rng(91)
    ny, nx, ky, kx = 100, 200, 13, 9
    R = (0.5 + rng.random((ny, nx))).astype(np.float32)
    K = 0.5 + rng.random((ky, kx))
    S, plan = run(lp, torch, R, K, (128, 256), 1)
    for s in (-60, 60):
        Rs = np.ldexp(R, s).astype(np.float32)
        y = plan.convolve(torch.from_numpy(Rs).cuda()).cpu().numpy()
        assert np.array_equal(y, np.ldexp(S, s).astype(np.float32)), s


def test_fp16_wide_dynamic_range(lp, torch):
    """Lognormal radiance over ~13 decades, wider than FP16's own range
    (~6e-8 to 6.5e4): the per-butterfly scale keeps every split in range."""
    rng = np.random.default_rng(92)
    ny, nx, ky, kx = 240, 230, 17, 27
    R = np.exp(rng.normal(0.0, 4.0, (ny, nx))).astype(np.float32)
    K = rng.random((ky, kx))
    S, _ = run(lp, torch, R, K, (256, 256), 1)
    e2, em = errors(S, oracle.conv_same(R, K), "fp16 wide range")
    assert e2 <= TOL and em <= TOL


@pytest.mark.parametrize("mode", MODES.values(), ids=list(MODES))
def test_split_continental_workload_sampled(lp, torch, mode):
    """16384^2 map, 2001^2 kernel, P = 18432 = 16^2 * 72: columns and rows
    with two radix-16 matrix passes each; 512 sampled output pixels."""
    R, K = synth.continental_inputs()
    plan = lp.make_plan(K, *R.shape, padding=(18432, 18432), precision=mode)
    x = torch.from_numpy(R).cuda()
    y = plan.convolve(x)
    torch.cuda.synchronize()
    rng = np.random.default_rng(44)
    idx = synth.sample_pixels(R, 512, rng)
    got = y.cpu().numpy().ravel()[idx]
    e2, em = errors(got, oracle.conv_same_pixels(R, K, idx), f"continental split {mode}")
    assert e2 <= TOL and em <= TOL
    del x, y, plan
    torch.cuda.empty_cache()
