"""GPU parity of the source-class sum (Eq. 4): B = sum_t K_t (*) L_1t with the
products summed in the Fourier domain before one inverse transform, against
the FP64 oracle's class sum; per-class gradients against the oracle's
transposed operator."""
import numpy as np
import pytest

import oracle
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


def check(got, ref, label):
    e2, em = oracle.rel_l2(got, ref), oracle.max_err_frac(got, ref)
    print(f"{label}: rel-L2 {e2:.3e} max-err/max {em:.3e}", flush=True)
    assert e2 <= TOL and em <= TOL, (label, e2, em)


def sym_kernel(rng, ky, kx):
    cy, cx = ky // 2, kx // 2
    Q = rng.random((cy + 1, cx + 1))
    return Q[np.abs(np.arange(ky) - cy)][:, np.abs(np.arange(kx) - cx)]


def cuda(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


CASES = [  # ny, nx, ky, kx, padding (None: default), classes, symmetric kernels, kernels, precision
    (200, 64, 9, 9, (512, 80), 3, True, "auto", 0),       # specialised columns, real quadrant
    (300, 40, 11, 5, (512, 48), 2, False, "auto", 0),     # specialised columns, complex
    (250, 250, 101, 101, (512, 512), 4, True, "auto", 0),  # specialised rows and columns
    (2870, 30, 11, 7, (2880, 36), 3, False, "auto", 0),
    (97, 83, 13, 17, None, 3, False, "auto", 0),          # generic kernels, ragged
    (97, 83, 13, 17, None, 5, True, "generic", 0),
    (130, 140, 21, 31, (160, 180), 3, False, "auto", 1),  # split FP16 (generic, radix 16)
    (61, 70, 7, 9, None, 1, False, "auto", 0),            # one class = plain convolution
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}k{c[2]}T{c[5]}{c[7][0]}p{c[8]}" for c in CASES])
def test_class_sum_full_field(lp, torch, case):
    ny, nx, ky, kx, pad, T, sym, kern, prec = case
    rng = np.random.default_rng(ny * 31 + nx + T)
    maps = [synth.radiance_map(ny, nx, 3, 0.05, (1.0, 6.0), rng) + 0.1 * rng.random((ny, nx)).astype(np.float32)
            for _ in range(T)]
    Ks = [sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx)) for _ in range(T)]
    plan = lp.make_plan_classes(Ks, ny, nx, padding=pad, precision=prec,
                                kernels=lp.KERNELS_GENERIC if kern == "generic" else lp.KERNELS_AUTO)
    assert plan.classes == T
    assert plan.form == (lp.FORM_REAL_QUADRANT if sym else lp.FORM_COMPLEX)
    y = plan.convolve_classes([cuda(torch, m) for m in maps])
    torch.cuda.synchronize()
    check(y.cpu().numpy(), oracle.conv_same_classes(maps, Ks), f"classes {case}")


def test_mixed_symmetry_uses_complex_form(lp, torch):
    rng = np.random.default_rng(3)
    ny, nx, ky, kx = 120, 100, 15, 15
    Ks = [sym_kernel(rng, ky, kx), rng.random((ky, kx))]
    maps = [rng.random((ny, nx)).astype(np.float32) for _ in Ks]
    plan = lp.make_plan_classes(Ks, ny, nx)
    assert plan.form == lp.FORM_COMPLEX
    y = plan.convolve_classes([cuda(torch, m) for m in maps])
    check(y.cpu().numpy(), oracle.conv_same_classes(maps, Ks), "mixed symmetry")


def test_shared_kernel_equals_summed_map(lp, torch):
    """Classes sharing one kernel give the convolution of the summed map."""
    rng = np.random.default_rng(4)
    ny, nx, ky, kx = 200, 64, 9, 9
    K = rng.random((ky, kx))
    maps = [rng.random((ny, nx)).astype(np.float32) for _ in range(3)]
    pc = lp.make_plan_classes([K] * 3, ny, nx, padding=(512, 80))
    p1 = lp.make_plan(K, ny, nx, padding=(512, 80))
    a = pc.convolve_classes([cuda(torch, m) for m in maps]).cpu().numpy()
    b = p1.convolve(cuda(torch, sum(m.astype(np.float64) for m in maps))).cpu().numpy()
    assert oracle.rel_l2(a, b) <= 2e-7


def test_output_may_alias_a_class_map(lp, torch):
    rng = np.random.default_rng(5)
    ny, nx, ky, kx = 90, 70, 11, 11
    Ks = [rng.random((ky, kx)) for _ in range(2)]
    maps = [rng.random((ny, nx)).astype(np.float32) for _ in Ks]
    plan = lp.make_plan_classes(Ks, ny, nx)
    xs = [cuda(torch, m) for m in maps]
    ref = plan.convolve_classes(xs).cpu().numpy()
    plan.convolve_classes(xs, out=xs[1])
    assert np.array_equal(xs[1].cpu().numpy(), ref)


def test_per_class_adjoint_and_autograd(lp, torch):
    rng = np.random.default_rng(6)
    ny, nx, ky, kx = 80, 96, 13, 10
    Ks = [rng.random((ky, kx)) for _ in range(3)]
    maps = [rng.random((ny, nx)).astype(np.float32) for _ in Ks]
    G = (rng.random((ny, nx)) - 0.5).astype(np.float32)
    plan = lp.make_plan_classes(Ks, ny, nx)
    for t, K in enumerate(Ks):
        A = plan.adjoint_class(t, cuda(torch, G)).cpu().numpy()
        check(A, oracle.adjoint_same(G, K), f"adjoint class {t}")
    # autograd: loss = <B, G>, so d loss / d L_t = C_t^T G
    xs = [cuda(torch, m).requires_grad_(True) for m in maps]
    B = lp.convolve_classes(xs, plan)
    (B * cuda(torch, G)).sum().backward()
    for t, K in enumerate(Ks):
        check(xs[t].grad.cpu().numpy(), oracle.adjoint_same(G, K), f"autograd class {t}")


def test_classes_workload_sampled(lp, torch):
    """Three 4096^2 class maps with three 1201^2 kernels, P = 5400: 2048
    sampled output pixels of the summed map."""
    maps, Ks = synth.classes_inputs()
    plan = lp.make_plan_classes(Ks, 4096, 4096, padding=(5400, 5400))
    assert plan.kernels == lp.KERNELS_SPECIALISED
    y = plan.convolve_classes([cuda(torch, m) for m in maps])
    torch.cuda.synchronize()
    rng = np.random.default_rng(45)
    idx = synth.sample_pixels(maps[0], 2048, rng)
    check(y.cpu().numpy().ravel()[idx], oracle.conv_same_classes_pixels(maps, Ks, idx), "classes workload")
    del y, plan
    torch.cuda.empty_cache()


@pytest.mark.parametrize("case", [(4096, 9, 1201, 3, (5400, 12), True), (17000, 5, 1201, 3, (18432, 8), False)],
                         ids=["p5400", "p18432"])
def test_class_sum_every_column_variant(lp, torch, case):
    """Class-sum column kernels of every compiled column variant."""
    ny, nx, ky, kx, pad, sym = case
    rng = np.random.default_rng(ny + nx)
    T = 3
    maps = [rng.random((ny, nx)).astype(np.float32) for _ in range(T)]
    Ks = [sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx)) for _ in range(T)]
    ref = oracle.conv_same_classes(maps, Ks)
    plan = lp.make_plan_classes(Ks, ny, nx, padding=pad)
    xs = [cuda(torch, m) for m in maps]
    n = plan.variant_count(lp.STAGE_COLUMNS)
    assert n >= 2
    for k in range(n):
        plan.set_variant(lp.STAGE_COLUMNS, k)
        check(plan.convolve_classes(xs).cpu().numpy(), ref, f"classes {case} column v{k} {plan.variant_info(lp.STAGE_COLUMNS, k)}")
