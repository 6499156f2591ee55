"""Debug poison mode (lp_plan_set_poison, lp_batch_set_poison): with the
intermediate spectra (and the four-step scratch) NaN-filled before every
call, each path must give the same bits as without, so that no stage reads
an element no stage wrote: specialised and generic kernels, both spectrum
forms, the transposed operator, split precision, four-step columns, the
class sum, the no-allocation entry point and the batched graph."""
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


def sym_kernel(rng, ky, kx):
    q = rng.random(((ky + 1) // 2, (kx + 1) // 2))
    iy = np.abs(np.arange(ky) - (ky - 1) // 2)
    ix = np.abs(np.arange(kx) - (kx - 1) // 2)
    return q[iy][:, ix]


def check(got, ref, label):
    e2, em = oracle.rel_l2(got, ref), oracle.max_err_frac(got, ref)
    print(f"{label}: rel-L2 {e2:.3e} max-err/max {em:.3e}", flush=True)
    assert e2 <= TOL and em <= TOL, (label, e2, em)


def same_bits(plan, run, torch):
    """run() under poison off and on; returns the poisoned result after
    asserting that both are finite and identical bit for bit."""
    plan.set_poison(False)
    a = run().cpu().numpy()
    plan.set_poison(True)
    b = run().cpu().numpy()
    plan.set_poison(False)
    torch.cuda.synchronize()
    assert np.isfinite(b).all()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    return b


CASES = [  # label, ny, nx, ky, kx, padding, symmetric kernel, kernels, precision
    ("specialised 512 quadrant", 300, 260, 41, 41, (512, 512), True, "auto", "fp32"),
    ("specialised 512x2880 complex, odd width", 301, 2001, 51, 41, (512, 2880), False, "auto", "fp32"),
    ("specialised 5400 rows and columns", 900, 3001, 101, 1201, (1200, 5400), True, "auto", "fp32"),
    ("generic 360", 200, 150, 31, 21, (360, 360), False, "generic", "fp32"),
    ("split FP16 on MFMA", 300, 260, 41, 41, (512, 512), True, "auto", "fp16x2"),
    ("split BF16 on MFMA, complex form", 300, 260, 41, 31, (512, 512), False, "auto", "bf16x3"),
    ("four-step columns 4 x 5400", 20000, 4, 1001, 3, None, True, "auto", "fp32"),
    # register kernels with the radix-16 pass on the matrix cores
    ("split BF16 matrix-core rows 9216", 37, 18000, 5, 401, None, True, "auto", "bf16x3"),
    ("split FP16 matrix-core columns 18432, complex form", 18000, 37, 401, 5, None, False, "auto", "fp16x2"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_poisoned_intermediate_is_never_read(lp, torch, case):
    label, ny, nx, ky, kx, pad, sym, kern, prec = case
    rng = np.random.default_rng(ny * 7 + nx)
    R = rng.random((ny, nx)).astype(np.float32)
    G = (rng.random((ny, nx)) - 0.5).astype(np.float32)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    precision = {"fp32": lp.PRECISION_FP32, "fp16x2": lp.PRECISION_SPLIT_FP16, "bf16x3": lp.PRECISION_SPLIT_BF16}[prec]
    plan = lp.make_plan(K, ny, nx, padding=pad, precision=precision,
                        kernels=lp.KERNELS_GENERIC if kern == "generic" else lp.KERNELS_AUTO)
    x = torch.from_numpy(R).cuda()
    g = torch.from_numpy(G).cuda()
    print(f"poison: {label}, padding {plan.padding}, split {plan.column_split}", flush=True)
    s = same_bits(plan, lambda: plan.convolve(x), torch)
    a = same_bits(plan, lambda: plan.adjoint(g), torch)
    if ny * nx <= 400_000:
        check(s, oracle.conv_same(R, K), f"{label} forward")
        check(a, oracle.adjoint_same(G, K), f"{label} adjoint")
    else:
        idx = rng.choice(ny * nx, 512, replace=False)
        check(s.ravel()[idx], oracle.conv_same_pixels(R, K, idx), f"{label} forward, 512 px")
    del plan
    torch.cuda.empty_cache()


def test_poisoned_class_sum_and_noalloc(lp, torch):
    rng = np.random.default_rng(5)
    ny, nx = 700, 900
    Ks = [sym_kernel(rng, 101, 101), rng.random((101, 101)), sym_kernel(rng, 101, 101)]
    maps = [rng.random((ny, nx)).astype(np.float32) for _ in Ks]
    xs = [torch.from_numpy(m).cuda() for m in maps]
    pc = lp.make_plan_classes(Ks, ny, nx)
    s = same_bits(pc, lambda: pc.convolve_classes(xs), torch)
    check(s, oracle.conv_same_classes(maps, Ks), "class sum")
    plan = lp.make_plan(Ks[0], ny, nx, padding=(1200, 1200))
    out = torch.empty_like(xs[0])
    n = same_bits(plan, lambda: plan.convolve_noalloc(xs[0], out), torch)
    plan.set_poison(False)
    assert np.array_equal(n.view(np.uint32), plan.convolve(xs[0]).cpu().numpy().view(np.uint32))


def test_poisoned_batch_graph_and_direct(lp, torch):
    rng = np.random.default_rng(300)
    K0 = sym_kernel(rng, 51, 51)
    K1 = rng.random((41, 31))
    shapes = [(200, 300), (700, 150), (150, 1500), (901, 799), (37, 20)]
    ids = [0, 0, 1, 1, 1]
    maps = [rng.random(s).astype(np.float32) for s in shapes]
    xs = [torch.from_numpy(m).cuda() for m in maps]
    b = lp.Batch(shapes, ids, [K0.shape, K1.shape]).bind()
    b.set_kernels([K0, K1])
    for graph in (True, False):
        b.use_graph(graph)
        b.set_poison(False)
        a = [o.cpu().numpy() for o in b.convolve(xs)]
        b.set_poison(True)
        p = [o.cpu().numpy() for o in b.convolve(xs)]
        p2 = [o.cpu().numpy() for o in b.convolve(xs)]   # a graph replay with the fill inside
        torch.cuda.synchronize()
        for t in range(len(maps)):
            assert np.isfinite(p[t]).all(), (graph, t)
            assert np.array_equal(a[t].view(np.uint32), p[t].view(np.uint32)), (graph, t)
            assert np.array_equal(p[t].view(np.uint32), p2[t].view(np.uint32)), (graph, t)
        b.set_poison(False)
    for t, m in enumerate(maps):
        check(p[t], oracle.conv_same(m, [K0, K1][ids[t]]), f"batch map {t} poisoned")
