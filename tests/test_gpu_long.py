"""GPU parity of the four-step column stage (padded columns longer than one
LDS tile, Py > 20480): full fields against the FP64 oracle on narrow maps
whose columns are long, with P1 = 2, 4 and 5 (radix-2/4/5 outer transforms)
and both spectrum forms; the transposed operator and autograd; sampled pixels
of a 24000 x 24000 map with a 2001 x 2001 kernel."""
import numpy as np
import pytest

import oracle

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


CASES = [  # ny, nx, ky, kx, padding (None: default), symmetric kernel, expected (P1, P2), kernels
    (20000, 4, 1001, 3, None, True, (4, 5400), "auto"),          # Py 21600, middle in registers (5400)
    (20000, 5, 1001, 3, None, False, (4, 5400), "auto"),         # complex form, odd nx
    (20000, 5, 1001, 3, None, False, (4, 5400), "generic"),      # the same split with LDS middle passes
    (20000, 4, 1001, 3, (20736, 6), False, (8, 2592), "auto"),   # the window bound n + floor(k/2) = 20500
    (60000, 3, 3001, 3, None, True, (40, 1600), "auto"),         # Py 64000
    (75000, 3, 3001, 1, None, False, (5, 15625), "auto"),        # Py 78125 = 5^7: no specialised divisor
    (130000, 2, 1001, 1, None, True, (64, 2048), "auto"),        # Py 131072 = LP_MAX_PY
]


@pytest.mark.parametrize("case", CASES, ids=[f"py{c[6][0] * c[6][1]}{'s' if c[5] else 'c'}{c[7][0]}" for c in CASES])
def test_four_step_full_field(lp, torch, case):
    ny, nx, ky, kx, pad, sym, split, kern = case
    rng = np.random.default_rng(ny + nx + ky)
    R = rng.random((ny, nx)).astype(np.float32)
    K = sym_kernel(rng, ky, kx) if sym else rng.random((ky, kx))
    plan = lp.make_plan(K, ny, nx, padding=pad,
                        kernels=lp.KERNELS_GENERIC if kern == "generic" else lp.KERNELS_AUTO)
    assert plan.column_split == split
    assert plan.form == (lp.FORM_REAL_QUADRANT if sym else lp.FORM_COMPLEX)
    y = plan.convolve(torch.from_numpy(R).cuda())
    torch.cuda.synchronize()
    check(y.cpu().numpy(), oracle.conv_same(R, K), f"four-step {case[:5]} {kern} P={plan.padding}")


def test_four_step_adjoint_and_autograd(lp, torch):
    rng = np.random.default_rng(11)
    ny, nx, ky, kx = 20000, 6, 1001, 5
    K = rng.random((ky, kx))
    R = rng.random((ny, nx)).astype(np.float32)
    G = (rng.random((ny, nx)) - 0.5).astype(np.float32)
    plan = lp.make_plan(K, ny, nx)
    assert plan.column_split[0] > 1
    A = plan.adjoint(torch.from_numpy(G).cuda()).cpu().numpy()
    check(A, oracle.adjoint_same(G, K), "four-step adjoint")
    x = torch.from_numpy(R).cuda().requires_grad_(True)
    y = lp.convolve(x, plan)
    (y * torch.from_numpy(G).cuda()).sum().backward()
    check(x.grad.cpu().numpy(), oracle.adjoint_same(G, K), "four-step autograd")


def test_four_step_large_map_sampled(lp, torch):
    """24000 x 24000 map, 2001 x 2001 kernel (Py = Px = 26244 = 2 x 13122):
    512 sampled output pixels against direct FP64 sums."""
    rng = np.random.default_rng(24000)
    n, k = 24000, 2001
    R = rng.random((n, n), dtype=np.float32)
    K = sym_kernel(rng, k, k)
    plan = lp.make_plan(K, n, n)
    assert plan.column_split == (2, 13122)
    y = plan.convolve(torch.from_numpy(R).cuda())
    torch.cuda.synchronize()
    idx = rng.choice(n * n, 512, replace=False)
    # the edges and corners too
    idx[:4] = [0, n - 1, (n - 1) * n, n * n - 1]
    got = y.cpu().numpy().ravel()[idx]
    check(got, oracle.conv_same_pixels(R, K, idx), "four-step 24000^2 sampled")
    del y, plan
    torch.cuda.empty_cache()
