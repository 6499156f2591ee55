"""GPU parity at the full workload sizes (sampled pixels the oracle computes
one by one, plus properties that hold at any size) and the adjoint workload
(loss over observing sites, gradient through torch.autograd)."""
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


def run_full(lp, torch, R, K, padding, kernels=None):
    plan = lp.make_plan(K, *R.shape, padding=padding)
    if kernels is not None:
        plan.set_kernels(kernels)
    x = torch.from_numpy(R).cuda()
    y = plan.convolve(x)
    torch.cuda.synchronize()
    return y, plan


def test_country_workload_sampled(lp, torch):
    """4096^2 map, 1201^2 kernel, P = 5400: 4096 sampled output pixels."""
    R, K = synth.country_inputs()
    y, plan = run_full(lp, torch, R, K, (5400, 5400))
    assert plan.kernels == lp.KERNELS_SPECIALISED
    rng = np.random.default_rng(41)
    idx = synth.sample_pixels(R, 4096, rng)
    check(y.cpu().numpy().ravel()[idx], oracle.conv_same_pixels(R, K, idx), "country sampled")
    # sum identity over the whole map: the "same" window loses only the light
    # that falls outside it, so sum S <= sum R * sum K
    assert float(y.double().sum()) <= R.astype(np.float64).sum() * K.sum() * (1 + 1e-6)


def test_country_shape_separable_full_field(lp, torch):
    """Separable kernel K = u v^T at the country shape: full-field reference
    from the oracle's separable form."""
    R, _ = synth.country_inputs()
    rng = np.random.default_rng(42)
    u, v = synth.psf_separable(1201, 1201, rng)
    K = np.outer(u, v)
    y, _ = run_full(lp, torch, R, K, (5400, 5400))
    check(y.cpu().numpy(), oracle.conv_same_separable(R, u, v), "country separable full field")


def test_continental_workload_sampled(lp, torch):
    """16384^2 map, 2001^2 kernel, P = 18432: 1024 sampled output pixels."""
    R, K = synth.continental_inputs()
    y, plan = run_full(lp, torch, R, K, (18432, 18432))
    assert plan.kernels == lp.KERNELS_SPECIALISED
    rng = np.random.default_rng(43)
    idx = synth.sample_pixels(R, 1024, rng)
    check(y.cpu().numpy().ravel()[idx], oracle.conv_same_pixels(R, K, idx), "continental sampled")
    del y, plan
    torch.cuda.empty_cache()


@pytest.mark.parametrize("case", [(17000, 8, 1001, 3, (18432, 12)), (6, 17000, 3, 1201, (8, 18432))],
                         ids=["cols18432", "rows9216"])
def test_continental_lengths_full_field(lp, torch, case):
    ny, nx, ky, kx, pad = case
    rng = np.random.default_rng(ny + nx)
    R = rng.random((ny, nx)).astype(np.float32)
    K = rng.random((ky, kx))
    y, plan = run_full(lp, torch, R, K, pad)
    assert plan.kernels == lp.KERNELS_SPECIALISED
    check(y.cpu().numpy(), oracle.conv_same(R, K), f"full field {case}")


# ------------------------------------------------------------ adjoint workload

@pytest.fixture(scope="module")
def adjoint_case(lp, torch):
    R0, K, sites, R_true, eps = synth.adjoint_inputs()
    S_true = oracle.conv_same_pixels(R_true, K, sites)
    m = S_true * (1.0 + 0.05 * eps)
    w = 1.0 / m ** 2
    plan = lp.make_plan(K, *R0.shape, padding=(2880, 2880))
    return R0, K, sites, m, w, plan


def test_adjoint_workload_forward_at_sites(lp, torch, adjoint_case):
    R0, K, sites, m, w, plan = adjoint_case
    S = plan.convolve(torch.from_numpy(R0).cuda()).cpu().numpy().ravel()
    check(S[sites], oracle.conv_same_pixels(R0, K, sites), "adjoint workload S at sites")


def test_adjoint_workload_backward_operator(lp, torch, adjoint_case):
    """lp_adjoint of the site residual map against the oracle's transposed
    operator on the same residuals (FP64), full 2048^2 field."""
    R0, K, sites, m, w, plan = adjoint_case
    S = oracle.conv_same_pixels(R0, K, sites)
    g = 2.0 * w * (S - m)
    G = np.zeros(R0.size, np.float32)
    G[sites] = g.astype(np.float32)
    A = plan.adjoint(torch.from_numpy(G.reshape(R0.shape)).cuda()).cpu().numpy()
    check(A, oracle.adjoint_sparse(sites, g.astype(np.float32), R0.shape, K), "adjoint workload backward")


def test_adjoint_workload_autograd_gradient(lp, torch, adjoint_case):
    """Loss sum_i w_i (S(x_i) - m_i)^2 through torch.autograd: the gradient
    equals the oracle's transposed operator applied to the residuals the
    forward produced, and matches central differences (exact for a quadratic
    loss up to round-off) on 50 pixels."""
    R0, K, sites, m, w, plan = adjoint_case
    st = torch.from_numpy(sites).cuda()
    mt = torch.from_numpy(m).cuda()
    wt = torch.from_numpy(w).cuda()

    def loss_fn(Rt):
        S = lp.convolve(Rt, plan)
        r = S.reshape(-1)[st].double() - mt
        return (wt * r * r).sum(), r

    x = torch.from_numpy(R0).cuda().requires_grad_(True)
    L, r = loss_fn(x)
    L.backward()
    grad = x.grad.cpu().numpy()
    g = (2.0 * w * r.detach().cpu().numpy()).astype(np.float32)
    check(grad, oracle.adjoint_sparse(sites, g, R0.shape, K), "autograd gradient vs oracle")
    # the oracle gradient with FP64 residuals, for the record (dim sites carry
    # large weights 1/m^2, so FP32 forward error enters it)
    ref64 = oracle.adjoint_sparse(sites, 2.0 * w * (oracle.conv_same_pixels(R0, K, sites) - m), R0.shape, K)
    print(f"autograd gradient vs FP64-residual oracle gradient: rel-L2 {oracle.rel_l2(grad, ref64):.3e}")
    # Central differences on the 50 pixels with the largest gradient.  The
    # loss is quadratic in R, so central differences are exact up to
    # round-off for any step; what limits them is the FP32 round-off of the
    # forward map (about 1e-7 of max|S|), amplified at dim sites by the
    # weights 1/m^2 -- the same effect that separates the FP32-residual
    # gradient from the FP64-residual one by ~2e-2.  So: with the workload's
    # weights, a 5e-2 consistency bound; with uniform weights (no
    # amplification), a tight one.
    ny, nx = R0.shape

    def central(weights, pix, h):
        wt_ = torch.from_numpy(weights).cuda()

        def L_of(Rt):
            r_ = plan.convolve(Rt.contiguous()).reshape(-1)[st].double() - mt
            return float((wt_ * r_ * r_).sum())

        out = []
        with torch.no_grad():
            base = torch.from_numpy(R0).cuda().reshape(-1)
            for p in pix:
                xp = base.clone()
                xp[p] += h
                Lp = L_of(xp.reshape(ny, nx))
                xp[p] -= 2 * h
                Lm = L_of(xp.reshape(ny, nx))
                out.append((Lp - Lm) / (2 * h))
        return np.array(out)

    pix = np.argsort(-np.abs(grad.ravel()))[:50]
    fd = central(w, pix, 1.0e2)
    an = grad.ravel()[pix].astype(np.float64)
    e_fd = float(np.linalg.norm(fd - an) / np.linalg.norm(an))
    e_64 = float(np.linalg.norm(fd - ref64.ravel()[pix]) / np.linalg.norm(ref64.ravel()[pix]))
    print(f"central differences, weights 1/m^2 (50 px): rel-L2 vs autograd {e_fd:.2e}, "
          f"vs FP64 oracle gradient {e_64:.2e}")
    assert e_fd <= 5e-2

    wu = np.full_like(w, 1.0 / np.mean(m) ** 2)
    xu = torch.from_numpy(R0).cuda().requires_grad_(True)
    Su = lp.convolve(xu, plan)
    ru = Su.reshape(-1)[st].double() - mt
    (torch.from_numpy(wu).cuda() * ru * ru).sum().backward()
    gu = xu.grad.cpu().numpy().ravel()
    pix_u = np.argsort(-np.abs(gu))[:50]
    fdu = central(wu, pix_u, 1.0e2)
    e_u = float(np.linalg.norm(fdu - gu[pix_u]) / np.linalg.norm(gu[pix_u]))
    print(f"central differences, uniform weights (50 px): rel-L2 vs autograd {e_u:.2e}")
    assert e_u <= 1e-3
