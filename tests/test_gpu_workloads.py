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


PRECISIONS = {"fp32": 0, "fp16x2": 1, "bf16x3": 2}


@pytest.fixture(scope="module")
def continental():
    """The continental map (16384^2, 2001^2 kernel), its blob centres, and the
    oracle at 4096 sampled pixels: 2048 uniform, the 1024 brightest input
    pixels, 1024 at least 200 px from every blob centre."""
    centres = []
    R, K = synth.continental_inputs(centres=centres)
    idx = synth.sample_pixels_c12(R, centres[0], np.random.default_rng(43))
    return R, K, idx, oracle.conv_same_pixels(R, K, idx)


def run_precision(lp, torch, R, K, precision):
    plan = lp.make_plan(K, *R.shape, padding=(18432, 18432), precision=PRECISIONS[precision])
    x = torch.from_numpy(R).cuda()
    y = plan.convolve(x)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    kern = plan.kernels
    del x, y, plan
    torch.cuda.empty_cache()
    return out, kern


@pytest.mark.parametrize("precision", list(PRECISIONS))
def test_continental_workload_sampled(lp, torch, continental, precision):
    """16384^2 map, 2001^2 kernel, P = 18432, FP32 and the two split-precision
    matrix-core forms: 4096 sampled output pixels (uniform, brightest, and
    dark countryside far from every city)."""
    R, K, idx, ref = continental
    S, kern = run_precision(lp, torch, R, K, precision)
    if precision == "fp32":
        assert kern == lp.KERNELS_SPECIALISED
    got = S.ravel()[idx]
    check(got, ref, f"continental {precision} sampled ({len(idx)} px)")
    # the darkest quarter of the sample on its own: transform round-off is
    # about uniform in absolute terms, so there it is largest relative to
    # the value; the bar (max error over the map's maximum) still holds
    sel = np.argsort(ref)[:len(idx) // 4]
    em = float(np.max(np.abs(got[sel] - ref[sel])) / np.max(np.abs(ref)))
    e2 = oracle.rel_l2(got[sel], ref[sel])
    print(f"continental {precision}: darkest {len(sel)} sampled pixels, rel-L2 {e2:.3e}, "
          f"max err / max|S| {em:.3e}", flush=True)
    assert em <= TOL


@pytest.fixture(scope="module")
def continental_separable(continental):
    """K = u v^T at the continental shape: the oracle's separable form gives
    the full 16384^2 field in FP64 (2 x 16384^2 x 2001 multiply-adds)."""
    R = continental[0]
    u, v = synth.psf_separable(2001, 2001, np.random.default_rng(44))
    return u, v, oracle.conv_same_separable(R, u, v)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", list(PRECISIONS))
def test_continental_separable_full_field(lp, torch, continental, continental_separable, precision):
    """Full-field parity at the continental shape, P = 18432, every form."""
    R = continental[0]
    u, v, ref = continental_separable
    S, _ = run_precision(lp, torch, R, np.outer(u, v), precision)
    check(S, ref, f"continental separable full field {precision}")


@pytest.fixture(scope="module")
def paper_case():
    """The paper's map grid (Sec. 3: 11920 x 11804 pixels of 404.4 m), with
    the ALR kernel of Eqs. 12-13 out to 300 km (1485 x 1485), padded to
    13500 x 13500; the oracle at 4096 pixels (2048 uniform, 1024 brightest,
    1024 at least 200 px from every blob centre)."""
    centres = []
    R, K = synth.paper_inputs(centres=centres)
    idx = synth.sample_pixels_c12(R, centres[0], np.random.default_rng(47))
    return R, K, idx, oracle.conv_same_pixels(R, K, idx)


def test_paper_workload_sampled(lp, torch, paper_case):
    R, K, idx, ref = paper_case
    plan = lp.make_plan(K, *R.shape, pitch_km=synth.PAPER.pitch_km, padding=(13500, 13500))
    assert plan.kernels == lp.KERNELS_SPECIALISED
    assert plan.variant_count(lp.STAGE_COLUMNS) > 0 and plan.variant_count(lp.STAGE_ROWS) > 0
    S = plan.convolve(torch.from_numpy(R).cuda()).cpu().numpy()
    check(S.ravel()[idx], ref, f"paper grid, ALR kernel ({len(idx)} px)")
    del plan
    torch.cuda.empty_cache()


@pytest.mark.timeout(600)
def test_paper_shape_separable_full_field(lp, torch, paper_case):
    """K = u v^T at the paper's shape (1485 x 1485, P = 13500): full field,
    every stage variant of both lengths."""
    R = paper_case[0]
    u, v = synth.psf_separable(1485, 1485, np.random.default_rng(48))
    ref = oracle.conv_same_separable(R, u, v)
    plan = lp.make_plan(np.outer(u, v), *R.shape, pitch_km=synth.PAPER.pitch_km, padding=(13500, 13500))
    x = torch.from_numpy(R).cuda()
    for stage in (lp.STAGE_ROWS, lp.STAGE_COLUMNS):
        for k in range(plan.variant_count(stage)):
            plan.set_variant(stage, k)
            check(plan.convolve(x).cpu().numpy(), ref, f"paper shape separable, stage {stage} variant {k}")
        plan.set_variant(stage, 0)
    del plan, x
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
    # Against the FP64 oracle gradient (FP64 forward, FP64 residuals).  The
    # gradient is the transposed operator applied to the weighted site
    # residuals 2 w (S - m); the GPU's residuals differ from the FP64 ones by
    # its forward error at the sites, S_gpu - S_64, about 1e-7 of max|S| in
    # absolute terms.  So the gradient differs from the FP64 one by C^T of
    # 2 w (S_gpu - S_64) -- asserted as a decomposition, to the bar -- and
    # its relative error tracks rho = |w (S_gpu - S_64)| / |w (S_64 - m)|,
    # the relative perturbation of the weighted residual vector.  With the
    # workload's weights 1/m^2 dim sites amplify that absolute error and rho
    # is about 2e-2 (a property of the loss, not of the kernels); with
    # uniform weights it is about 2e-6, and the gradient meets the bar.
    S64 = oracle.conv_same_pixels(R0, K, sites)
    s_gpu = r.detach().cpu().numpy() + m
    ref64 = oracle.adjoint_sparse(sites, 2.0 * w * (S64 - m), R0.shape, K)
    rho = float(np.linalg.norm(w * (s_gpu - S64)) / np.linalg.norm(w * (S64 - m)))
    e64 = oracle.rel_l2(grad, ref64)
    dec = oracle.adjoint_sparse(sites, 2.0 * w * (s_gpu - S64), R0.shape, K)
    e_dec = float(np.linalg.norm((grad - ref64) - dec) / np.linalg.norm(ref64))
    print(f"autograd gradient vs FP64 oracle gradient, weights 1/m^2: rel-L2 {e64:.3e}; "
          f"residual perturbation rho {rho:.3e}; after removing C^T 2w(S_gpu - S_64): {e_dec:.3e}", flush=True)
    assert e_dec <= TOL
    assert e64 <= 1.5 * rho + TOL
    # Central differences on the 50 pixels with the largest gradient.  The
    # loss is quadratic in R, so central differences are exact up to
    # round-off for any step; what limits them is the FP32 round-off of the
    # forward map (about 1e-7 of max|S|), amplified at dim sites by the
    # weights 1/m^2 -- the same effect that separates the FP32-residual
    # gradient from the FP64-residual one by ~2e-2 (rho above).  With the
    # workload's weights the differences are therefore printed only (they
    # land at a few 1e-2, a property of the loss); with uniform weights (no
    # amplification) they are held to a tight bound.
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
          f"vs FP64 oracle gradient {e_64:.2e} (informational)", flush=True)

    wu = np.full_like(w, 1.0 / np.mean(m) ** 2)
    xu = torch.from_numpy(R0).cuda().requires_grad_(True)
    Su = lp.convolve(xu, plan)
    ru = Su.reshape(-1)[st].double() - mt
    (torch.from_numpy(wu).cuda() * ru * ru).sum().backward()
    gu = xu.grad.cpu().numpy().ravel()
    gu64 = oracle.adjoint_sparse(sites, 2.0 * wu * (S64 - m), R0.shape, K).ravel()
    rho_u = float(np.linalg.norm(ru.detach().cpu().numpy() + m - S64) / np.linalg.norm(S64 - m))
    eu64 = oracle.rel_l2(gu, gu64)
    print(f"autograd gradient vs FP64 oracle gradient, uniform weights: rel-L2 {eu64:.3e} (rho {rho_u:.3e})",
          flush=True)
    assert eu64 <= TOL
    pix_u = np.argsort(-np.abs(gu))[:50]
    fdu = central(wu, pix_u, 1.0e2)
    e_u = float(np.linalg.norm(fdu - gu[pix_u]) / np.linalg.norm(gu[pix_u]))
    print(f"central differences, uniform weights (50 px): rel-L2 vs autograd {e_u:.2e}")
    assert e_u <= 1e-3
