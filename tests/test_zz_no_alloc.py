"""lp_convolve_noalloc (the entry point for callers that cannot allocate
device memory): through the C ABI, against lp_convolve on the same plan and
inputs, on two calls in a row, the second with a smaller map; and the size
and state checks it makes before touching the device."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1907_02891_amd import synth

TOL = 1e-5


@pytest.fixture(scope="module")
def lp():
    from paper_1907_02891_amd import lp as _lp
    return _lp


def _plan(lp, torch, R, K, padding):
    return lp.make_plan(K, *R.shape, padding=padding, device="cuda:0")


@pytest.mark.gpu
def test_noalloc_matches_convolve_two_calls(lp):
    import torch
    assert torch.cuda.is_available()
    lib = lp.raw()
    rng = np.random.default_rng(11)
    cases = [  # (map, kernel, padding): the second call has the smaller map
        (synth.radiance_map(2048, 2048, 100, 0.05, (2.0, 40.0), rng), synth.psf_powexp(400, 2.5, 80.0, 0.5, 200.0),
         (2880, 2880)),
        (synth.radiance_map(333, 517, 9, 0.05, (2.0, 8.0), rng), synth.psf_powexp(30, 2.5, 80.0, 0.5), None),
    ]
    for R, K, pad in cases:
        print(f"noalloc: map {R.shape}, kernel {K.shape}, padding {pad}", flush=True)
        plan = _plan(lp, torch, R, K, pad)
        x = torch.from_numpy(R).cuda()
        want = torch.empty_like(x)
        got = torch.full_like(x, float("nan"))
        assert lib.lp_convolve(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(want.data_ptr())) == 0
        rc = lib.lp_convolve_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(got.data_ptr()))
        assert rc == 0, lp.last_error()
        torch.cuda.synchronize()
        w, g = want.cpu().numpy(), got.cpu().numpy()
        # same kernels, same inputs: the same bits
        np.testing.assert_array_equal(g, w)
        idx = np.sort(rng.choice(R.size, 512, replace=False))
        ref = oracle.conv_same_pixels(R, K, idx)
        assert oracle.rel_l2(g.ravel()[idx], ref) <= TOL and oracle.max_err_frac(g.ravel()[idx], ref) <= TOL


@pytest.mark.gpu
def test_noalloc_in_place_and_repeat(lp):
    import torch
    lib = lp.raw()
    R, K = synth.small_inputs()
    plan = _plan(lp, torch, R, K, (512, 512))
    x = torch.from_numpy(R).cuda()
    want = plan.convolve(x).cpu().numpy()
    for _ in range(3):
        y = x.clone()
        assert lib.lp_convolve_noalloc(plan.handle, ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(y.data_ptr())) == 0
        torch.cuda.synchronize()
        np.testing.assert_array_equal(y.cpu().numpy(), want)


def test_noalloc_checks_before_any_device_call(lp):
    lib = lp.raw()
    fake = ctypes.c_void_p(256)
    p = lp.Plan(64, 48, 5, 5)
    assert lib.lp_convolve_noalloc(None, fake, fake) == lp.LP_E_INVALID
    assert lib.lp_convolve_noalloc(p.handle, None, fake) == lp.LP_E_INVALID
    assert lib.lp_convolve_noalloc(p.handle, fake, fake) == lp.LP_E_NOMEM  # unbound
    # the continental map's intermediate (16384 x 9218 x 8 B) exceeds the scratch array
    big = lp.Plan(16384, 16384, 2001, 2001, padding=(18432, 18432))
    assert lib.lp_convolve_noalloc(big.handle, fake, fake) == lp.LP_E_SIZE
    assert "scratch array" in lp.last_error()
    # a four-step plan keeps its scratch in the workspace
    long = lp.Plan(1000, 64, 21000, 5)
    assert long.column_split[0] > 1
    assert lib.lp_convolve_noalloc(long.handle, fake, fake) == lp.LP_E_SIZE
    cls = lp.Plan(64, 48, 5, 5)
    cls.set_classes(2)
    assert lib.lp_convolve_noalloc(cls.handle, fake, fake) == lp.LP_E_STATE
    # the largest map that fits: (Px/2+1 rounded up to even) * ny * 8 bytes <= the limit
    ok = lp.Plan(4096, 4096, 1201, 1201, padding=(5400, 5400))
    assert 2702 * 4096 * 8 <= lp.NOALLOC_MAX_BYTES
    assert lib.lp_convolve_noalloc(ok.handle, fake, fake) == lp.LP_E_NOMEM  # passes the size check
