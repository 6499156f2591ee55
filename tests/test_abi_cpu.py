"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/lp.h declares, and rejects bad arguments and out-of-order
calls before touching the HIP runtime."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1907_02891_amd import lp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "lp.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert "lp_convolve" in names and "lp_kernel_spectrum" in names
    lib = lp.raw()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(lp.EXPORTED) | set(names)


def test_version():
    assert "gfx950" in lp.version()


@pytest.mark.parametrize("args", [(0, 4, 3, 3, 0.5), (4, -1, 3, 3, 0.5), (4, 4, 0, 3, 0.5),
                                  (4, 4, 3, 3, 0.0), (4, 4, 3, 3, float("nan")),
                                  (4, 4, 3, 3, float("inf")), (4, 4, 3, 3, -1.0)])
def test_create_rejects_bad_arguments(args):
    assert not lp.raw().lp_plan_create(*args)
    assert lp.last_error()
    with pytest.raises(lp.LPError) as ei:
        lp.Plan(*args[:4], pitch_km=args[4])
    assert ei.value.code == lp.LP_E_INVALID


@pytest.mark.parametrize("shape", [(131000, 100, 2001, 3), (100, 40000, 3, 2001)])
def test_create_rejects_oversize(shape):
    with pytest.raises(lp.LPError) as ei:
        lp.Plan(*shape)
    assert ei.value.code == lp.LP_E_SIZE


def _four_step_p2(n, cap):
    """P2 of the four-step split: the longest divisor with a column
    specialisation whose exchange buffer (8 bytes per value, 80 KiB at most:
    two workgroups per CU) fits half the LDS (and P1 <= 4096), else the
    largest divisor within a tile."""
    spec = [d for d in lp.spec_lengths()[0]
            if d <= cap and n % d == 0 and n // d <= 4096 and d * 8 <= 80 * 1024]
    return max(spec) if spec else max(d for d in range(2, cap + 1) if n % d == 0)


@pytest.mark.parametrize("shape", [(20000, 4, 1001, 3), (24000, 24000, 2001, 2001), (60000, 10, 3001, 3),
                                   (75000, 3, 3001, 1), (130000, 2, 1001, 1)])
def test_four_step_column_split(shape):
    """Padded columns longer than one LDS tile (20480 values) split as
    Py = P1 P2, P2 a divisor within a tile (a specialised length if any)."""
    p = lp.Plan(*shape)
    py = p.padding[0]
    assert py > lp.MAX_COLUMN_TILE and py <= lp.MAX_PY
    p1, p2 = p.column_split
    assert p1 * p2 == py and p1 >= 2
    assert p2 == _four_step_p2(py, lp.MAX_COLUMN_TILE)
    # the workspace holds a Py-long scratch column per stored column
    h = p.padding[1] // 2 + 1
    assert p.workspace_bytes >= (h + h % 2) * py * 8
    q = lp.Plan(4096, 4096, 1201, 1201)
    assert q.column_split == (1, q.padding[0])


def test_four_step_split_prefers_two_workgroups_per_cu():
    """27000 = 2 x 13500 = 5 x 5400: the 13500-point middle kernel's exchange
    buffer (108 KiB) leaves one workgroup per CU, so the split is 5 x 5400."""
    p = lp.Plan(24000, 24000, 2001, 2001, padding=(27000, 27000))
    assert p.column_split == (5, 5400)


def test_four_step_takes_one_class():
    p = lp.Plan(20000, 4, 1001, 3)
    with pytest.raises(lp.LPError) as ei:
        p.set_classes(2)
    assert ei.value.code == lp.LP_E_SIZE
    p.set_classes(1)
    q = lp.Plan(19900, 4, 1001, 3)
    q.set_padding(20480, 6)  # one tile: classes allowed
    q.set_classes(3)
    with pytest.raises(lp.LPError) as ei:
        q.set_padding(20736, 6)
    assert ei.value.code == lp.LP_E_SIZE


@pytest.mark.parametrize("shape,pad", [((256, 256, 101, 101), (360, 360)),
                                       ((4096, 4096, 1201, 1201), (5400, 5400)),
                                       ((16384, 16384, 2001, 2001), (18432, 18432)),
                                       ((2048, 2048, 801, 801), (2880, 2880)),
                                       ((10, 7, 3, 3), (12, 10)),
                                       ((1, 1, 1, 1), (1, 2))])
def test_default_padding_is_smallest_5smooth(shape, pad):
    p = lp.Plan(*shape)
    assert p.padding == pad


def is_5smooth(n):
    for f in (2, 3, 5):
        while n % f == 0:
            n //= f
    return n == 1


@pytest.mark.parametrize("n", [7, 31, 100, 1711, 4321])
def test_default_padding_property(n):
    p = lp.Plan(n, n + 3, 5, 8)
    py, px = p.padding
    assert py >= n + 4 and px >= n + 10 and px % 2 == 0
    assert is_5smooth(py) and is_5smooth(px)
    assert not any(is_5smooth(m) for m in range(n + 4, py))
    assert not any(is_5smooth(m) and m % 2 == 0 for m in range(n + 10, px))


@pytest.mark.parametrize("pad,code", [((355, 360), lp.LP_E_SIZE), ((360, 355), lp.LP_E_SIZE),
                                      ((364, 360), lp.LP_E_SIZE), ((360, 375), lp.LP_E_SIZE),
                                      ((131220, 512), lp.LP_E_SIZE), ((21870, 512), None), ((375, 512), None),
                                      ((512, 512), None)])
def test_set_padding_validation(pad, code):
    p = lp.Plan(256, 256, 101, 101)
    if code is None:
        p.set_padding(*pad)
        assert p.padding == pad
    else:
        with pytest.raises(lp.LPError) as ei:
            p.set_padding(*pad)
        assert ei.value.code == code
        assert p.padding == (360, 360)


def test_workspace_grows_with_padding():
    p = lp.Plan(256, 256, 101, 101)
    a = p.workspace_bytes
    p.set_padding(512, 512)
    assert p.workspace_bytes > a > 0
    assert lp.raw().lp_plan_workspace_bytes(None) == 0


def test_state_errors_before_any_device_call():
    lib = lp.raw()
    p = lp.Plan(64, 48, 5, 5)
    fake = ctypes.c_void_p(256)
    # convolve with no workspace bound
    assert lib.lp_convolve(p.handle, fake, fake) == lp.LP_E_NOMEM
    assert lib.lp_adjoint(p.handle, fake, fake) == lp.LP_E_NOMEM
    # null data pointers
    assert lib.lp_convolve(p.handle, None, fake) == lp.LP_E_INVALID
    assert lib.lp_convolve(None, fake, fake) == lp.LP_E_INVALID
    # spectrum before bind
    K = np.ones((5, 5))
    assert lib.lp_kernel_spectrum(p.handle, K.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == lp.LP_E_STATE
    # non-finite kernel rejected first
    K[2, 3] = np.nan
    assert lib.lp_kernel_spectrum(p.handle, K.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == lp.LP_E_INVALID
    assert "not finite" in lp.last_error()
    K[2, 3] = np.inf
    assert lib.lp_kernel_spectrum(p.handle, K.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == lp.LP_E_INVALID
    # bind: null, misaligned, too small
    assert lib.lp_plan_bind(p.handle, None, 1 << 30, None) == lp.LP_E_INVALID
    assert lib.lp_plan_bind(p.handle, ctypes.c_void_p(4096 + 8), 1 << 30, None) == lp.LP_E_INVALID
    assert lib.lp_plan_bind(p.handle, ctypes.c_void_p(4096), 16, None) == lp.LP_E_NOMEM
    # spectrum readback before spectrum
    out = np.empty(10, np.float32)
    assert lib.lp_plan_read_spectrum(p.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))) == lp.LP_E_STATE
    assert lib.lp_plan_spectrum_form(p.handle) == lp.FORM_NONE


def test_shape_choice_fits_lds():
    for shape in [(256, 256, 101, 101), (4096, 4096, 1201, 1201), (16384, 16384, 2001, 2001),
                  (2048, 2048, 801, 801), (3, 5, 2, 2)]:
        p = lp.Plan(*shape)
        py, px = p.padding
        c, b = p.shape
        assert c >= 1 and b >= 1 and (c & (c - 1)) == 0 and (b & (b - 1)) == 0
        assert py * c * 8 <= 163840
        assert (px // 2 + 1) * b * 8 <= 163840


def test_batch_contract_errors():
    with pytest.raises(lp.LPError) as ei:
        lp.Batch([(100, 100)], [0], [(40000, 3)])  # 100 + 20000 beyond the longest specialised column
    assert ei.value.code == lp.LP_E_SIZE
    with pytest.raises(lp.LPError) as ei:
        lp.Batch([(100, 100)], [2], [(5, 5)])
    assert ei.value.code == lp.LP_E_INVALID
    with pytest.raises(lp.LPError) as ei:
        lp.Batch([(0, 100)], [0], [(5, 5)])
    assert ei.value.code == lp.LP_E_INVALID
    b = lp.Batch([(600, 700), (100, 100), (600, 700)], [0, 1, 1], [(101, 101), (5, 5)])
    assert b.workspace_bytes > 0
    gs = b.groups
    assert sum(g["maps"] for g in gs) == 3
    for g in gs:
        py, px = g["padding"]
        assert py >= 1 and px % 2 == 0 and g["row_variants"] >= 1 and g["column_variants"] >= 1
    assert b.tile_group(0) == b.tile_group(2) != b.tile_group(1)
    lib = lp.raw()
    fake = (ctypes.c_void_p * 3)(256, 256, 256)
    assert lib.lp_convolve_batched(b._b, fake, fake) == lp.LP_E_NOMEM
    assert lib.lp_batch_set_variant(b._b, 0, 7, 0) == lp.LP_E_INVALID
    assert lib.lp_batch_set_variant(b._b, 0, lp.STAGE_ROWS, 99) == lp.LP_E_INVALID
    assert lib.lp_batch_set_variant(b._b, 0, lp.STAGE_ROWS_INVERSE, 99) == lp.LP_E_INVALID
    # the inverse row stage alone, and both row stages together (a class of
    # padded rows that have several row variants)
    b2 = lp.Batch([(4000, 4000)], [0], [(1201, 1201)])
    assert b2.groups[0]["row_variants"] > 1
    assert lib.lp_batch_set_variant(b2._b, 0, lp.STAGE_ROWS_INVERSE, 1) == lp.LP_OK
    assert lib.lp_batch_get_variant(b2._b, 0, lp.STAGE_ROWS_INVERSE) == 1
    assert lib.lp_batch_get_variant(b2._b, 0, lp.STAGE_ROWS) == 0
    assert lib.lp_batch_set_variant(b2._b, 0, lp.STAGE_ROWS, 0) == lp.LP_OK
    assert lib.lp_batch_get_variant(b2._b, 0, lp.STAGE_ROWS_INVERSE) == 0


def test_python_binding_rejects_host_and_mismatched_tensors():
    """The binding checks tensors before anything reaches the library: host
    tensors, a wrong count of maps or outputs, and a workspace that is not a
    uint8 device tensor are errors (no host pointer is handed to a kernel)."""
    import torch
    b = lp.Batch([(60, 70), (30, 40)], [0, 0], [(11, 11)])
    host = [torch.zeros(60, 70), torch.zeros(30, 40)]
    with pytest.raises(ValueError, match="CUDA"):
        b.convolve(host)
    with pytest.raises(ValueError, match="1 maps for a batch of 2"):
        b.convolve(host[:1])
    with pytest.raises(ValueError, match="1 outputs for a batch of 2"):
        b.convolve(host, host[:1])
    p = lp.Plan(60, 70, 11, 11)
    with pytest.raises(ValueError, match="CUDA"):
        p.convolve(torch.zeros(60, 70))
    with pytest.raises(ValueError, match="workspace"):
        p.bind(workspace=torch.zeros(p.workspace_bytes + 256, dtype=torch.uint8))


def test_tune_cache_key_separates_precisions():
    """A split-precision plan numbers its variants among the matrix-core
    ones, so the autotuner's cache keeps its choices apart from FP32's."""
    from paper_1907_02891_amd import tune
    p = lp.Plan(16384, 16384, 2001, 2001)
    keys = set()
    for mode in (lp.PRECISION_FP32, lp.PRECISION_SPLIT_FP16, lp.PRECISION_SPLIT_BF16):
        p.set_precision(mode)
        keys.add(tune.plan_key(p))
    assert len(keys) == 3


def test_precision_modes_host_side():
    lib = lp.raw()
    p = lp.Plan(16384, 16384, 2001, 2001)
    assert p.precision == lp.PRECISION_FP32 and p.kernels == lp.KERNELS_SPECIALISED
    ws = p.workspace_bytes
    n_fp32 = {st: p.variant_count(st) for st in (lp.STAGE_ROWS, lp.STAGE_COLUMNS)}
    for st, n in n_fp32.items():
        assert n >= 1 and not any(p.variant_info(st, k)["matrix_core"] for k in range(n))
    p.set_variant(lp.STAGE_COLUMNS, 1)
    for mode in (lp.PRECISION_SPLIT_FP16, lp.PRECISION_SPLIT_BF16, lp.PRECISION_FP32):
        p.set_precision(mode)
        assert p.precision == mode
        # 9216-point rows and 18432-point columns have specialisations with
        # the radix-16 pass on the matrix cores: the split forms run them (and
        # only such variants), starting from variant 0; the layout does not
        # change
        assert p.kernels == lp.KERNELS_SPECIALISED
        split = mode != lp.PRECISION_FP32
        for st in (lp.STAGE_ROWS, lp.STAGE_COLUMNS):
            assert p.variant(st) == 0
            n = p.variant_count(st)
            infos = [p.variant_info(st, k) for k in range(n)]
            assert n >= 1 and all(i["matrix_core"] == split for i in infos)
            if split:
                assert all(i["radices"][0] == 16 for i in infos)
            else:
                assert n == n_fp32[st]
        assert p.workspace_bytes == ws
    # lengths with no matrix-core row variant: a split plan runs the generic
    # kernels in every stage
    q = lp.Plan(4096, 4096, 1201, 1201)
    q.set_precision(lp.PRECISION_SPLIT_BF16)
    assert q.variant_count(lp.STAGE_ROWS) == 0 and q.kernels == lp.KERNELS_GENERIC
    for bad in (-1, 3, 99):
        with pytest.raises(lp.LPError) as ei:
            p.set_precision(bad)
        assert ei.value.code == lp.LP_E_INVALID
    assert p.precision == lp.PRECISION_FP32
    assert lib.lp_plan_precision(None) == -1
    assert lib.lp_plan_set_precision(None, 1) == lp.LP_E_INVALID


def test_class_plan_host_side():
    lib = lp.raw()
    p = lp.Plan(300, 200, 31, 21)
    one = p.workspace_bytes
    for bad in (0, -1, lp.MAX_CLASSES + 1):
        with pytest.raises(lp.LPError) as ei:
            p.set_classes(bad)
        assert ei.value.code == lp.LP_E_INVALID
    assert p.classes == 1
    p.set_classes(3)
    assert p.classes == 3 and p.workspace_bytes > 2 * one
    # single-class entry points refuse a plan of several classes, before any
    # device work
    K = np.ones((31, 21))
    fake = ctypes.c_void_p(256)
    assert lib.lp_kernel_spectrum(p.handle, K.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == lp.LP_E_STATE
    assert lib.lp_convolve(p.handle, fake, fake) == lp.LP_E_STATE
    assert lib.lp_adjoint(p.handle, fake, fake) == lp.LP_E_STATE
    maps = (ctypes.c_void_p * 3)(256, 256, 256)
    assert lib.lp_convolve_classes(p.handle, None, fake) == lp.LP_E_INVALID
    assert lib.lp_convolve_classes(p.handle, maps, None) == lp.LP_E_INVALID
    assert lib.lp_convolve_classes(p.handle, maps, fake) == lp.LP_E_NOMEM  # unbound
    holes = (ctypes.c_void_p * 3)(256, None, 256)
    assert lib.lp_convolve_classes(p.handle, holes, fake) == lp.LP_E_INVALID
    assert lib.lp_adjoint_class(p.handle, 3, fake, fake) == lp.LP_E_INVALID
    assert lib.lp_adjoint_class(p.handle, -1, fake, fake) == lp.LP_E_INVALID
    assert lib.lp_kernel_spectra(p.handle, None) == lp.LP_E_INVALID
    assert lib.lp_plan_classes(None) == -1
    p.set_classes(1)
    assert p.workspace_bytes == one


def test_reprojection_argument_errors():
    lib = lp.raw()
    sg = lp.LatLonGrid(10, 10, 40.0, -3.0, 0.01, 0.01)
    dg = lp.TMGrid(10, 10, 0.0, 4400.0, 1.0, -3.0, 0.9996, 6367.0)
    fake = ctypes.c_void_p(256)
    ok = lambda s, d: lib.lp_reproject_nn(ctypes.byref(s), fake, ctypes.byref(d), fake, 0, None)
    assert lib.lp_reproject_nn(None, fake, ctypes.byref(dg), fake, 0, None) == lp.LP_E_INVALID
    assert lib.lp_reproject_nn(ctypes.byref(sg), None, ctypes.byref(dg), fake, 0, None) == lp.LP_E_INVALID
    assert lib.lp_reproject_nn(ctypes.byref(sg), fake, ctypes.byref(dg), None, 0, None) == lp.LP_E_INVALID
    for field, bad in [("rows", 0), ("dlat_deg", 0.0), ("dlon_deg", -1.0), ("lat_first_deg", float("nan"))]:
        s2 = lp.LatLonGrid(10, 10, 40.0, -3.0, 0.01, 0.01)
        setattr(s2, field, bad)
        assert ok(s2, dg) == lp.LP_E_INVALID, field
    for field, bad in [("cols", -3), ("pitch_km", 0.0), ("k0", float("inf")), ("radius_km", 0.0),
                       ("y_first_km", float("nan"))]:
        d2 = lp.TMGrid(10, 10, 0.0, 4400.0, 1.0, -3.0, 0.9996, 6367.0)
        setattr(d2, field, bad)
        assert ok(sg, d2) == lp.LP_E_INVALID, field
    big = lp.TMGrid(300000, 10, 0.0, 4400.0, 1.0, -3.0, 0.9996, 6367.0)
    assert ok(sg, big) == lp.LP_E_SIZE


def test_batch_output_rows_errors():
    lib = lp.raw()
    b = lp.Batch([(600, 700), (100, 100)], [0, 0], [(101, 101)])
    for tile, first, count in [(2, 0, 1), (-1, 0, 1), (0, -1, 5), (0, 0, 0), (0, 590, 11), (1, 0, 101)]:
        assert lib.lp_batch_set_output_rows(b._b, tile, first, count) == lp.LP_E_INVALID
    assert lib.lp_batch_set_output_rows(b._b, 0, 10, 590) == lp.LP_OK


def _need_rows(ny, ky, k0, k1):
    cy = (ky - 1) // 2
    return k1 + cy if k0 + cy - (ky - 1) >= 0 else max(k1 + cy, ny + ky - 1 - cy - k0)


@pytest.mark.parametrize("ny,ky,k0,k1", [(4048, 2001, 1000, 3048), (4048, 2001, 0, 4048), (1180, 201, 100, 1080),
                                         (948, 649, 324, 624), (948, 648, 0, 300), (700, 100, 650, 700)])
def test_batch_windows_replan_padding(ny, ky, k0, k1):
    """Output-row windows set before bind choose the padding class from
    max(k1 + cy, ny + ky - 1 - cy - k0): n + floor(k/2) for the whole map,
    ny for a slab whose kept rows have their whole kernel footprint."""
    assert _need_rows(ny, ky, 0, ny) == ny + ky // 2
    b = lp.Batch([(ny, 300)], [0], [(ky, 31)])
    full = b.groups[0]["padding"][0]
    bytes_full = b.workspace_bytes
    b.set_output_rows(0, k0, k1 - k0)
    need = _need_rows(ny, ky, k0, k1)
    ly, _ = lp.spec_lengths()
    py = b.groups[0]["padding"][0]
    assert py == min(L for L in ly if L >= need)
    assert py <= full and (py < full) == (b.workspace_bytes < bytes_full)
    # whole halos: the slab needs no more rows than it has
    cy = (ky - 1) // 2
    if k0 >= ky - 1 - cy and k1 <= ny - cy:
        assert need <= ny
    if k0 == ky - 1 - cy and k1 == ny - cy:
        assert need == ny


def test_band_kernel_matches_oracle_geometry():
    from oracle import latlon as olat
    from paper_1907_02891_amd import latlon
    radial = lambda d: np.exp(-d / 30.0) / (1.0 + d)
    for lat in (0.0, 35.5, 61.0, -48.0):
        a = latlon.band_kernel(radial, lat, 1 / 240, 1 / 240, 20, 33)
        b = olat.band_kernel(radial, lat, 1 / 240, 1 / 240, 20, 33, 6367.0)
        np.testing.assert_allclose(a, b, rtol=1e-13)
    c = latlon.band_centres([0, 10, 30], 50.0, 0.1)
    np.testing.assert_allclose(c, [50.0 - 0.1 * 4.5, 50.0 - 0.1 * 19.5])


def test_window_padding_bounds():
    """Padding may go down to n + floor(k/2) (the input-sized window), no lower."""
    p = lp.Plan(4096, 4096, 1201, 1201)
    assert p.padding == (5400, 5400)
    assert lp.window_padding(4096, 4096, 1201, 1201) == (4800, 4800)
    p.set_padding(4800, 4800)
    assert p.padding == (4800, 4800)
    q = lp.Plan(250, 250, 101, 101)
    q.set_padding(300, 300)  # exactly n + floor(k/2)
    for bad in [(288, 300), (300, 288)]:  # 5-smooth but below the bound
        with pytest.raises(lp.LPError) as ei:
            q.set_padding(*bad)
        assert ei.value.code == lp.LP_E_SIZE
    e = lp.Plan(100, 120, 20, 31)
    assert lp.window_padding(100, 120, 20, 31) == (120, 144)
    e.set_padding(120, 144)
    with pytest.raises(lp.LPError):
        e.set_padding(108, 144)  # 108 < 100 + 10
    # a map whose n + k - 1 exceeds the maximum still gets a plan
    big = lp.Plan(19000, 100, 2001, 3)
    assert big.padding[0] >= 19000 + 1000 and big.padding[0] <= lp.MAX_PY


def test_graph_branches_and_column_split_errors():
    lib = lp.raw()
    b = lp.Batch([(600, 700), (100, 100)], [0, 0], [(101, 101)])
    for n in (0, 5, -1):
        assert lib.lp_batch_set_graph_branches(b._b, n) == lp.LP_E_INVALID
    for n in (1, 2, 3, 4):
        assert lib.lp_batch_set_graph_branches(b._b, n) == lp.LP_OK
    assert lib.lp_batch_set_graph_branches(None, 2) == lp.LP_E_INVALID
    p = lp.Plan(20000, 4, 1001, 3)
    one = ctypes.c_int64()
    assert lib.lp_plan_column_split(p._p, None, ctypes.byref(one)) == lp.LP_E_INVALID
    assert lib.lp_plan_column_split(None, ctypes.byref(one), ctypes.byref(one)) == lp.LP_E_INVALID


def test_timing_interval_errors():
    """lp_plan_timing takes an interval N >= 0 (0 stops; no events are made
    for 0); a negative interval or a null plan is refused."""
    lib = lp.raw()
    p = lp.Plan(300, 200, 31, 31)
    assert lib.lp_plan_timing(p._p, -1) == lp.LP_E_INVALID
    assert lib.lp_plan_timing(p._p, 0) == lp.LP_OK
    assert lib.lp_plan_timing(None, 1) == lp.LP_E_INVALID


def test_poison_setters():
    """The debug fill is switched per plan and per batch; null handles are
    LP_E_INVALID (no device work happens until a call runs the path)."""
    lib = lp.raw()
    assert lib.lp_plan_set_poison(None, 1) == lp.LP_E_INVALID
    assert lib.lp_batch_set_poison(None, 1) == lp.LP_E_INVALID
    p = lp.Plan(64, 48, 5, 7)
    assert lib.lp_plan_set_poison(p._p, 1) == lp.LP_OK
    assert lib.lp_plan_set_poison(p._p, 0) == lp.LP_OK
    b = lp.Batch([(30, 40), (50, 20)], [0, 0], [(5, 5)])
    assert lib.lp_batch_set_poison(b._b, 1) == lp.LP_OK
    assert lib.lp_batch_set_poison(b._b, 0) == lp.LP_OK
