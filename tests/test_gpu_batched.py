"""Batched maps (tiles x bands, several kernels) through lp_convolve_batched:
parity per map against the oracle, HIP-graph replays against direct
launches, and the 64-tile x 3-band workload on sampled pixels."""
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


def small_batch():
    rng = np.random.default_rng(300)
    cy = 25
    Q = rng.random((cy + 1, cy + 1))
    K0 = Q[np.abs(np.arange(51) - cy)][:, np.abs(np.arange(51) - cy)]   # mirror-symmetric
    K1 = rng.random((41, 31))                                            # general
    shapes = [(200, 300), (200, 300), (700, 150), (150, 1500), (900, 800), (901, 799), (37, 20)]
    ids = [0, 1, 0, 1, 0, 1, 1]
    maps = [(synth.radiance_map(a, b, 3, 0.05, (2.0, 8.0), rng) + rng.random((a, b))).astype(np.float32)
            for a, b in shapes]
    return shapes, ids, [K0, K1], maps


def test_batch_parity_and_graph(lp, torch):
    shapes, ids, psfs, maps = small_batch()
    b = lp.Batch(shapes, ids, [p.shape for p in psfs]).bind()
    b.set_kernels(psfs)
    groups = b.groups
    assert len(groups) >= 3, groups
    xs = [torch.from_numpy(m).cuda() for m in maps]
    outs = b.convolve(xs)
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in outs]
    for t, (m, r) in enumerate(zip(maps, res)):
        check(r, oracle.conv_same(m, psfs[ids[t]]), f"batch map {t} {shapes[t]} psf {ids[t]} class {b.tile_group(t)}")
    # graph replays with eager work in between, each against direct launches
    b2 = lp.Batch(shapes, ids, [p.shape for p in psfs]).bind()
    b2.set_kernels(psfs)
    b2.use_graph(False)
    for rep in range(3):
        for x in xs:
            x.mul_(1.5).add_(0.25)          # eager work on the same stream
        torch.cuda.synchronize()
        g = [o.cpu().numpy() for o in b.convolve(xs, outs)]
        d = [o.cpu().numpy() for o in b2.convolve(xs)]
        torch.cuda.synchronize()
        for t in range(len(xs)):
            assert np.array_equal(g[t], d[t]), (rep, t)
    # new output pointers: the table is re-uploaded, results unchanged
    outs2 = [torch.full_like(x, float("nan")) for x in xs]
    g2 = [o.cpu().numpy() for o in b.convolve(xs, outs2)]
    for t in range(len(xs)):
        assert np.array_equal(g2[t], d[t])


@pytest.mark.parametrize("branches", [1, 2, 3])
def test_graph_branches_match_direct(lp, torch, branches):
    """The captured graph with 1 to 4 parallel class branches gives the
    direct launches' results bitwise, over replays with eager work between."""
    shapes, ids, psfs, maps = small_batch()
    b = lp.Batch(shapes, ids, [p.shape for p in psfs]).bind()
    b.set_kernels(psfs)
    b.set_graph_branches(branches)
    d = lp.Batch(shapes, ids, [p.shape for p in psfs]).bind()
    d.set_kernels(psfs)
    d.use_graph(False)
    xs = [torch.from_numpy(m).cuda() for m in maps]
    outs = [torch.empty_like(x) for x in xs]
    for rep in range(3):
        for x in xs:
            x.mul_(0.75).add_(0.5)
        g = [o.cpu().numpy() for o in b.convolve(xs, outs)]
        r = [o.cpu().numpy() for o in d.convolve(xs)]
        for t in range(len(xs)):
            assert np.array_equal(g[t], r[t]), (branches, rep, t)
    with pytest.raises(lp.LPError):
        b.set_graph_branches(5)


def test_batch_in_place(lp, torch):
    shapes, ids, psfs, maps = small_batch()
    b = lp.Batch(shapes, ids, [p.shape for p in psfs]).bind()
    b.set_kernels(psfs)
    xs = [torch.from_numpy(m).cuda() for m in maps]
    ref = [o.cpu().numpy() for o in b.convolve(xs)]
    ys = [x.clone() for x in xs]
    b.convolve(ys, ys)
    for y, r in zip(ys, ref):
        assert np.array_equal(y.cpu().numpy(), r)


def test_batch_variants(lp, torch):
    shapes, ids, psfs, maps = small_batch()
    b = lp.Batch(shapes, ids, [p.shape for p in psfs]).bind()
    b.set_kernels(psfs)
    xs = [torch.from_numpy(m).cuda() for m in maps]
    refs = [oracle.conv_same(m, psfs[ids[t]]) for t, m in enumerate(maps)]
    for g, info in enumerate(b.groups):
        for stage, key in ((lp.STAGE_ROWS, "row_variants"), (lp.STAGE_COLUMNS, "column_variants")):
            for k in range(info[key]):
                b.set_variant(g, stage, k)
                outs = [o.cpu().numpy() for o in b.convolve(xs)]
                for t in range(len(maps)):
                    if b.tile_group(t) == g:
                        check(outs[t], refs[t], f"class {g} stage {stage} variant {k} map {t}")
            b.set_variant(g, stage, 0)
        # the two row directions of a class on different variants (each its own tables)
        n = info["row_variants"]
        for k in range(n if n > 1 else 0):
            b.set_variant(g, lp.STAGE_ROWS, k)
            b.set_variant(g, lp.STAGE_ROWS_INVERSE, (k + 1) % n)
            assert b.variant(g, lp.STAGE_ROWS) == k and b.variant(g, lp.STAGE_ROWS_INVERSE) == (k + 1) % n
            outs = [o.cpu().numpy() for o in b.convolve(xs)]
            for t in range(len(maps)):
                if b.tile_group(t) == g:
                    check(outs[t], refs[t], f"class {g} rows fwd v{k} inv v{(k + 1) % n} map {t}")
        b.set_variant(g, lp.STAGE_ROWS, 0)


@pytest.mark.timeout(900)
def test_batched_workload_sampled(lp, torch):
    """64 tiles (sides 512..3072) x 3 bands, 4 kernels (1201^2): 256 sampled
    pixels per tile-band against the oracle, and the full field of the
    first band of the four smallest tiles."""
    tiles, psf_ids, psfs = synth.batched_inputs()
    shapes, ids, maps = [], [], []
    for t, bands in enumerate(tiles):
        for band in bands:
            shapes.append(band.shape)
            ids.append(int(psf_ids[t]))
            maps.append(band)
    b = lp.Batch(shapes, ids, [p.shape for p in psfs]).bind()
    b.set_kernels(psfs)
    print(f"batched workload: {len(maps)} maps in {len(b.groups)} classes", flush=True)
    xs = [torch.from_numpy(m).cuda() for m in maps]
    outs = b.convolve(xs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(301)
    got, ref = [], []
    for t, (m, o) in enumerate(zip(maps, outs)):
        idx = rng.choice(m.size, 256, replace=False)
        got.append(o.reshape(-1)[torch.from_numpy(idx).cuda()].cpu().numpy())
        ref.append(oracle.conv_same_pixels(m, psfs[ids[t]], idx))
        check(got[-1], ref[-1], f"batched map {t} {m.shape} (256 px)")
    got, ref = np.concatenate(got), np.concatenate(ref)
    check(got, ref, "batched workload sampled")
    # full fields: band 0 of the four smallest tiles (maps 3 t)
    smallest = sorted(range(len(tiles)), key=lambda t: tiles[t][0].size)[:4]
    for t in smallest:
        k = 3 * t
        check(outs[k].cpu().numpy(), oracle.conv_same(maps[k], psfs[ids[k]]),
              f"batched tile {t} band 0 {maps[k].shape} full field")


@pytest.mark.parametrize("case", [(1180, 200, 201, 31, 100, 1080, 1440, 1200),   # whole halos: Py >= ny
                                  (1300, 90, 21, 7, 20, 1180, 1440, 1200)],     # no wrap: Py = 1200 < ny
                         ids=["halo", "short"])
def test_window_padding_slab(lp, torch, case):
    """An overlap-save slab: kept rows [k0, k1) with their whole kernel
    footprint inside the slab, so the class pads only as far as the kept
    rows reach (k1 + cy), here less than the full map's class; in the second
    case less than the map itself (only the first Py rows are transformed).
    The kept rows equal the oracle's."""
    rng = np.random.default_rng(71)
    ny, nx, ky, kx, k0, k1, full, cls = case
    R = rng.random((ny, nx)).astype(np.float32)
    K = rng.random((ky, kx))
    b = lp.Batch([(ny, nx)], [0], [K.shape])
    assert b.groups[0]["padding"][0] == full
    b.set_output_rows(0, k0, k1 - k0)
    assert b.groups[0]["padding"][0] == cls
    b.bind()
    b.set_kernels([K])
    out = b.convolve([torch.from_numpy(R).cuda()])[0]
    torch.cuda.synchronize()
    assert tuple(out.shape) == (k1 - k0, nx)
    ref = oracle.conv_same(R, K)[k0:k1]
    e2, em = oracle.rel_l2(out.cpu().numpy(), ref), oracle.max_err_frac(out.cpu().numpy(), ref)
    print(f"slab window: rel-L2 {e2:.3e} max-err/max {em:.3e}", flush=True)
    assert e2 <= 1e-5 and em <= 1e-5
    # after bind a window needing more rows than the class has is refused
    with pytest.raises(lp.LPError) as ei:
        b.set_output_rows(0, 0, ny)
    assert ei.value.code == lp.LP_E_STATE
    b.set_output_rows(0, k0 + 10, k1 - k0 - 20)  # a narrower window fits the class
    out2 = b.convolve([torch.from_numpy(R).cuda()])[0]
    assert np.array_equal(out2.cpu().numpy(), out.cpu().numpy()[10:-10])


def test_uneven_maps_and_windows_in_one_class(lp, torch):
    """Maps of very different heights in one padding class: the grid spans
    the tallest map, and each map's own tiles (in the inverse rows, only
    those that hold kept rows) are dealt over the XCDs.  Output-row windows
    at the top, in the middle and at the bottom of maps; every kept row
    equals the oracle's, and so does every whole map."""
    rng = np.random.default_rng(404)
    K = rng.random((61, 41))
    shapes = [(1170, 300), (500, 300), (1100, 300), (1100, 300), (800, 300), (1, 300)]
    windows = {2: (0, 100), 3: (450, 37), 4: (700, 100)}
    maps = [rng.random(s).astype(np.float32) for s in shapes]
    b = lp.Batch(shapes, [0] * len(shapes), [K.shape])
    for t, (k0, n) in windows.items():
        b.set_output_rows(t, k0, n)
    b.bind()
    b.set_kernels([K])
    groups, g = b.groups, b.tile_group(0)
    assert [b.tile_group(t) for t in range(5)] == [g] * 5, groups   # the one-row map has a class of its own
    assert groups[g]["padding"] == (1200, 512) and groups[g]["maps"] == 5 and groups[g]["max_ny"] == 1170, groups
    outs = b.convolve([torch.from_numpy(m).cuda() for m in maps])
    torch.cuda.synchronize()
    for t, (m, o) in enumerate(zip(maps, outs)):
        k0, n = windows.get(t, (0, shapes[t][0]))
        got = o.cpu().numpy()
        assert got.shape == (n, shapes[t][1])
        check(got, oracle.conv_same(m, K)[k0:k0 + n], f"uneven map {t} {shapes[t]} rows [{k0}, {k0 + n})")
