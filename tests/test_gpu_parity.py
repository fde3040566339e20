"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Preprocess records, the bit-exact sort, the tile key lists and the rendered
images: at the tiny size against the brute-force oracle, and at the full
1M / 6M sizes (every Gaussian, every key, every pixel, in the launch
configurations the benchmark times) against the tiled oracle, which equals
the brute-force definition.
"""
import numpy as np
import pytest
import torch

from paper_2512_08478_amd import scenes as S
from gpu_util import (assert_pairs_harmless, compare_records, extra_pairs_harmless, image_check,
                      pair_set_check, print_case, rect_pairs, scene_cached, splats_np, u32, u64)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_08478_amd.render import Renderer
    return Renderer()


def gp(scene):
    from paper_2512_08478_amd.render import GaussianParams
    return GaussianParams.from_scene(scene)


# ------------------------------------------------------------------ preprocess

def test_preprocess_tiny(R, orc):
    print_case("preprocess tiny 4096")
    sc, cam = S.tiny_scene()
    splats, dkeys, rects, counts = R.preprocess(gp(sc), cam)
    torch.cuda.synchronize()
    rec = splats_np(splats, sc.n)
    ref = orc.preprocess(sc, cam)
    v = compare_records(orc, rec, ref, cam)
    extra_pairs_harmless(orc, ref, rec, cam, v)
    vis = rec["tx1"] >= rec["tx0"]
    cnt = np.where(vis, (rec["tx1"].astype(np.int64) - rec["tx0"] + 1) * (rec["ty1"].astype(np.int64) - rec["ty0"] + 1), 0)
    c = u32(counts)
    assert int(c[0]) == cnt.sum() and int(c[1]) == vis.sum()
    # the visible depth key range
    vk = rec["depth"][vis].astype(np.float32).view(np.uint32)
    assert int(c[2]) == int(vk.min()) and int(c[3]) == int(vk.max())
    # the compact tile rects match the records' pixel bboxes
    tr = u32(rects).reshape(-1, 2)[vis]
    np.testing.assert_array_equal(tr[:, 0] & 0xFFFF, rec["tx0"][vis])
    np.testing.assert_array_equal(tr[:, 0] >> 16, rec["ty0"][vis])
    np.testing.assert_array_equal(tr[:, 1] & 0xFFFF, rec["tx1"][vis])
    np.testing.assert_array_equal(tr[:, 1] >> 16, rec["ty1"][vis])
    # depth sort keys: float32 depth bits, the largest key when culled
    expect = np.where(vis, rec["depth"].view(np.uint32), np.uint32(0xFFFFFFFF))
    np.testing.assert_array_equal(u32(dkeys), expect)


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_preprocess_sh_degrees(R, orc, deg):
    print_case(f"preprocess sh degree {deg}")
    rng = np.random.default_rng(40 + deg)
    sc, cam = S.tiny_scene(n=2000)
    K = (deg + 1) ** 2
    sh = np.zeros((sc.n, K, 3), np.float32)
    sh[:, 0] = sc.sh[:, 0]
    if K > 1:
        sh[:, 1:] = rng.normal(0, 0.2, (sc.n, K - 1, 3))
    sc = S.Scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sh, deg)
    cam2 = S.pinhole_camera(S.look_at((1.5, 1.0, -2.5)), 200, 150, 50.0)
    splats = R.preprocess(gp(sc), cam2)[0]
    torch.cuda.synchronize()
    compare_records(orc, splats_np(splats, sc.n), orc.preprocess(sc, cam2), cam2)


def test_preprocess_model_transform(R, orc):
    print_case("preprocess with model transform")
    from scipy.spatial.transform import Rotation
    sc, _ = S.medium_scene(n=20000)
    A = 0.7 * Rotation.from_euler("xyz", [0.4, -1.0, 0.3]).as_matrix()
    sc.model = np.concatenate([A, np.array([[1.0], [-0.5], [2.0]])], 1).astype(np.float32)
    cam = S.pinhole_camera(S.look_at((2.0, 1.0, -9.0)), 640, 480, 60.0)
    splats = R.preprocess(gp(sc), cam)[0]
    torch.cuda.synchronize()
    compare_records(orc, splats_np(splats, sc.n), orc.preprocess(sc, cam), cam)


@pytest.mark.parametrize("workload", ["medium", "large"])
def test_preprocess_records_full_size(R, orc, workload):
    """Every Gaussian's record of the 1M and 6M frames against the oracle,
    and the (Gaussian, tile) pairs of the benchmark's tile shape: all of the
    oracle's, plus only harmless extras."""
    print_case(f"preprocess records, all Gaussians, {workload}")
    sc, cam = scene_cached(workload)
    splats, dkeys, rects, counts = R.preprocess(gp(sc), cam)
    torch.cuda.synchronize()
    rec = splats_np(splats, sc.n)
    ref = orc.preprocess(sc, cam)
    v = compare_records(orc, rec, ref, cam)
    tile = (32, 16) if workload == "medium" else (8, 8)
    n_o, n_x = pair_set_check(orc, ref, rec, cam, v, tile)
    c = u32(counts)
    assert int(c[1]) == int((rec["px1"] >= rec["px0"]).sum())
    print(f"{workload}: {int(v.sum())} visible records compared, {n_o} oracle pairs, "
          f"{n_x} harmless extra pairs")


# ------------------------------------------------------------------ sort

SIZES = [1, 2, 63, 64, 65, 4095, 4096, 4097, 3 * 4096 + 17, 100_003]


def sort_pairs_gpu(keys, vals, key_bits, radix_bits=8, sort_mode=0):
    from paper_2512_08478_amd import _lib as L
    import ctypes
    lib = L.load()
    s = L.default_settings(radix_bits=radix_bits, sort_mode=sort_mode)
    n = len(keys)
    kin = torch.from_numpy(keys.view(np.int64)).cuda()
    vin = torch.from_numpy(vals.view(np.int32)).cuda()
    kout = torch.empty_like(kin)
    vout = torch.empty_like(vin)
    ws_b = lib.gs_workspace_size(L.GS_STAGE_SORT_PAIRS, 0, n, None, ctypes.byref(s))
    ws = torch.empty(ws_b, dtype=torch.uint8, device="cuda")
    st = lib.gs_sort_pairs(n, ctypes.c_void_p(kin.data_ptr()), ctypes.c_void_p(vin.data_ptr()),
                           key_bits, ctypes.c_void_p(kout.data_ptr()), ctypes.c_void_p(vout.data_ptr()),
                           ctypes.byref(s), ctypes.c_void_p(ws.data_ptr()), ws_b,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check(st, "gs_sort_pairs")
    torch.cuda.synchronize()
    # the input must be untouched
    np.testing.assert_array_equal(u64(kin), keys)
    return u64(kout), u32(vout)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("kind", S.SORT_KEY_KINDS)
def test_sort_pairs_bitexact(R, orc, kind, mode):
    for n in SIZES:
        print_case(f"sort_pairs {kind} n={n} mode={mode}")
        k, v = S.sort_keys(kind, n, seed=n)
        kb = 45 if kind in ("random45",) else 64
        ks, vs = sort_pairs_gpu(k, v, kb, sort_mode=mode)
        rk, rv = orc.stable_sort_pairs(k, v)
        np.testing.assert_array_equal(ks, rk, err_msg=f"{kind} n={n}")
        np.testing.assert_array_equal(vs, rv, err_msg=f"{kind} n={n}")


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("bits", [6, 7, 8])
def test_sort_pairs_digit_widths(R, orc, bits, mode):
    for kind in ("random64", "depth_like", "tile_runs"):
        print_case(f"sort_pairs bits={bits} {kind} mode={mode}")
        k, v = S.sort_keys(kind, 50_001, seed=bits)
        ks, vs = sort_pairs_gpu(k, v, 64, radix_bits=bits, sort_mode=mode)
        rk, rv = orc.stable_sort_pairs(k, v)
        np.testing.assert_array_equal(ks, rk)
        np.testing.assert_array_equal(vs, rv)


def test_sort_pairs_large(R, orc):
    print_case("sort_pairs depth_like 10M")
    k, v = S.sort_keys("depth_like", 10_000_000, seed=3)
    ks, vs = sort_pairs_gpu(k, v, 45)
    perm = np.argsort(k, kind="stable")
    np.testing.assert_array_equal(ks, k[perm])
    np.testing.assert_array_equal(vs, v[perm])


def test_sort_pairs_empty(R):
    print_case("sort_pairs n=0")
    ks, vs = sort_pairs_gpu(np.zeros(0, np.uint64), np.zeros(0, np.uint32), 64)
    assert ks.size == 0 and vs.size == 0


# ------------------------------------------------------------------ keys + image

def expected_sorted_pairs(rec, tiles_x):
    """The unique stable order of (tile, depth bits, index) over the GPU's
    own (Gaussian, tile) pairs -- the property the sort must produce."""
    keys, vals = [], []
    for g in np.nonzero(rec["tx1"] >= rec["tx0"])[0]:
        a = rec[g]
        zb = np.uint64(np.float32(a["depth"]).view(np.uint32))
        for ty in range(a["ty0"], a["ty1"] + 1):
            for tx in range(a["tx0"], a["tx1"] + 1):
                keys.append((np.uint64(ty * tiles_x + tx) << np.uint64(32)) | zb)
                vals.append(g)
    keys = np.array(keys, np.uint64)
    vals = np.array(vals, np.uint32)
    perm = np.argsort(keys, kind="stable")
    return keys[perm], vals[perm]


def test_sort_keys_tiny(R, orc):
    print_case("gs_sort keys tiny")
    sc, cam = S.tiny_scene()
    fr = R.forward(gp(sc), cam, want_keys=True)
    torch.cuda.synchronize()
    rec = splats_np(fr.splats, sc.n)
    n = fr.capacity
    ek, ev = expected_sorted_pairs(rec, 16)
    np.testing.assert_array_equal(u64(fr.keys)[:n], ek)
    np.testing.assert_array_equal(u32(fr.values)[:n], ev)
    # tile ranges
    rng = u32(fr.ranges)[:2 * R.tiles(cam)].reshape(-1, 2)
    tile = (ek >> np.uint64(32)).astype(np.int64)
    for t in range(rng.shape[0]):
        idx = np.nonzero(tile == t)[0]
        if idx.size:
            assert (rng[t, 0], rng[t, 1]) == (idx[0], idx[-1] + 1)
        else:
            assert rng[t, 0] == rng[t, 1]
    # against the oracle's own FP64 key list: same pairs up to harmless ones
    ref = orc.preprocess(sc, cam)
    ok, ov = orc.keys(ref, cam)
    gset = set(zip((ek >> np.uint64(32)).tolist(), ev.tolist()))
    oset = set(zip((ok >> np.uint64(32)).tolist(), ov.tolist()))
    assert oset - gset == set()
    extra = gset - oset
    if extra:
        t, g = map(np.array, zip(*extra))
        w = orc.pair_max_weight(ref, cam, g, t)
        assert w.max() < 1 / 255


def expected_sorted_pairs_np(rec, tiles_x):
    """Vectorised expected_sorted_pairs for full-size frames: every
    (Gaussian, tile) pair of the GPU's own records, keyed by (tile, float32
    depth bits), in numpy's stable order."""
    vis = np.nonzero(rec["tx1"] >= rec["tx0"])[0]
    r = rec[vis]
    w = (r["tx1"] - r["tx0"] + 1).astype(np.int64)
    h = (r["ty1"] - r["ty0"] + 1).astype(np.int64)
    cnt = w * h
    rep = np.repeat(np.arange(vis.size), cnt)
    local = np.arange(int(cnt.sum()), dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    wr = w[rep]
    ty = r["ty0"][rep] + local // wr
    tx = r["tx0"][rep] + local % wr
    zb = np.float32(r["depth"]).view(np.uint32).astype(np.uint64)[rep]
    keys = ((ty * tiles_x + tx).astype(np.uint64) << np.uint64(32)) | zb
    vals = vis[rep].astype(np.uint32)
    perm = np.argsort(keys, kind="stable")
    return keys[perm], vals[perm]


@pytest.mark.parametrize("workload,shape,mode", [("medium", (32, 16, 7), 0), ("medium", (16, 16, 8), 0),
                                                 ("medium", (64, 32, 6), 0), ("medium", (64, 16, 8), 1),
                                                 ("large", (8, 8, 8), 0), ("large", (16, 8, 6), 0),
                                                 ("medium", (16, 16, 8), 1), ("large", (8, 8, 8), 1)])
def test_sort_keys_full_size(R, orc, workload, shape, mode):
    """gs_sort at the benchmark sizes: keys, permutation and tile ranges
    bit-exact against numpy's stable sort of the GPU's own pairs.  Sort mode
    1 covers the onesweep look-back across the switch from the depth passes
    (visible Gaussians only after the first) to the tile passes (more
    partitions): every look-back word must be clear when its pass starts."""
    tw, th, bits = shape
    print_case(f"gs_sort keys {workload} tiles {tw}x{th} {bits}-bit digits, sort mode {mode}")
    from paper_2512_08478_amd.render import Renderer
    Rs = Renderer(dict(tile_w=tw, tile_h=th, radix_bits=bits, sort_mode=mode))
    sc, cam = scene_cached(workload)
    fr = Rs.forward(gp(sc), cam, want_keys=True)
    torch.cuda.synchronize()
    tiles_x = -(-cam.width // tw)
    rec = splats_np(fr.splats, sc.n, (tw, th))
    ek, ev = expected_sorted_pairs_np(rec, tiles_x)
    n = fr.capacity
    assert n == ek.size
    np.testing.assert_array_equal(u64(fr.keys)[:n], ek)
    np.testing.assert_array_equal(u32(fr.values)[:n], ev)
    tiles = Rs.tiles(cam)
    rng = u32(fr.ranges)[:2 * tiles].reshape(-1, 2).astype(np.int64)
    tile = (ek >> np.uint64(32)).astype(np.int64)
    starts = np.searchsorted(tile, np.arange(tiles), "left")
    ends = np.searchsorted(tile, np.arange(tiles), "right")
    nonempty = ends > starts
    np.testing.assert_array_equal(rng[nonempty, 0], starts[nonempty])
    np.testing.assert_array_equal(rng[nonempty, 1], ends[nonempty])
    assert np.all(rng[~nonempty, 0] == rng[~nonempty, 1])
    # the key list's (Gaussian, tile) pairs against the oracle's exact rects:
    # every oracle pair is there, every extra one is harmless
    ref = orc.preprocess(sc, cam)
    vis = np.nonzero(ref.visible)[0]
    it = ref.i[vis]
    o = rect_pairs(it[:, orc.I_PX0], it[:, orc.I_PX1], it[:, orc.I_PY0], it[:, orc.I_PY1],
                   vis, tw, th, tiles_x)
    g = (ev.astype(np.int64) << 32) | tile
    assert np.unique(g).size == g.size
    missing = np.setdiff1d(o, g)
    assert missing.size == 0, missing[:5]
    extra = np.setdiff1d(g, o)
    assert_pairs_harmless(orc, ref, cam, extra, (tw, th))
    print(f"{workload}: {n} pairs ({o.size} oracle, {extra.size} harmless extra), "
          f"{int(nonempty.sum())} non-empty tiles")


@pytest.mark.parametrize("mode", [0, 1])
def test_sort_depth_bits(R, mode):
    """The depth passes over the visible key range (depth_bits planned from
    the counts) give the same sort as all 32 bits; a range wider than the
    planned bits raises bit 1 of the status flag."""
    print_case(f"gs_sort depth_bits, sort mode {mode}")
    from paper_2512_08478_amd.render import Renderer, depth_range_bits
    Rs = Renderer(dict(tile_w=16, tile_h=16, radix_bits=8, sort_mode=mode))
    sc, cam = S.medium_scene(n=300_000)
    p = gp(sc)
    full = Rs.forward(p, cam, depth_bits=0, want_keys=True)
    torch.cuda.synchronize()
    cn = u32(full.counts)
    b = depth_range_bits(cn)
    print(f"visible depth key range {int(cn[3]) - int(cn[2])}: {b} bits")
    assert 20 <= b <= 30
    ref_v, ref_k = u32(full.values).copy(), u64(full.keys).copy()
    for bits in (b, b + 1, 32):
        fr = Rs.forward(p, cam, depth_bits=bits, want_keys=True)
        torch.cuda.synchronize()
        assert int(u32(fr.flag)[0]) == 0, bits
        np.testing.assert_array_equal(u32(fr.values), ref_v, err_msg=f"depth_bits {bits}")
        np.testing.assert_array_equal(u64(fr.keys), ref_k, err_msg=f"depth_bits {bits}")
    # too few bits: reported, and the sort stays a permutation of the pairs
    fr = Rs.forward(p, cam, capacity=full.capacity, depth_bits=b - 2)
    torch.cuda.synchronize()
    assert int(u32(fr.flag)[0]) & 2
    assert sorted(u32(fr.values).tolist()) == sorted(ref_v.tolist())


def test_render_tiny_whole_image(R, orc):
    print_case("render tiny 256x256 vs brute force")
    sc, cam = S.tiny_scene()
    fr = R.forward(gp(sc), cam)
    img = fr.image.cpu().numpy().reshape(-1, 4)
    T = fr.T_final.cpu().numpy().reshape(-1)
    ref = orc.render_pixels(orc.preprocess(sc, cam), cam, orc.all_pixels(cam))
    e, nflag, nloose = image_check(img, ref, max_flagged=0.005, max_loosened=0.001, T=T)
    print(f"tiny max err {e:.2e}, flagged {nflag}, jump above 1e-4 {nloose}")


def test_blend_counts_match_oracle(R, orc):
    """The optional per-pixel blend count equals the oracle's count of
    composited Gaussians wherever no decision is near a threshold (whole
    tiny and 1M images), and requesting it leaves the image bitwise
    unchanged."""
    print_case("n_blend tiny 256x256 + 1M 1920x1080, whole images")
    for sc, cam in (S.tiny_scene(), scene_cached("medium")):
        fr = R.forward(gp(sc), cam)
        nb = torch.empty((cam.height, cam.width), dtype=torch.int32, device="cuda")
        img2, T2, last2 = R.rasterize(fr.splats, fr.values, fr.ranges, cam, n_blend=nb)
        assert torch.equal(img2, fr.image) and torch.equal(last2, fr.last)
        ref = orc.render_image(orc.preprocess(sc, cam), cam, tiled=True)
        got = nb.cpu().numpy()
        ok = (ref["margin"] >= 1e-5) & (ref["flags"] == 0)
        assert ok.mean() > 0.94
        np.testing.assert_array_equal(got[ok], ref["n_blend"][ok])
        assert (got <= fr.last.cpu().numpy()).all()
        print(f"n_blend mean {got.mean():.1f}, checked {int(ok.sum())} px")


MEDIUM_CASES = ([(v, (32, 16, 6)) for v in range(8)] + [(0, (16, 16, 8)), (0, (8, 8, 7)),
                                                         (0, (64, 32, 6)), (3, (32, 32, 7))])


@pytest.mark.parametrize("view,shape", MEDIUM_CASES)
def test_render_medium_1080p_whole_image(R, orc, view, shape):
    """Every pixel of the 1M frame (each of the 8 orbit views, in the
    benchmark's launch configuration and two others) against the tiled FP64
    oracle, which equals the brute-force definition."""
    print_case(f"render 1M 1920x1080 view {view}, whole image, tiles {shape[0]}x{shape[1]}, "
               f"{shape[2]}-bit digits")
    from paper_2512_08478_amd.render import Renderer
    Rs = Renderer(dict(tile_w=shape[0], tile_h=shape[1], radix_bits=shape[2]))
    sc, _ = scene_cached("medium")
    cam = S.orbit_camera(view, 8, 8.0, 1920, 1080)
    fr = Rs.forward(gp(sc), cam)
    img = fr.image.cpu().numpy().reshape(-1, 4)
    T = fr.T_final.cpu().numpy().reshape(-1)
    ref = orc.render_pixels(orc.preprocess(sc, cam), cam, orc.all_pixels(cam), tiled=True)
    e, nflag, nloose = image_check(img, ref, T=T)
    print(f"1M view {view}: max err unflagged {e:.2e}, flagged {nflag}, jump above 1e-4 {nloose}, "
          f"instances {fr.capacity}")


@pytest.mark.parametrize("shape", [(8, 8, 8, 5), (8, 8, 8, 1), (16, 16, 8, 1)])
def test_render_large_6m_whole_image(R, orc, shape):
    """Every pixel of the 6M frame (eye inside the cloud; its densest 8x8
    tiles hold tens of thousands of splats) against the tiled oracle, in the
    benchmark's launch configuration (8x8 tiles, heavy tiles first, each
    quadrant in 4 bands of 2 rows) and with whole quadrants."""
    print_case(f"render 6M 1920x1080 whole image, tiles {shape[0]}x{shape[1]}, "
               f"raster_order {shape[3]}")
    from paper_2512_08478_amd.render import Renderer
    Rs = Renderer(dict(tile_w=shape[0], tile_h=shape[1], radix_bits=shape[2],
                       raster_order=shape[3]))
    sc, cam = scene_cached("large")
    fr = Rs.forward(gp(sc), cam)
    img = fr.image.cpu().numpy().reshape(-1, 4)
    T = fr.T_final.cpu().numpy().reshape(-1)
    rec = splats_np(fr.splats, sc.n)
    culled = float(np.mean(rec["px1"] < rec["px0"]))
    print(f"6M culled fraction {culled:.3f}, instances {fr.capacity}")
    assert 0.35 <= culled <= 0.45
    ref = orc.render_pixels(orc.preprocess(sc, cam), cam, orc.all_pixels(cam), tiled=True)
    e, nflag, nloose = image_check(img, ref, T=T)
    # the densest tiles (where the compositing kernel's long walks run)
    rng_ = u32(fr.ranges)[:2 * Rs.tiles(cam)].reshape(-1, 2).astype(np.int64)
    lens = rng_[:, 1] - rng_[:, 0]
    print(f"6M: max err unflagged {e:.2e}, flagged {nflag}, jump above 1e-4 {nloose}; "
          f"longest tile list {lens.max()}, 99th percentile {np.percentile(lens, 99):.0f}")


# ------------------------------------------------------------------ edge cases + invariances

def test_empty_and_all_culled(R):
    print_case("n=0 and all-culled")
    from paper_2512_08478_amd.render import Renderer
    sc, cam = S.tiny_scene(n=16)
    r2 = Renderer(dict(bg=(0.2, 0.4, 0.6)))
    empty = sc.subset(np.arange(0))
    fr = r2.forward(gp(empty), cam)
    img = fr.image.cpu().numpy()
    assert np.all(img[..., :3] == np.float32([0.2, 0.4, 0.6])) and np.all(img[..., 3] == 0)
    behind = sc.subset(np.arange(16))
    behind.means[:, 2] = -10.0  # all behind the camera
    fr = r2.forward(gp(behind), cam)
    img = fr.image.cpu().numpy()
    assert fr.capacity == 0
    assert np.all(img[..., 3] == 0)


def test_tile_shape_and_digit_width_invariance(R):
    print_case("tile shapes / digit widths give bitwise-identical images")
    from paper_2512_08478_amd.render import Renderer
    sc, cam = S.tiny_scene()
    cam = S.pinhole_camera(S.look_at((0.3, -0.2, -3.0)), 250, 190, 60.0)  # ragged edge tiles
    base = R.forward(gp(sc), cam).image.cpu().numpy()
    for tw, th, bits, mode, order in [(8, 8, 8, 0, 0), (16, 8, 7, 1, 1), (32, 8, 6, 0, 0),
                                      (32, 16, 8, 1, 1), (16, 16, 6, 1, 0), (16, 16, 7, 0, 1),
                                      (8, 8, 8, 0, 1), (32, 16, 7, 0, 0), (32, 32, 6, 0, 1),
                                      (64, 16, 7, 1, 1), (64, 32, 8, 0, 0), (64, 32, 6, 0, 1),
                                      (8, 8, 8, 0, 2), (16, 8, 7, 1, 3), (32, 16, 8, 0, 2),
                                      (64, 32, 6, 1, 3), (8, 8, 7, 0, 4), (16, 16, 8, 0, 5)]:
        img = Renderer(dict(tile_w=tw, tile_h=th, radix_bits=bits, sort_mode=mode,
                            raster_order=order)).forward(gp(sc), cam).image.cpu().numpy()
        np.testing.assert_array_equal(img, base,
                                      err_msg=f"{tw}x{th} bits {bits} mode {mode} order {order}")


@pytest.mark.parametrize("order,tile", [(0, 8), (1, 8), (2, 8), (3, 8), (4, 8), (5, 8),
                                        (1, 32), (3, 32)])
def test_tile_order_is_a_permutation(R, order, tile):
    """8x8 tiles at 1080p (32,400 tiles): the order comes from the class and
    order kernels; 32x16 (4,080 tiles): from the one-workgroup kernel."""
    print_case(f"tile order written by the sort (raster_order {order}, {tile}x{tile // 2 if tile > 8 else 8} tiles)")
    from paper_2512_08478_amd.render import Renderer
    Rs = Renderer(dict(tile_w=tile, tile_h=tile // 2 if tile > 8 else 8, raster_order=order))
    sc, cam = S.medium_scene(n=200_000)
    fr = Rs.forward(gp(sc), cam)
    tiles = Rs.tiles(cam)
    rg = u32(fr.ranges)
    lens = (rg[1:2 * tiles:2].astype(np.int64) - rg[0:2 * tiles:2]).clip(min=0)
    if order & 1:
        perm = rg[2 * tiles:3 * tiles].astype(np.int64)
        assert sorted(perm.tolist()) == list(range(tiles))
        cls = np.minimum(np.floor(np.log2(lens[perm] + 1)), 15)
        assert np.all(np.diff(cls) <= 0)      # longest classes first
    # the backward walks the same order: gradients exist and are finite
    g = Rs.backward(gp(sc), cam, fr, torch.ones_like(fr.image))
    assert all(torch.isfinite(t).all() for t in g)
    if order >> 1:
        # half-quadrant units: every per-pixel output of the forward equals
        # the whole-quadrant walk's bitwise (the backward reads T_final and
        # the last splat index), and the gradients agree up to the order of
        # the backward's float atomics (which differs from run to run)
        R0 = Renderer(dict(tile_w=Rs.settings.tile_w, tile_h=Rs.settings.tile_h,
                           raster_order=order & 1))
        f0 = R0.forward(gp(sc), cam)
        for name in ("image", "T_final", "last"):
            assert torch.equal(getattr(f0, name), getattr(fr, name)), name
        nb = []
        for Rx, fx in ((R0, f0), (Rs, fr)):
            nb.append(torch.zeros((cam.height, cam.width), dtype=torch.int32, device="cuda"))
            Rx.rasterize(fx.splats, fx.values, fx.ranges, cam, n_blend=nb[-1])
        assert torch.equal(nb[0], nb[1]) and int(nb[0].sum()) > 0
        g0 = R0.backward(gp(sc), cam, f0, torch.ones_like(f0.image))
        for a, b in zip(g0, g):
            assert float((b - a).norm()) <= 1e-5 * float(a.norm())


@pytest.mark.parametrize("tile", [(8, 8), (32, 16)])
def test_tile_order_with_no_instances(R, tile):
    """A capacity given but no instance in the frame: every tile is empty,
    and the heavy-first order is still a permutation of all tiles (1080p:
    32,400 tiles at 8x8, ordered by the class and order kernels; 4,080 at
    32x16, by the one-workgroup kernel)."""
    print_case(f"tile order of an empty frame, {tile[0]}x{tile[1]} tiles")
    from paper_2512_08478_amd.render import Renderer
    sc, _ = S.tiny_scene()
    cam = S.pinhole_camera(S.look_at((0.0, 0.0, -3.0)), 1920, 1080, 60.0)
    sc = sc.subset(np.arange(16))
    sc.means[:, 2] = -10.0  # all behind the camera
    Rs = Renderer(dict(tile_w=tile[0], tile_h=tile[1], raster_order=1))
    fr = Rs.forward(gp(sc), cam, capacity=1024)
    tiles = Rs.tiles(cam)
    rg = u32(fr.ranges)
    assert np.all(rg[:2 * tiles] == 0)
    assert sorted(rg[2 * tiles:3 * tiles].tolist()) == list(range(tiles))
    assert np.all(fr.image.cpu().numpy()[..., 3] == 0)


def test_shuffle_and_repeat_invariance(R):
    print_case("input shuffle and repeated runs")
    sc, cam = S.tiny_scene()
    a = R.forward(gp(sc), cam).image.cpu().numpy()
    b = R.forward(gp(sc), cam).image.cpu().numpy()
    np.testing.assert_array_equal(a, b)
    perm = np.random.default_rng(5).permutation(sc.n)
    c = R.forward(gp(sc.subset(perm)), cam).image.cpu().numpy()
    np.testing.assert_array_equal(a, c)


def generation_order(dkeys, rects, tiles_x):
    """(tile, Gaussian) instances in the order key generation emits them:
    visible Gaussians by depth key (index order among equal keys), each
    Gaussian's tiles row-major."""
    vis = np.nonzero(dkeys != 0xFFFFFFFF)[0]
    vis = vis[np.argsort(dkeys[vis], kind="stable")]
    r = rects.reshape(-1, 2)
    out = []
    for g in vis:
        tx0, ty0 = int(r[g, 0] & 0xFFFF), int(r[g, 0] >> 16)
        tx1, ty1 = int(r[g, 1] & 0xFFFF), int(r[g, 1] >> 16)
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                out.append((ty * tiles_x + tx, g))
    return np.array(out, dtype=np.int64).reshape(-1, 2)


@pytest.mark.parametrize("mode", [0, 1])
def test_capacity_overflow_keeps_the_documented_instances(mode):
    """A too-small capacity raises bit 0 of the flag and keeps exactly the
    instances gs_sort documents: sort mode 1 the first `capacity` in
    generation (depth) order, sort mode 0 those the first tile-digit pass
    places below `capacity`; each tile's list holds its kept instances in
    depth order.  The full capacity clears the flag."""
    from paper_2512_08478_amd.render import Renderer
    print_case(f"capacity overflow, sort mode {mode}")
    bits = 6
    Rm = Renderer(dict(sort_mode=mode, radix_bits=bits))
    sc, cam = S.tiny_scene()
    p = gp(sc)
    pre = Rm.preprocess(p, cam)
    tot = int(u32(pre[3])[0])
    tiles = Rm.tiles(cam)
    tx = (cam.width + 15) // 16
    gen = generation_order(u32(pre[1]), u32(pre[2]), tx)
    assert len(gen) == tot
    cap = tot // 2
    if mode == 1:
        kept = gen[:cap]
    else:
        kept = gen[np.argsort(gen[:, 0] & ((1 << bits) - 1), kind="stable")][:cap]
    _, values, ranges, flag, _ = Rm.sort(sc.n, *pre, cam, capacity=cap)
    torch.cuda.synchronize()
    assert int(u32(flag)[0]) & 1 == 1
    rng = u32(ranges)[:2 * tiles].reshape(-1, 2).astype(np.int64)
    vals = u32(values)
    assert rng[:, 1].max() <= cap
    order = np.argsort(kept[:, 0], kind="stable")   # kept instances by tile, generation order within
    kt = kept[order]
    for t in range(tiles):
        want = kt[kt[:, 0] == t, 1]
        got = vals[rng[t, 0]:rng[t, 1]] if rng[t, 1] > rng[t, 0] else np.zeros(0, np.uint32)
        np.testing.assert_array_equal(got, want, err_msg=f"tile {t}")
    _, values, ranges, flag, _ = Rm.sort(sc.n, *pre, cam, capacity=tot)
    torch.cuda.synchronize()
    assert int(u32(flag)[0]) == 0


def test_sort_checked_reports_the_required_capacity(R):
    """gs_sort_checked returns GS_ERR_CAPACITY with the instance count when
    the capacity is short, and otherwise sorts exactly as gs_sort."""
    import ctypes
    from paper_2512_08478_amd import _lib as L
    print_case("gs_sort_checked")
    lib = L.load()
    sc, cam = S.tiny_scene()
    p = gp(sc)
    pre = R.preprocess(p, cam)
    torch.cuda.synchronize()
    tot = int(u32(pre[3])[0])
    _, v_ref, r_ref, _, _ = R.sort(sc.n, *pre, cam, capacity=tot)
    v_ref, r_ref = u32(v_ref).copy(), u32(r_ref).copy()
    c, s = L.make_camera(cam), R.settings
    tiles = R.tiles(cam)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for cap, want in ((tot - 1, L.GS_ERR_CAPACITY), (tot, L.GS_OK), (tot + 100, L.GS_OK)):
        values = torch.zeros(max(cap, 1), dtype=torch.int32, device="cuda")
        ranges = torch.zeros(3 * tiles, dtype=torch.int32, device="cuda")
        flag = torch.zeros(1, dtype=torch.int32, device="cuda")
        wsb = lib.gs_workspace_size(L.GS_STAGE_SORT, sc.n, cap, ctypes.byref(c), ctypes.byref(s))
        ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
        req = ctypes.c_int64(-1)
        st = lib.gs_sort_checked(sc.n, *[ptr(t) for t in pre], ctypes.byref(c), ctypes.byref(s),
                                 cap, None, ptr(values), ptr(ranges), ptr(flag), ptr(ws), ws.numel(),
                                 ctypes.byref(req), stream)
        torch.cuda.synchronize()
        assert st == want, (cap, st)
        assert req.value == tot
        if want == L.GS_OK:
            assert int(u32(flag)[0]) == 0
            np.testing.assert_array_equal(u32(ranges)[:2 * tiles], r_ref[:2 * tiles])
            np.testing.assert_array_equal(u32(values)[:tot], v_ref[:tot])
        else:
            assert int(u32(values).max()) == 0  # nothing sorted


@pytest.mark.parametrize("bits", [6, 8])
def test_sort_pairs32_bitexact(R, bits):
    """The 32-bit-key sort: keys and the permutation equal NumPy's stable
    argsort, with and without explicit values and output keys."""
    from paper_2512_08478_amd.render import Renderer
    Rs = Renderer(dict(radix_bits=bits))
    rng = np.random.default_rng(77)
    for n in (1, 63, 64, 4097, 100003, 1_500_000):
        for kind in ("random", "depth", "few"):
            print_case(f"sort_pairs32 {kind} n={n} bits={bits}")
            if kind == "random":
                k = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
            elif kind == "depth":
                k = rng.uniform(0.2, 40.0, n).astype(np.float32).view(np.uint32)
                k[rng.random(n) < 0.3] = 0xFFFFFFFF  # culled
            else:
                k = rng.integers(0, 3, n).astype(np.uint32) << np.uint32(20)
            kt = torch.from_numpy(k.view(np.int32)).cuda()
            perm = np.argsort(k, kind="stable").astype(np.uint32)
            ks, vs = Rs.sort_pairs32(kt, want_keys=True)
            np.testing.assert_array_equal(u32(vs), perm)
            np.testing.assert_array_equal(u32(ks), k[perm])
            vals = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
            _, vs2 = Rs.sort_pairs32(kt, torch.from_numpy(vals.view(np.int32)).cuda())
            np.testing.assert_array_equal(u32(vs2), vals[perm])
            np.testing.assert_array_equal(u32(kt), k)  # input untouched
