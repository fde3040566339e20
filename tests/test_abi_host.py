"""Host-side checks of the C ABI: the library loads, exports every function
include/gs.h declares, and rejects bad arguments before any HIP call (so
these run without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2512_08478_amd import _lib as L
from paper_2512_08478_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2512_08478_amd import build
        build.build()
    return L.load()


def header_functions():
    txt = open(os.path.join(ROOT, "include", "gs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 11
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(L.EXPORTED) <= set(names)


def test_version_and_status_strings(lib):
    assert b"gfx950" in lib.gs_version()
    assert L.status_string(0) == "ok"
    for s in range(1, 7):
        assert L.status_string(s) != "unknown status"
    assert L.status_string(99) == "unknown status"


def test_default_settings(lib):
    s = L.default_settings()
    assert (s.tile_w, s.tile_h, s.radix_bits, s.sort_mode, s.raster_order) == (16, 16, 8, 0, 1)
    assert s.depth_bits == 0
    assert s.eps2d == pytest.approx(0.3)
    assert s.alpha_min == pytest.approx(1 / 255)
    assert s.alpha_max == pytest.approx(0.99)
    assert s.t_eps == pytest.approx(1e-4)
    assert s.clip == pytest.approx(1.3)
    assert list(s.bg) == [0.0, 0.0, 0.0]


def cam_1080():
    return L.make_camera(S.orbit_camera(0, 8, 8.0, 1920, 1080))


def test_key_bits_and_workspace_sizes(lib):
    c, s = cam_1080(), L.default_settings()
    # 120 x 68 = 8160 tiles -> 13 tile bits above the 32 depth bits
    assert lib.gs_sort_key_bits(ctypes.byref(c), ctypes.byref(s)) == 45
    s8 = L.default_settings(tile_w=8, tile_h=8)
    assert lib.gs_sort_key_bits(ctypes.byref(c), ctypes.byref(s8)) == 32 + 15  # 240x135
    tiny = L.make_camera(S.tiny_scene(n=4)[1])
    assert lib.gs_sort_key_bits(ctypes.byref(tiny), ctypes.byref(s)) == 40  # 256 tiles
    assert lib.gs_workspace_size(L.GS_STAGE_PREPROCESS, 1_000_000, 0, ctypes.byref(c), ctypes.byref(s)) >= 3907 * 8
    w1 = lib.gs_workspace_size(L.GS_STAGE_SORT, 1_000_000, 4_000_000, ctypes.byref(c), ctypes.byref(s))
    assert w1 >= 4_000_000 * 24
    assert lib.gs_workspace_size(L.GS_STAGE_BACKWARD, 10, 0, ctypes.byref(c), ctypes.byref(s)) >= 480
    assert lib.gs_workspace_size(L.GS_STAGE_SORT, 10, -1, ctypes.byref(c), ctypes.byref(s)) == 0
    assert lib.gs_workspace_size(L.GS_STAGE_SORT, 10, 1 << 31, ctypes.byref(c), ctypes.byref(s)) == 0
    assert lib.gs_workspace_size(99, 10, 10, ctypes.byref(c), ctypes.byref(s)) == 0


FAKE = 0x7F0000000000  # aligned, never dereferenced: every call below fails validation first


def pre(lib, n=4, deg=0, cam=None, st=None, ptrs=None, total=FAKE, ws_bytes=1 << 20):
    c = cam or cam_1080()
    s = st or L.default_settings()
    p = ptrs or [FAKE] * 5
    return lib.gs_preprocess(n, *[ctypes.c_void_p(x) if x else None for x in p], deg, None,
                             ctypes.byref(c), ctypes.byref(s), ctypes.c_void_p(FAKE),
                             ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE),
                             ctypes.c_void_p(total) if total else None,
                             ctypes.c_void_p(FAKE), ws_bytes, None)


def test_preprocess_argument_validation(lib):
    assert pre(lib, n=-1) == L.GS_ERR_INVALID_ARGUMENT
    assert pre(lib, n=1 << 31) == L.GS_ERR_INVALID_ARGUMENT
    assert pre(lib, deg=4) == L.GS_ERR_UNSUPPORTED
    assert pre(lib, deg=-1) == L.GS_ERR_UNSUPPORTED
    assert pre(lib, ptrs=[FAKE, 0, FAKE, FAKE, FAKE]) == L.GS_ERR_INVALID_ARGUMENT
    assert pre(lib, ptrs=[FAKE, FAKE + 4, FAKE, FAKE, FAKE]) == L.GS_ERR_MISALIGNED
    assert pre(lib, total=0) == L.GS_ERR_INVALID_ARGUMENT
    assert pre(lib, st=L.default_settings(sort_mode=2)) == L.GS_ERR_UNSUPPORTED
    assert pre(lib, ws_bytes=0) == L.GS_ERR_WORKSPACE
    assert pre(lib, st=L.default_settings(tile_w=12)) == L.GS_ERR_UNSUPPORTED
    assert pre(lib, st=L.default_settings(radix_bits=9)) == L.GS_ERR_UNSUPPORTED
    assert pre(lib, st=L.default_settings(depth_bits=33)) == L.GS_ERR_INVALID_ARGUMENT
    assert pre(lib, st=L.default_settings(depth_bits=-1)) == L.GS_ERR_INVALID_ARGUMENT
    assert pre(lib, st=L.default_settings(alpha_max=1.0)) == L.GS_ERR_INVALID_ARGUMENT
    assert pre(lib, st=L.default_settings(alpha_min=0.0)) == L.GS_ERR_INVALID_ARGUMENT
    assert pre(lib, st=L.default_settings(eps2d=-1.0)) == L.GS_ERR_INVALID_ARGUMENT
    bad = cam_1080()
    bad.width = 0
    assert pre(lib, cam=bad) == L.GS_ERR_INVALID_ARGUMENT
    bad = cam_1080()
    bad.viewmat[0] = 2.0  # not a rotation
    assert pre(lib, cam=bad) == L.GS_ERR_INVALID_ARGUMENT
    bad = cam_1080()
    bad.fx = float("nan")
    assert pre(lib, cam=bad) == L.GS_ERR_INVALID_ARGUMENT


def test_model_transform_must_be_similarity(lib):
    c, s = cam_1080(), L.default_settings()
    F = ctypes.c_void_p(FAKE)
    shear = (ctypes.c_float * 12)(1, 0.5, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    r = lib.gs_preprocess(4, *[F] * 5, 0, shear, ctypes.byref(c), ctypes.byref(s), F, F, F, F, F,
                          1 << 20, None)
    assert r == L.GS_ERR_INVALID_ARGUMENT
    mirror = (ctypes.c_float * 12)(-1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    r = lib.gs_preprocess(4, *[F] * 5, 0, mirror, ctypes.byref(c), ctypes.byref(s), F, F, F, F, F,
                          1 << 20, None)
    assert r == L.GS_ERR_INVALID_ARGUMENT


def test_sort_argument_validation(lib):
    c, s = cam_1080(), L.default_settings()
    F = ctypes.c_void_p(FAKE)

    def srt(n=4, cap=16, keys=F, values=F, ws=1 << 30, flag=None):
        return lib.gs_sort(n, F, F, F, F, ctypes.byref(c), ctypes.byref(s), cap, keys, values, F,
                           flag, F, ws, None)
    assert srt(cap=-1) == L.GS_ERR_INVALID_ARGUMENT
    assert srt(cap=1 << 30) == L.GS_ERR_INVALID_ARGUMENT
    assert srt(values=None) == L.GS_ERR_INVALID_ARGUMENT
    assert srt(keys=ctypes.c_void_p(FAKE + 8)) == L.GS_ERR_MISALIGNED
    assert srt(flag=ctypes.c_void_p(FAKE + 4)) == L.GS_ERR_MISALIGNED
    assert srt(ws=16) == L.GS_ERR_WORKSPACE

    # gs_sort_checked validates the same way before its host sync
    req = ctypes.c_int64(-7)

    def chk(cap=16, values=F, ws=1 << 30, counts=F):
        return lib.gs_sort_checked(4, F, F, F, counts, ctypes.byref(c), ctypes.byref(s), cap, None,
                                   values, F, None, F, ws, ctypes.byref(req), None)
    assert chk(cap=-1) == L.GS_ERR_INVALID_ARGUMENT
    assert chk(values=None) == L.GS_ERR_INVALID_ARGUMENT
    assert chk(counts=None) == L.GS_ERR_INVALID_ARGUMENT
    assert chk(ws=16) == L.GS_ERR_WORKSPACE
    assert req.value == -7  # untouched when the arguments are rejected

    def sp(n=8, kb=64, kin=F, kout=ctypes.c_void_p(FAKE + 4096), ws=1 << 30):
        return lib.gs_sort_pairs(n, kin, F, kb, kout, ctypes.c_void_p(FAKE + 8192), ctypes.byref(s),
                                 F, ws, None)
    assert sp(kb=0) == L.GS_ERR_INVALID_ARGUMENT
    assert sp(kb=65) == L.GS_ERR_INVALID_ARGUMENT
    assert sp(n=-2) == L.GS_ERR_INVALID_ARGUMENT
    assert sp(kout=F) == L.GS_ERR_INVALID_ARGUMENT  # in == out
    assert sp(ws=0) == L.GS_ERR_WORKSPACE


def test_raster_argument_validation(lib):
    c, s = cam_1080(), L.default_settings()
    F = ctypes.c_void_p(FAKE)
    r = lib.gs_rasterize(F, F, F, ctypes.byref(c), ctypes.byref(s), None, F, F, None, None)
    assert r == L.GS_ERR_INVALID_ARGUMENT
    r = lib.gs_rasterize(F, F, ctypes.c_void_p(FAKE + 2), ctypes.byref(c), ctypes.byref(s), F, F, F,
                         None, None)
    assert r == L.GS_ERR_MISALIGNED
    r = lib.gs_rasterize(F, F, F, ctypes.byref(c), ctypes.byref(s), F, F, F,
                         ctypes.c_void_p(FAKE + 2), None)
    assert r == L.GS_ERR_MISALIGNED
    r = lib.gs_rasterize_backward(4, F, F, F, F, F, 7, None, ctypes.byref(c), ctypes.byref(s),
                                  F, F, F, F, F, F, F, F, F, F, F, 0, F, 1 << 20, None)
    assert r == L.GS_ERR_UNSUPPORTED
    r = lib.gs_rasterize_backward(4, F, F, F, F, F, 3, None, ctypes.byref(c), ctypes.byref(s),
                                  F, F, F, F, F, F, F, F, F, F, F, 0, F, 8, None)
    assert r == L.GS_ERR_WORKSPACE


def test_asset_table_validation(lib):
    c, s = cam_1080(), L.default_settings()
    F = ctypes.c_void_p(FAKE)

    def pa(table, n, n_assets=None):
        arr, keep = L.asset_table(table)
        na = len(table) if n_assets is None else n_assets
        return lib.gs_preprocess_assets(na, arr, n, *[F] * 5, 0, ctypes.byref(c), ctypes.byref(s),
                                        F, F, F, F, F, 1 << 20, None)

    def ba(table, n):
        arr, keep = L.asset_table(table)
        return lib.gs_rasterize_backward_assets(len(table), arr, n, *[F] * 5, 0, ctypes.byref(c),
                                                ctypes.byref(s), F, F, F, F, F, F, F, F, F, F, F,
                                                0, F, 1 << 30, None)
    assert pa([(0, 4, None), (5, 4, None)], 9) == L.GS_ERR_INVALID_ARGUMENT   # gap
    assert pa([(0, 4, None), (4, 4, None)], 9) == L.GS_ERR_INVALID_ARGUMENT   # short of n
    assert pa([(0, 4, None), (4, -1, None)], 3) == L.GS_ERR_INVALID_ARGUMENT  # negative count
    assert pa([(1, 4, None)], 5) == L.GS_ERR_INVALID_ARGUMENT                 # not from 0
    assert pa([(0, 4, None)], 4, n_assets=0) == L.GS_ERR_INVALID_ARGUMENT
    assert pa([(0, 1, None)] + [(1 + k, 1, None) for k in range(64)], 65) == L.GS_ERR_INVALID_ARGUMENT
    shear = [[1, 0.5, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]]
    assert pa([(0, 4, None), (4, 4, shear)], 8) == L.GS_ERR_INVALID_ARGUMENT
    assert ba([(0, 4, None), (5, 4, None)], 9) == L.GS_ERR_INVALID_ARGUMENT
    assert ba([(0, 4, None), (4, 4, shear)], 8) == L.GS_ERR_INVALID_ARGUMENT


def test_multi_view_backward_validation(lib):
    c, s = cam_1080(), L.default_settings()
    F = ctypes.c_void_p(FAKE)
    cams = (L.GsCamera * 2)(c, c)
    ptrs = (ctypes.c_void_p * 2)(FAKE, FAKE)

    def pv(nv=2, table=((0, 4, None),), n=4, cam_arr=cams, p=ptrs):
        arr, keep = L.asset_table(list(table))
        return lib.gs_preprocess_backward_views(nv, cam_arr, p, len(table), arr, n, *[F] * 5, 0,
                                                ctypes.byref(s), *[F] * 5, 0, None)
    assert pv(nv=0) == L.GS_ERR_INVALID_ARGUMENT
    assert pv(table=((0, 3, None),)) == L.GS_ERR_INVALID_ARGUMENT
    bad = (L.GsCamera * 2)(c, c)
    bad[1].width = 0
    assert pv(cam_arr=bad) == L.GS_ERR_INVALID_ARGUMENT
    assert pv(p=(ctypes.c_void_p * 2)(FAKE, FAKE + 4)) == L.GS_ERR_MISALIGNED
    r = lib.gs_rasterize_backward_2d(F, F, F, ctypes.byref(c), ctypes.byref(s), F, F, F, -1, F, None)
    assert r == L.GS_ERR_INVALID_ARGUMENT
    r = lib.gs_rasterize_backward_2d(F, F, F, ctypes.byref(c), ctypes.byref(s), F, F, F, 4,
                                     ctypes.c_void_p(FAKE + 4), None)
    assert r == L.GS_ERR_MISALIGNED


def test_sort_pairs32_validation(lib):
    s = L.default_settings()
    F = ctypes.c_void_p(FAKE)

    def sp(n=8, kb=32, kin=F, vin=None, kout=ctypes.c_void_p(FAKE + 4096),
           vout=ctypes.c_void_p(FAKE + 8192), ws=1 << 30):
        return lib.gs_sort_pairs32(n, kin, vin, kb, kout, vout, ctypes.byref(s), F, ws, None)
    assert sp(kb=0) == L.GS_ERR_INVALID_ARGUMENT
    assert sp(kb=33) == L.GS_ERR_INVALID_ARGUMENT
    assert sp(n=-1) == L.GS_ERR_INVALID_ARGUMENT
    assert sp(kout=F) == L.GS_ERR_INVALID_ARGUMENT            # in == out
    assert sp(vin=ctypes.c_void_p(FAKE + 8192)) == L.GS_ERR_INVALID_ARGUMENT
    assert sp(vout=None) == L.GS_ERR_INVALID_ARGUMENT
    assert sp(vout=ctypes.c_void_p(FAKE + 8196)) == L.GS_ERR_MISALIGNED
    assert sp(ws=0) == L.GS_ERR_WORKSPACE


def test_packed_layout_and_validation(lib):
    assert [lib.gs_packed_sh_stride(d) for d in range(4)] == [4, 12, 28, 48]
    assert lib.gs_packed_sh_stride(4) == -1 and lib.gs_packed_sh_stride(-1) == -1
    c, s = cam_1080(), L.default_settings()
    F = ctypes.c_void_p(FAKE)
    G = lambda k: ctypes.c_void_p(FAKE + 4096 * k)

    def pp(n=8, deg=3, means=F, out=(G(1), G(2), G(3))):
        return lib.gs_prepack(n, means, F, F, F, F, deg, *out, None)
    assert pp(n=-1) == L.GS_ERR_INVALID_ARGUMENT
    assert pp(deg=4) == L.GS_ERR_UNSUPPORTED
    assert pp(means=None) == L.GS_ERR_INVALID_ARGUMENT
    assert pp(out=(G(1), None, G(3))) == L.GS_ERR_INVALID_ARGUMENT
    assert pp(out=(G(1), G(2), ctypes.c_void_p(FAKE + 3 * 4096 + 8))) == L.GS_ERR_MISALIGNED

    tab, _keep = L.asset_table([(0, 8, None)])
    bad_tab, _k2 = L.asset_table([(0, 7, None)])

    def pk(n=8, deg=3, tab=tab, na=1, cov=G(2), ws=1 << 20, sset=s):
        return lib.gs_preprocess_packed(na, tab, n, G(1), cov, G(3), deg, ctypes.byref(c),
                                        ctypes.byref(sset), G(4), G(5), G(6), G(7), G(8), ws, None)
    assert pk(deg=5) == L.GS_ERR_UNSUPPORTED
    assert pk(n=-1) == L.GS_ERR_INVALID_ARGUMENT
    assert pk(tab=bad_tab) == L.GS_ERR_INVALID_ARGUMENT
    assert pk(na=0) == L.GS_ERR_INVALID_ARGUMENT
    assert pk(cov=None) == L.GS_ERR_INVALID_ARGUMENT
    assert pk(cov=ctypes.c_void_p(FAKE + 2 * 4096 + 4)) == L.GS_ERR_MISALIGNED
    assert pk(ws=0) == L.GS_ERR_WORKSPACE
    assert pk(sset=L.default_settings(tile_w=12)) == L.GS_ERR_UNSUPPORTED


def test_mesh_entry_points_validation(lib):
    c, s = cam_1080(), L.default_settings()
    F = ctypes.c_void_p(FAKE)
    G = lambda k: ctypes.c_void_p(FAKE + 4096 * k)
    bad = ctypes.c_void_p(FAKE + 4)

    def rm(md=G(5), mr=G(6), sset=s, img=G(7)):
        return lib.gs_rasterize_mesh(F, G(1), G(2), ctypes.byref(c), ctypes.byref(sset), md, mr,
                                     img, G(8), G(9), None, None)
    assert rm(md=bad) == L.GS_ERR_MISALIGNED
    assert rm(mr=bad) == L.GS_ERR_MISALIGNED
    assert rm(img=None) == L.GS_ERR_INVALID_ARGUMENT
    assert rm(sset=L.default_settings(radix_bits=9)) == L.GS_ERR_UNSUPPORTED

    def rb(mr=G(6), n=8):
        return lib.gs_rasterize_backward_2d_mesh(F, G(1), G(2), ctypes.byref(c), ctypes.byref(s),
                                                 mr, G(3), G(4), G(5), n, G(7), None)
    assert rb(mr=bad) == L.GS_ERR_MISALIGNED
    assert rb(n=-1) == L.GS_ERR_INVALID_ARGUMENT


def test_lbs_validation(lib):
    F = ctypes.c_void_p(FAKE)
    G = lambda k: ctypes.c_void_p(FAKE + 4096 * k)

    def lb(n=8, nj=55, joints=G(5), po=G(6), cv=G(7)):
        return lib.gs_lbs_deform(n, F, G(1), G(2), G(3), nj, joints, po, cv, None)
    assert lb(nj=0) == L.GS_ERR_INVALID_ARGUMENT
    assert lb(nj=257) == L.GS_ERR_INVALID_ARGUMENT
    assert lb(n=-1) == L.GS_ERR_INVALID_ARGUMENT
    assert lb(joints=None) == L.GS_ERR_INVALID_ARGUMENT
    assert lb(po=F) == L.GS_ERR_INVALID_ARGUMENT          # aliases the canonical input
    assert lb(cv=ctypes.c_void_p(FAKE + 7 * 4096 + 2)) == L.GS_ERR_MISALIGNED


def test_raster_order_validation_and_sort_workspace(lib):
    c = cam_1080()
    bad = L.default_settings(raster_order=6)
    assert lib.gs_sort_key_bits(ctypes.byref(c), ctypes.byref(bad)) == -1
    s = L.default_settings()
    # the sort workspace holds 16 tile-class segments of `tiles` entries
    w = lib.gs_workspace_size(L.GS_STAGE_SORT, 1000, 1000, ctypes.byref(c), ctypes.byref(s))
    assert w >= 16 * 120 * 68 * 4


def test_preprocess_noalloc_limits(lib):
    """The allocation-free preprocess states its limit and rejects larger n
    (and negative n) before any HIP call, so no pointers are needed."""
    m = lib.gs_preprocess_noalloc_max_n()
    assert m == (2**20 // 16 - L.MAX_ASSETS) * 256 == 16_760_832
    s = L.default_settings()
    c = L.make_camera(S.pinhole_camera(S.look_at((0, 0, -3)), 64, 64))
    args = [None] * 5 + [0, None, ctypes.byref(c), ctypes.byref(s)] + [None] * 4 + [None]
    assert lib.gs_preprocess_noalloc(m + 1, *args) == L.GS_ERR_WORKSPACE
    assert lib.gs_preprocess_noalloc(-1, *args) == L.GS_ERR_INVALID_ARGUMENT
    assert lib.gs_preprocess_noalloc(2**31, *args) == L.GS_ERR_INVALID_ARGUMENT


def batch_desc(n_views=3, n=100, tables=None, means=FAKE, cams=None, targets=None):
    cams = cams or [cam_1080() for _ in range(n_views)]
    arr_c = (L.GsCamera * max(1, len(cams)))(*cams)
    tab, keep = L.asset_table(tables or [(0, n, None)])
    d = L.GsBatchDesc()
    d.n_views = n_views
    d.cams = ctypes.cast(arr_c, ctypes.c_void_p)
    d.n_assets = len(tables or [0])
    d.assets = ctypes.cast(tab, ctypes.c_void_p)
    d.n = n
    d.means = means
    d.log_scales = d.quats = d.opacity_logits = d.sh = FAKE
    d.sh_degree = 0
    d.targets = targets
    return d, (arr_c, tab, keep)


def test_batch_api_validation(lib):
    """gs_batch_create makes a batch without any HIP call; the batch calls
    reject bad arguments and calls out of order before touching the device."""
    s = L.default_settings()
    h = ctypes.c_void_p()

    def create(d, st=s):
        return lib.gs_batch_create(ctypes.byref(d), ctypes.byref(st), ctypes.byref(h))
    assert lib.gs_batch_create(None, ctypes.byref(s), ctypes.byref(h)) == L.GS_ERR_INVALID_ARGUMENT
    d, keep = batch_desc(n_views=0)
    assert create(d) == L.GS_ERR_INVALID_ARGUMENT
    d, keep = batch_desc(n_views=257, cams=[cam_1080()] * 257)
    assert create(d) == L.GS_ERR_INVALID_ARGUMENT
    d, keep = batch_desc(means=FAKE + 4)
    assert create(d) == L.GS_ERR_MISALIGNED
    d, keep = batch_desc(tables=[(0, 40, None), (50, 50, None)])       # a gap
    assert create(d) == L.GS_ERR_INVALID_ARGUMENT
    d, keep = batch_desc(targets=FAKE + 8)
    assert create(d) == L.GS_ERR_MISALIGNED
    d, keep = batch_desc()
    assert create(d, L.default_settings(tile_w=7, tile_h=7)) == L.GS_ERR_UNSUPPORTED
    tall = L.make_camera(S.pinhole_camera(S.look_at((0, 0, -8)), 512, 4096))
    d, keep = batch_desc(n_views=200, cams=[tall] * 200)              # 51200 tile rows x 2 > 65535
    assert create(d, L.default_settings(tile_w=16, tile_h=8)) == L.GS_ERR_UNSUPPORTED

    # a valid batch of three 1080p views
    d, keep = batch_desc()
    assert create(d) == L.GS_OK and h.value
    b = h
    try:
        assert lib.gs_batch_pixels(b) == 3 * 1920 * 1080
        assert [lib.gs_batch_pixel_offset(b, v) for v in (0, 1, 2, 3, -1)] == \
            [0, 1920 * 1080, 2 * 1920 * 1080, -1, -1]
        assert lib.gs_batch_capacity(b) == -1                     # not planned
        assert lib.gs_batch_workspace_size(b, 0) > 0
        assert lib.gs_batch_workspace_size(b, -1) == 0
        assert lib.gs_batch_workspace_size(b, 1 << 30) == 0
        F = ctypes.c_void_p(FAKE)
        cap = ctypes.c_int64(0)
        need = lib.gs_batch_workspace_size(b, 0)
        plan = lambda hr=1.1, ws=F, nb=need, c=ctypes.byref(cap): lib.gs_batch_plan(
            b, ctypes.c_float(hr), ws, nb, c, None)
        assert plan(hr=0.5) == L.GS_ERR_INVALID_ARGUMENT
        assert plan(hr=5.0) == L.GS_ERR_INVALID_ARGUMENT
        assert plan(hr=float("nan")) == L.GS_ERR_INVALID_ARGUMENT
        assert plan(c=None) == L.GS_ERR_INVALID_ARGUMENT
        assert plan(nb=need - 1) == L.GS_ERR_WORKSPACE
        assert plan(ws=ctypes.c_void_p(FAKE + 4)) == L.GS_ERR_MISALIGNED
        outs = [F] * 6 + [None]
        # run and capture need a plan first; launch needs a capture
        assert lib.gs_batch_run(b, F, 1 << 40, *outs, None) == L.GS_ERR_INVALID_ARGUMENT
        assert lib.gs_batch_capture(b, F, 1 << 40, *outs, F) == L.GS_ERR_INVALID_ARGUMENT
        assert lib.gs_batch_launch(b, None) == L.GS_ERR_INVALID_ARGUMENT
        assert lib.gs_batch_launch(None, None) == L.GS_ERR_INVALID_ARGUMENT
        assert lib.gs_batch_plan(None, ctypes.c_float(1.1), F, need, ctypes.byref(cap), None) == \
            L.GS_ERR_INVALID_ARGUMENT
    finally:
        lib.gs_batch_destroy(b)
    lib.gs_batch_destroy(None)
    assert lib.gs_batch_pixels(None) == -1 and lib.gs_batch_workspace_size(None, 0) == 0

    # gs_autotune rejects a malformed search space or repetition count
    d, keep = batch_desc()
    sp = L.GsAutotuneSpace()
    best, ms, nev = L.GsSettings(), ctypes.c_float(0), ctypes.c_int32(0)
    F = ctypes.c_void_p(FAKE)

    def tune(space=sp, reps=2):
        return lib.gs_autotune(ctypes.byref(d), ctypes.byref(s), ctypes.byref(space), reps,
                               ctypes.c_float(1.1), F, 1 << 40, *([F] * 6), None,
                               ctypes.byref(best), ctypes.byref(ms), ctypes.byref(nev), None)
    assert tune(reps=0) == L.GS_ERR_INVALID_ARGUMENT
    assert tune(reps=101) == L.GS_ERR_INVALID_ARGUMENT
    bad = L.GsAutotuneSpace()
    bad.n_tiles = 17
    assert tune(space=bad) == L.GS_ERR_INVALID_ARGUMENT
    bad = L.GsAutotuneSpace()
    bad.n_modes = 3
    assert tune(space=bad) == L.GS_ERR_INVALID_ARGUMENT
    bad = L.GsAutotuneSpace()
    bad.n_orders = 7
    assert tune(space=bad) == L.GS_ERR_INVALID_ARGUMENT
