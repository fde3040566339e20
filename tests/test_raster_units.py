"""The compositing kernels' split of a frame into workgroups (CPU).

gs_raster_grid / gs_raster_unit run on the host the same function the
compositing kernels run to pick their work.  For every tile shape,
compositing order (spatial runs or heavy tiles first, whole quadrants or
2 or 4 row bands) and both directions, every (tile, quadrant, band) of the
frame must be taken by exactly one workgroup and the padding workgroups by
none: a unit taken by no workgroup would leave pixels unwritten, one taken
twice would composite (or, in the backward, accumulate gradients) twice.
"""
import ctypes
import os

import numpy as np
import pytest

from paper_2512_08478_amd import _lib as L
from paper_2512_08478_amd import scenes as S

SHAPES = ((8, 8), (16, 8), (16, 16), (32, 8), (32, 16), (32, 32), (64, 16), (64, 32))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2512_08478_amd import build
        build.build()
    return L.load()


def units(lib, cam, settings, forward, order):
    c = L.make_camera(cam)
    grid = lib.gs_raster_grid(ctypes.byref(c), ctypes.byref(settings), int(forward))
    assert grid > 0
    out = (ctypes.c_int32 * 3)()
    op = order.ctypes.data_as(ctypes.c_void_p) if order is not None else None
    taken, padding = [], 0
    for b in range(grid):
        r = lib.gs_raster_unit(ctypes.byref(c), ctypes.byref(settings), int(forward), op, b, out)
        assert r in (0, 1), r
        if r:
            taken.append((out[0], out[1], out[2]))
        else:
            padding += 1
    return grid, taken, padding


def check_split(lib, cam, tw, th, order_code, forward, seed=0):
    s = L.default_settings(tile_w=tw, tile_h=th, raster_order=order_code)
    tiles = (-(-cam.width // tw)) * (-(-cam.height // th))
    nq = (tw // 8) * (th // 8)
    bands = 1 << (order_code >> 1) if forward else 1
    order = None
    if order_code & 1:  # heavy-first: any permutation of the tiles
        order = np.random.default_rng(seed).permutation(tiles).astype(np.uint32)
    grid, taken, padding = units(lib, cam, s, forward, order)
    want = {(t, q, b) for t in range(tiles) for q in range(nq) for b in range(bands)}
    assert len(taken) == len(want), (len(taken), len(want))
    assert set(taken) == want
    assert padding == grid - len(want)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("order_code", range(6))
@pytest.mark.parametrize("forward", [True, False])
def test_every_unit_taken_once_ragged(lib, shape, order_code, forward):
    # 250 x 190: ragged edge tiles in both directions
    cam = S.pinhole_camera(S.look_at((0.3, -0.2, -3.0)), 250, 190, 60.0)
    check_split(lib, cam, *shape, order_code, forward, seed=order_code)


@pytest.mark.parametrize("shape,order_code", [((32, 16), 1), ((8, 8), 5), ((8, 8), 3),
                                              ((16, 8), 0)])
def test_every_unit_taken_once_1080p(lib, shape, order_code):
    """The benchmark's launch configurations (1M: 32x16, heavy first; 6M:
    8x8 in 4 bands, heavy first) and two others, at 1920 x 1080."""
    cam = S.orbit_camera(0, 8, 8.0, 1920, 1080)
    check_split(lib, cam, *shape, order_code, True, seed=7)


def test_heavy_first_units_follow_the_order(lib):
    """With heavy tiles first, the first workgroup of each XCD (workgroups
    0-7) takes the first quadrant of ranks 0, 16, 32, ... of the order."""
    cam = S.pinhole_camera(S.look_at((0.0, 0.0, -3.0)), 256, 256, 60.0)
    s = L.default_settings(tile_w=16, tile_h=16, raster_order=1)
    order = np.random.default_rng(3).permutation(256).astype(np.uint32)
    c = L.make_camera(cam)
    out = (ctypes.c_int32 * 3)()
    for b in range(8):
        r = lib.gs_raster_unit(ctypes.byref(c), ctypes.byref(s), 1,
                               order.ctypes.data_as(ctypes.c_void_p), b, out)
        assert r == 1 and (out[0], out[1], out[2]) == (int(order[16 * b]), 0, 0)


def test_raster_unit_arguments(lib):
    cam = L.make_camera(S.pinhole_camera(S.look_at((0.0, 0.0, -3.0)), 64, 64, 60.0))
    s = L.default_settings(tile_w=16, tile_h=16, raster_order=1)
    out = (ctypes.c_int32 * 3)()
    grid = lib.gs_raster_grid(ctypes.byref(cam), ctypes.byref(s), 1)
    assert lib.gs_raster_unit(ctypes.byref(cam), ctypes.byref(s), 1, None, 0, out) == \
        L.GS_ERR_INVALID_ARGUMENT                      # heavy-first needs the order
    order = np.arange(16, dtype=np.uint32)
    op = order.ctypes.data_as(ctypes.c_void_p)
    assert lib.gs_raster_unit(ctypes.byref(cam), ctypes.byref(s), 1, op, grid, out) == \
        L.GS_ERR_INVALID_ARGUMENT                      # past the grid
    assert lib.gs_raster_unit(ctypes.byref(cam), ctypes.byref(s), 1, op, -1, out) == \
        L.GS_ERR_INVALID_ARGUMENT
    bad = L.default_settings(raster_order=6)
    assert lib.gs_raster_grid(ctypes.byref(cam), ctypes.byref(bad), 1) == -1
