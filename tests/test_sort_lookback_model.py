"""CPU model of the onesweep sort's look-back buffer over the real pass plan.

In sort mode 1 every radix pass publishes, per partition and digit, a
look-back word that later partitions of the same pass read (decoupled
look-back).  The words of consecutive passes alternate between two halves
of one buffer; gs_sort clears both halves first, and each pass clears the
next pass's half for every partition of its grid.  A pass that read a word
left over from an earlier pass would take a wrong prefix and scatter out of
its range, so the invariant is: when a pass starts, every word it reads is
clear.

The plan comes from the library (gs_sort_plan, host-only, the same planner
gs_sort uses); the counts the device reads (visible Gaussians, instances)
are swept over their whole range, including the cases that once broke the
invariant: later depth passes that sort only the visible Gaussians, then
tile passes with more partitions.
"""
import itertools

import pytest

from paper_2512_08478_amd import _lib as L
from paper_2512_08478_amd import scenes as S


def simulate(plan, words, n, n_vis, inst, clear_all_grid=True):
    """Replay the buffer protocol; returns the first violation, or None.
    With clear_all_grid=False a pass clears only the partitions that hold
    keys (the rule before the fix), for the test of the model itself."""
    half = words // 2
    dirty = [bytearray(half), bytearray(half)]   # sort_init cleared both halves
    for p in plan:
        nb = 1 << p["digit_bits"]
        part = p["partition_keys"]
        keys = {L.GS_PASS_KEYS_ALL: n, L.GS_PASS_KEYS_VISIBLE: n_vis,
                L.GS_PASS_KEYS_INSTANCES: inst}[p["keys"]]
        active = -(-keys // part)
        assert active <= p["grid_partitions"]
        assert p["grid_partitions"] * nb <= half, "look-back words past the buffer"
        h = p["index"] & 1
        read = active * nb
        if any(dirty[h][:read]):
            return (p["index"], dirty[h][:read].index(1))
        dirty[h][:read] = b"\x01" * read            # published by this pass
        cleared = (p["grid_partitions"] if clear_all_grid else active) * nb
        dirty[h ^ 1][:cleared] = bytes(cleared)     # the next half, cleared
    return None


CAMS = {"tiny 256x256": S.pinhole_camera(S.look_at((0, 0, -3)), 256, 256),
        "1080p": S.pinhole_camera(S.look_at((0, 0, -8)), 1920, 1080)}


def cases():
    for (cname, cam), bits, tile, db in itertools.product(
            CAMS.items(), (6, 7, 8), ((8, 8), (32, 16)), (0, 25)):
        yield cname, cam, bits, tile, db


@pytest.mark.parametrize("cname,cam,bits,tile,db", list(cases()))
def test_every_word_read_is_clear(cname, cam, bits, tile, db):
    s = L.default_settings(tile_w=tile[0], tile_h=tile[1], radix_bits=bits, sort_mode=1,
                           depth_bits=db)
    for n, capacity in ((4096, 20_000), (1_000_000, 3_500_000), (6_000_000, 9_000_000),
                        (50_000, 4_000_000), (3_000_000, 100_000)):
        plan, words = L.sort_plan(n, capacity, cam, s)
        assert words > 0 and len(plan) >= 2
        assert [p["index"] for p in plan] == list(range(len(plan)))
        for n_vis in sorted({0, 1, n // 7, n // 2, n}):
            for inst in sorted({0, 1, capacity // 3, capacity}):
                bad = simulate(plan, words, n, n_vis, inst)
                assert bad is None, (cname, bits, tile, db, n, capacity, n_vis, inst, bad)


def test_model_catches_the_old_clearing_rule():
    """Clearing only the partitions that hold keys leaves the first depth
    pass's words behind for the tile passes when later depth passes sort
    fewer keys: the model must see that."""
    s = L.default_settings(tile_w=8, tile_h=8, radix_bits=8, sort_mode=1)
    plan, words = L.sort_plan(6_000_000, 9_000_000, CAMS["1080p"], s)
    assert simulate(plan, words, 6_000_000, 3_500_000, 9_000_000, clear_all_grid=True) is None
    assert simulate(plan, words, 6_000_000, 3_500_000, 9_000_000, clear_all_grid=False) is not None


def test_plan_matches_key_bits():
    """Mode 0 plans the same digits (no look-back words); the tile passes
    cover the key bits above the 32 depth bits."""
    import ctypes
    lib = L.load()
    for mode in (0, 1):
        s = L.default_settings(tile_w=16, tile_h=16, radix_bits=7, sort_mode=mode)
        cam = CAMS["1080p"]
        plan, words = L.sort_plan(1000, 5000, cam, s)
        kb = lib.gs_sort_key_bits(ctypes.byref(L.make_camera(cam)), ctypes.byref(s))
        depth = [p for p in plan if p["keys"] != L.GS_PASS_KEYS_INSTANCES]
        tile = [p for p in plan if p["keys"] == L.GS_PASS_KEYS_INSTANCES]
        assert sum(p["digit_bits"] for p in depth) >= 32
        assert len(tile) == -(-(kb - 32) // 7)
        assert (words > 0) == (mode == 1)
