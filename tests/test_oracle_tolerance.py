"""Pins of the oracle's tolerance machinery and of its tiled mode.

* ``pair_max_weight`` (the largest weight of a Gaussian over a tile's pixel
  centres, which certifies extra GPU (Gaussian, tile) pairs as harmless)
  against the closed form for an isotropic footprint: o exp(-r^2 / 2 s^2)
  at the pixel centre nearest the mean, within the tile and the image.
* Every kind of near decision (Section 3.2's discrete choices read as in
  the tolerance protocol: skip at tau, stop at t_eps, depth order, culls
  near a threshold, the mesh depth test) sets its flag or margin, and the
  jump the oracle reports equals the closed-form change of the pixel when
  that decision is taken the other way.
* The tiled oracle equals the brute-force definition (Eq. 3 over every
  Gaussian) exactly: on the tiny scene, with a mesh, and on a 64x64 crop of
  the 1M frame.
"""
import math

import numpy as np
import pytest

from paper_2512_08478_amd import scenes as S

TAU = 1.0 / 255.0
C0 = 1.0 / (2.0 * math.sqrt(math.pi))


def one_scene(points, log_scale, logit, dc):
    n = len(points)
    means = np.asarray(points, np.float32).reshape(n, 3)
    ls = np.broadcast_to(np.asarray(log_scale, np.float32), (n, 3)).copy()
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1))
    lg = np.broadcast_to(np.asarray(logit, np.float32), (n,)).copy()
    sh = np.zeros((n, 1, 3), np.float32)
    sh[:, 0, :] = np.asarray(dc, np.float32)
    return S.Scene(means, ls, q, lg, sh, 0)


def iso_camera(W, H, f, cx, cy):
    """Identity view, so a Gaussian on the optical axis projects to (cx, cy)
    with S = ((f sigma / d)^2 + eps) I (closed form P1)."""
    return S.Camera(np.eye(4, dtype=np.float32), f, f, cx, cy, W, H, 0.2)


def sigmoid32(logit):
    return 1.0 / (1.0 + math.exp(-float(np.float32(logit))))


def rgb_of(dc):
    return np.maximum(0.0, np.asarray(dc, np.float32).astype(np.float64) * C0 + 0.5)


def s2_of(log_scale, f, d, eps=0.3):
    return (f * float(np.exp(np.float64(np.float32(log_scale)))) / d) ** 2 + eps


# ---------------------------------------------------------------- pair_max_weight

@pytest.mark.parametrize("centre", [(21.3, 13.7), (49.8, 29.6), (-3.2, 12.4), (30.0, 8.0),
                                    (52.3, 33.1)])
def test_pair_max_weight_closed_form(orc, centre):
    # 50x30 image in 16x8 tiles: the last tile column holds 2 pixel columns
    # and the last tile row 6 rows; the mean sits inside a tile, on an image
    # corner, left of the image, on a tile corner, and beyond the last
    # (ragged) tile's right and bottom edges.
    W, H, tw, th, f, d = 50, 30, 16, 8, 40.0, 2.0
    ls, logit = math.log(0.05), 1.0
    cx, cy = centre
    cam = iso_camera(W, H, f, cx, cy)
    r = orc.preprocess(one_scene([[0, 0, d]], ls, logit, [0, 0, 0]), cam)
    tiles_x, tiles_y = -(-W // tw), -(-H // th)
    t = np.arange(tiles_x * tiles_y)
    got = orc.pair_max_weight(r, cam, np.zeros_like(t), t, dict(tile_w=tw, tile_h=th))
    o, s2 = sigmoid32(logit), s2_of(ls, f, d)
    for k in t:
        tx, ty = k % tiles_x, k // tiles_x
        x_lo, x_hi = tx * tw, min(W, (tx + 1) * tw) - 1
        y_lo, y_hi = ty * th, min(H, (ty + 1) * th) - 1
        # nearest pixel centre: the centre nearest the mean, clamped to the tile
        nx = min(max(math.floor(cx) + 0.5, x_lo + 0.5), x_hi + 0.5)
        ny = min(max(math.floor(cy) + 0.5, y_lo + 0.5), y_hi + 0.5)
        expect = o * math.exp(-((nx - cx) ** 2 + (ny - cy) ** 2) / (2 * s2))
        assert got[k] == pytest.approx(expect, rel=1e-12, abs=1e-300), (centre, tx, ty)


# ---------------------------------------------------------------- near decisions

def test_near_tie_flag_and_swap_jump(orc):
    # Two Gaussians on the axis at depth ~3.5 (float32 spacing 2^-22), where
    # a near tie is a difference up to 2^-22 (3.5 + 3.5) = 7 spacings.  Index
    # 0 is the deeper one, so depth order and index order disagree.  At the
    # pixel holding their mean (Q = 0, alpha = o) the order is a near
    # decision: swapping two blends changes C by alpha_a alpha_b (c_a - c_b)
    # and leaves T unchanged.  4 spacings apart they tie, 12 apart they do not.
    cam = iso_camera(16, 16, 30.0, 8.5, 8.5)
    z = np.float32(3.5)
    ls, logits = math.log(0.05), [0.3, 1.2]
    dcs = [[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]]
    for steps, tie in ((4, True), (12, False)):
        far = z
        for _ in range(steps):
            far = np.nextafter(far, np.float32(4.0))
        sc = one_scene([[0, 0, far], [0, 0, z]], ls, logits, dcs)
        r = orc.preprocess(sc, cam)
        out = orc.render_pixels(r, cam, [[8, 8], [0, 0]])
        a = [min(0.99, sigmoid32(l)) for l in logits]
        c = [rgb_of(dc) for dc in dcs]
        assert bool(out["flags"][0] & 1) == tie
        expect = a[0] * a[1] * np.abs(c[0] - c[1]).max() if tie else 0.0
        assert out["jump"][0] == pytest.approx(expect, rel=1e-12, abs=1e-15)
        assert out["flags"][1] == 0 and out["jump"][1] == 0.0


@pytest.mark.parametrize("tie", [True, False])
def test_near_tie_across_the_stop(orc, tie):
    # Three coincident Gaussians (alpha = 0.97) take T below t_eps, so the
    # walk stops on the third; Gaussian 0 lies one float32 step deeper (a
    # near tie; 100 steps apart it is not) and would blend next.  A float32
    # order may take it first: walk G1, G2, B, G3 instead of G1, G2, G3.
    # With T2 = (1 - a)^2: dC = T2 a_B (c_B - a c), dA = T2 (1 - a) a_B.
    z = np.float32(2.0)
    zb = z
    for _ in range(1 if tie else 100):
        zb = np.nextafter(zb, np.float32(3.0))
    la, lb = math.log(0.97 / 0.03), 0.8
    dcs = [[0.1, 0.9, 0.3], [1.2, 0.0, 0.5]]
    sc = one_scene([[0, 0, zb], [0, 0, z], [0, 0, z], [0, 0, z]], math.log(0.05),
                   [lb, la, la, la], [dcs[1], dcs[0], dcs[0], dcs[0]])
    cam = iso_camera(16, 16, 30.0, 8.5, 8.5)
    out = orc.render_pixels(orc.preprocess(sc, cam), cam, [[8, 8]])
    a, ab = sigmoid32(la), sigmoid32(lb)
    assert (1 - a) ** 2 >= 1e-4 > (1 - a) ** 3
    assert out["n_blend"][0] == 3
    # the coincident stack ties with itself (swaps of equal Gaussians: no jump)
    assert out["flags"][0] & 1
    T2 = (1 - a) ** 2
    c, cb = rgb_of(dcs[0]), rgb_of(dcs[1])
    expect = max(np.abs(T2 * ab * (cb - a * c)).max(), T2 * (1 - a) * ab) if tie else 0.0
    assert out["jump"][0] == pytest.approx(expect, rel=1e-9, abs=1e-15)


@pytest.mark.parametrize("rel,ambiguous", [(5e-6, True), (5e-5, False)])
def test_ambiguous_opacity_cull(orc, rel, ambiguous):
    # opacity just below tau: culled; within a relative 1e-5 it is ambiguous,
    # and at the pixel holding its mean (weight = o) keeping it would blend
    # alpha = o: the jump is o max(1, max rgb) (alone, black background)
    logit = np.float32(math.log(TAU * (1 - rel) / (1 - TAU * (1 - rel))))
    o = sigmoid32(logit)
    assert TAU * (1 - 2 * rel) < o < TAU
    dc = [0.2, 0.5, 2.9]
    sc = one_scene([[0, 0, 2.0]], math.log(0.05), logit, dc)
    cam = iso_camera(16, 16, 30.0, 8.5, 8.5)
    r = orc.preprocess(sc, cam)
    assert r.i[0, orc.I_CULL] == orc.C_OPACITY
    assert r.i[0, orc.I_AMBIG] == int(ambiguous)
    out = orc.render_pixels(r, cam, [[8, 8], [3, 3]])
    np.testing.assert_array_equal(out["rgba"], 0.0)
    assert bool(out["flags"][0] & 2) == ambiguous
    expect = o * max(1.0, rgb_of(dc).max()) if ambiguous else 0.0
    assert out["jump"][0] == pytest.approx(expect, rel=1e-12, abs=1e-15)
    assert out["flags"][1] == 0 and out["jump"][1] == 0.0


@pytest.mark.parametrize("z,ambiguous", [(0.2 * (1 - 5e-6), True), (0.19, False)])
def test_ambiguous_near_plane_cull(orc, z, ambiguous):
    zf = np.float32(z)
    assert zf <= 0.2
    logit, dc = 1.0, [0.9, 0.1, 0.4]
    sc = one_scene([[0, 0, zf]], math.log(0.002), logit, dc)
    cam = iso_camera(16, 16, 30.0, 8.5, 8.5)
    r = orc.preprocess(sc, cam)
    assert r.i[0, orc.I_CULL] == orc.C_NEAR
    assert r.i[0, orc.I_AMBIG] == int(ambiguous)
    out = orc.render_pixels(r, cam, [[8, 8]])
    assert bool(out["flags"][0] & 2) == ambiguous
    o = sigmoid32(logit)
    expect = o * max(1.0, rgb_of(dc).max()) if ambiguous else 0.0
    assert out["jump"][0] == pytest.approx(expect, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("ambiguous", [True, False])
def test_ambiguous_off_image_cull(orc, ambiguous):
    # An isotropic footprint whose support {o exp(-r^2/2s^2) >= tau} ends just
    # left of the first pixel centre column (x = 0.5): culled as off-image.
    # When the centre (0.5, 8.5) sees a weight within a relative 1e-5 of tau
    # the cull is ambiguous; keeping the Gaussian would blend that weight.
    f, d, ls, logit = 30.0, 2.0, math.log(0.05), 1.0
    o, s2 = sigmoid32(logit), s2_of(ls, f, d)
    r_tau = math.sqrt(2 * s2 * math.log(o / TAU))          # weight = tau at this distance
    rel = 5e-6 if ambiguous else 5e-5
    r_px = math.sqrt(2 * s2 * math.log(o / (TAU * (1 - rel))))
    cx = 0.5 - r_px
    assert r_px > r_tau
    dc = [0.3, 0.3, 0.3]
    cam = iso_camera(16, 16, f, cx, 8.5)
    r = orc.preprocess(one_scene([[0, 0, d]], ls, logit, dc), cam)
    assert r.i[0, orc.I_CULL] == orc.C_OFFIMAGE
    assert r.i[0, orc.I_AMBIG] == int(ambiguous)
    out = orc.render_pixels(r, cam, [[0, 8], [0, 2]])
    assert bool(out["flags"][0] & 2) == ambiguous
    g = o * math.exp(-(0.5 - cx) ** 2 / (2 * s2))
    expect = g * max(1.0, rgb_of(dc).max()) if ambiguous else 0.0
    assert out["jump"][0] == pytest.approx(expect, rel=1e-9, abs=1e-15)
    assert out["flags"][1] == 0


def test_near_skip_jump(orc):
    # one Gaussian whose weight at the centre (0.5, 8.5) is tau (1 + 5e-6):
    # blended, with a margin of 5e-6; skipping it instead removes g rgb and g
    f, d, ls, logit = 30.0, 2.0, math.log(0.05), 0.7
    o, s2 = sigmoid32(logit), s2_of(ls, f, d)
    cx = 0.5 + math.sqrt(2 * s2 * math.log(o / (TAU * (1 + 5e-6))))
    dc = [1.5, 0.2, 0.7]
    cam = iso_camera(16, 16, f, cx, 8.5)
    out = orc.render_pixels(orc.preprocess(one_scene([[0, 0, d]], ls, logit, dc), cam), cam,
                            [[0, 8]])
    g = o * math.exp(-(0.5 - cx) ** 2 / (2 * s2))
    assert out["n_blend"][0] == 1
    assert out["margin"][0] == pytest.approx(5e-6, rel=1e-6)
    assert out["jump"][0] == pytest.approx(g * max(1.0, rgb_of(dc).max()), rel=1e-9)


def test_near_stop_jump(orc):
    # coincident Gaussians at the pixel holding their mean (alpha = o): after
    # 3 blends T_3 = (1 - o)^3 = t_eps (1 - 5e-6), so the walk stops with a
    # margin of ~5e-6; continuing would blend one more: the jump is
    # T_3 o max(1, max rgb)
    o_t = 1.0 - (1e-4 * (1 - 5e-6)) ** (1.0 / 3.0)
    logit = np.float32(math.log(o_t / (1 - o_t)))
    o = sigmoid32(logit)
    T3 = (1 - o) ** 3
    assert 1e-4 * (1 - 1e-5) < T3 < 1e-4
    dc = [0.4, -0.2, 0.8]
    cam = iso_camera(16, 16, 20.0, 8.5, 8.5)
    sc = one_scene([[0, 0, 2.0]] * 6, math.log(0.1), logit, dc)
    out = orc.render_pixels(orc.preprocess(sc, cam), cam, [[8, 8]])
    assert out["n_blend"][0] == 3
    assert out["margin"][0] < 1e-5
    assert out["jump"][0] == pytest.approx(T3 * o * max(1.0, rgb_of(dc).max()), rel=1e-9)


def test_near_mesh_depth_jump(orc):
    # a wall exactly at the depth of a lone Gaussian keeps it (only greater
    # depths are hidden); hiding it instead shows the mesh colour m: the jump
    # is max(alpha max|c - m|, alpha)
    logit, dc, m = 0.4, [0.9, 0.1, 0.5], np.array([0.2, 0.7, 0.1])
    cam = iso_camera(16, 16, 30.0, 8.5, 8.5)
    r = orc.preprocess(one_scene([[0, 0, 2.0]], math.log(0.05), logit, dc), cam)
    mesh = dict(depth=np.full((16, 16), 2.0, np.float32), rgb=np.tile(m, (16, 16, 1)))
    out = orc.render_pixels(r, cam, [[8, 8]], mesh=mesh)
    a = sigmoid32(logit)
    assert out["flags"][0] & 4
    assert out["jump"][0] == pytest.approx(max(a * np.abs(rgb_of(dc) - m).max(), a), rel=1e-12)


# ---------------------------------------------------------------- tiled == brute force

def assert_same(a, b):
    for k in ("rgba", "T", "n_blend", "flags", "jump"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    low = (a["margin"] < 1e-3) | (b["margin"] < 1e-3)
    np.testing.assert_array_equal(a["margin"][low], b["margin"][low])
    assert np.all(b["margin"][~low] >= 1e-3)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_tiled_equals_brute_force_tiny(orc, tile):
    sc, cam = S.tiny_scene()
    st = dict(tile_w=tile[0], tile_h=tile[1])
    r = orc.preprocess(sc, cam, st)
    a = orc.render_image(r, cam, st)
    b = orc.render_image(r, cam, st, tiled=True)
    assert_same(a, b)
    assert int(a["n_blend"].sum()) > 100_000


def test_tiled_equals_brute_force_with_mesh(orc):
    sc, cam = S.tiny_scene()
    fwd = np.asarray(cam.viewmat, np.float64)[2, :3]
    mesh = S.plane_mesh(cam, fwd + np.array([0.1, 0.3, 0.0]), 0.0, seed=3, occupancy=0.6)
    r = orc.preprocess(sc, cam)
    a = orc.render_image(r, cam, mesh=mesh)
    b = orc.render_image(r, cam, mesh=mesh, tiled=True)
    assert_same(a, b)


def test_tiled_equals_brute_force_1m_crop(orc):
    # the 64x64 pixels at the centre of the 1M frame (its densest region)
    sc, cam = S.medium_scene()
    r = orc.preprocess(sc, cam)
    ys, xs = np.mgrid[508:572, 928:992]
    pix = np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)
    a = orc.render_pixels(r, cam, pix)
    b = orc.render_pixels(r, cam, pix, tiled=True)
    assert_same(a, b)
    assert a["n_blend"].mean() > 20
