"""Helpers for the GPU tests: run the HIP path through the C ABI and read
its outputs back as numpy."""
import numpy as np
import torch

SPLAT_DTYPE = np.dtype([("mx", "<f4"), ("my", "<f4"), ("qa", "<f4"), ("qb", "<f4"), ("qc", "<f4"),
                        ("op", "<f4"), ("r", "<f4"), ("g", "<f4"), ("b", "<f4"), ("depth", "<f4"),
                        ("px0", "<u2"), ("py0", "<u2"), ("px1", "<u2"), ("py1", "<u2")])
assert SPLAT_DTYPE.itemsize == 48
_TILED = np.dtype([(nm, "<f8" if nm in ("mx", "my") else t) for nm, t in SPLAT_DTYPE.descr] +
                  [("tx0", "<i8"), ("ty0", "<i8"), ("tx1", "<i8"), ("ty1", "<i8")])


def splats_np(splats_u8, n, tile=(16, 16)):
    """The records as a structured array -- with the 2-D mean made absolute
    (the record stores it relative to the pixel bbox corner (px0, py0)) in
    float64 -- plus the tile rect (tx0, ty0, tx1, ty1) of each record's pixel
    bbox for tiles of `tile` pixels (culled records keep an empty rect,
    tx1 < tx0)."""
    raw = splats_u8[: n * 48].cpu().numpy().view(SPLAT_DTYPE)
    out = np.zeros(raw.shape, _TILED)
    for f in SPLAT_DTYPE.names:
        out[f] = raw[f]
    out["mx"] = raw["mx"].astype(np.float64) + raw["px0"]
    out["my"] = raw["my"].astype(np.float64) + raw["py0"]
    vis = raw["px1"] >= raw["px0"]
    tw, th = tile
    out["tx0"] = np.where(vis, raw["px0"] // tw, 1)
    out["tx1"] = np.where(vis, raw["px1"] // tw, 0)
    out["ty0"] = np.where(vis, raw["py0"] // th, 0)
    out["ty1"] = np.where(vis, raw["py1"] // th, 0)
    return out


def conic_from_whitened(rec):
    """(A, B, C) of S^-1 from the whitened record (qa, qb, qc)."""
    qa, qb, qc = rec["qa"].astype(np.float64), rec["qb"].astype(np.float64), rec["qc"].astype(np.float64)
    return np.stack([qa, -qa * qb, qa * qb * qb + qc], 1)


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def u64(t):
    return t.cpu().numpy().view(np.uint64)


def print_case(msg):
    print(f"[gpu case] {msg}", flush=True)


def image_check(gpu_rgba, ref, tol=1e-4, max_flagged=0.08, max_loosened=0.01, T=None):
    """Compare a GPU image (P,4) to oracle outputs at the same pixels, by the
    tolerance protocol.

    Unflagged pixels (every decision margin >= 1e-5, no depth near-tie, no
    ambiguous cull, no near mesh test) must be within `tol` on RGB and A.
    A flagged pixel must be within `tol` plus the jump its near decisions
    straddle (the oracle re-walks each of them taken the other way).  At most
    `max_flagged` of the pixels may be flagged, and at most `max_loosened`
    may have a jump above `tol`.  With `T` (the GPU's final transmittance at
    the same pixels) the same bounds hold for T.
    Returns (max err unflagged, n flagged, n loosened)."""
    err = np.abs(gpu_rgba.astype(np.float64) - ref["rgba"]).max(1)
    flagged = (ref["margin"] < 1e-5) | (ref["flags"] != 0)
    jump = np.where(flagged, ref["jump"], 0.0)
    assert np.isfinite(jump).all(), "a pixel with more near decisions than the oracle bounds"
    bad = err > tol + jump
    assert not bad.any(), (
        f"{int(bad.sum())} pixels beyond tol + jump; worst: index {int(np.argmax(err - jump))}, "
        f"err {float((err - jump).max()):.3e} over the allowance, flagged {bool(flagged[np.argmax(err - jump)])}")
    if T is not None:
        eT = np.abs(np.asarray(T, np.float64) - ref["T"])
        assert not (eT > tol + jump).any(), float((eT - jump).max())
    n = err.size
    nf, nl = int(flagged.sum()), int((jump > tol).sum())
    assert nf <= max_flagged * n, (nf, n)
    assert nl <= max_loosened * n, (nl, n)
    e_ok = float(err[~flagged].max()) if (~flagged).any() else 0.0
    return e_ok, nf, nl


def rect_pairs(px0, px1, py0, py1, idx, tw, th, tiles_x):
    """(Gaussian, tile) pairs of pixel bboxes in tiles of tw x th: every
    tile of each rect, as int64 codes gaussian * 2^32 + tile."""
    tx0, tx1 = px0 // tw, px1 // tw
    ty0, ty1 = py0 // th, py1 // th
    w = (tx1 - tx0 + 1).astype(np.int64)
    h = (ty1 - ty0 + 1).astype(np.int64)
    cnt = w * h
    rep = np.repeat(np.arange(idx.size), cnt)
    local = np.arange(int(cnt.sum()), dtype=np.int64) - np.repeat(np.cumsum(cnt) - cnt, cnt)
    ty = ty0[rep].astype(np.int64) + local // w[rep]
    tx = tx0[rep].astype(np.int64) + local % w[rep]
    return (idx[rep].astype(np.int64) << 32) | (ty * tiles_x + tx)


def assert_pairs_harmless(orc, ref, cam, codes, tile=(16, 16)):
    """Every (Gaussian, tile) pair in `codes` has weight below alpha_min at
    every pixel centre of the tile (the oracle's exact maximum): the pair
    cannot change any pixel."""
    if codes.size == 0:
        return 0
    g = (codes >> 32).astype(np.uint32)
    t = (codes & 0xFFFFFFFF).astype(np.uint32)
    w = orc.pair_max_weight(ref, cam, g, t, dict(tile_w=tile[0], tile_h=tile[1]))
    assert w.max() < (1.0 / 255.0), (float(w.max()), int(g[np.argmax(w)]))
    return int(codes.size)


def compare_records(orc, rec, ref, cam):
    """GPU per-Gaussian records vs oracle records (Eq. 1, colour, culls)."""
    vis_o = ref.visible
    vis_g = rec["px1"] >= rec["px0"]
    amb = ref.i[:, orc.I_AMBIG] == 1
    # The GPU widens the opacity-aware bbox by a rounding margin, so a
    # Gaussian whose exact footprint holds no pixel centre can keep a
    # non-empty bbox: allowed only where every pixel of its tiles has
    # weight below alpha_min (compositing then skips it everywhere).
    kept = vis_g & ~vis_o & ~amb & (ref.i[:, orc.I_CULL] == orc.C_OFFIMAGE)
    if kept.any():
        k = np.nonzero(kept)[0]
        r = rec[k]
        tiles_x = (cam.width + 15) // 16
        assert_pairs_harmless(orc, ref, cam, rect_pairs(r["px0"], r["px1"], r["py0"], r["py1"],
                                                        k, 16, 16, tiles_x))
    mismatch = (vis_o != vis_g) & ~amb & ~kept
    assert not mismatch.any(), np.nonzero(mismatch)[0][:10]
    v = vis_o & vis_g
    d = ref.d[v]
    r = rec[v]
    # the 2-D mean to 1e-4 px anywhere in the image (it enters the weight
    # through the pixel offset), the depth (the sort key) to one float32 spacing
    np.testing.assert_allclose(r["mx"], d[:, orc.D_MX], rtol=0, atol=1e-4)
    np.testing.assert_allclose(r["my"], d[:, orc.D_MY], rtol=0, atol=1e-4)
    np.testing.assert_allclose(r["depth"], d[:, orc.D_DEPTH], rtol=2.0 ** -23)
    np.testing.assert_allclose(r["op"], d[:, orc.D_OPAC], rtol=2e-6)
    np.testing.assert_allclose(np.stack([r["r"], r["g"], r["b"]], 1), d[:, orc.D_R:orc.D_B + 1], atol=2e-6)
    con = conic_from_whitened(r)
    ref_con = d[:, orc.D_CA:orc.D_CC + 1]
    scale = np.abs(ref_con).max(1, keepdims=True)
    np.testing.assert_allclose(con / scale, ref_con / scale, atol=2e-5)
    # pixel bboxes: the GPU's may only be larger, by pixels that hold no
    # weight >= alpha_min (extra_pairs_harmless checks the tiles)
    it = ref.i[v]
    assert np.all(r["px0"] <= it[:, orc.I_PX0]) and np.all(r["px1"] >= it[:, orc.I_PX1])
    assert np.all(r["py0"] <= it[:, orc.I_PY0]) and np.all(r["py1"] >= it[:, orc.I_PY1])
    return v


def pair_set_check(orc, ref, rec, cam, v, tile=(16, 16)):
    """The GPU's (Gaussian, tile) pairs of the Gaussians in `v` (from its
    pixel bboxes) against the oracle's exact rects in tiles of `tile`:
    every oracle pair is present, and every extra GPU pair is harmless.
    Returns (oracle pairs, extra pairs)."""
    tw, th = tile
    tiles_x = -(-cam.width // tw)
    idx = np.nonzero(v)[0]
    r, it = rec[idx], ref.i[idx]
    g = rect_pairs(r["px0"], r["px1"], r["py0"], r["py1"], idx, tw, th, tiles_x)
    o = rect_pairs(it[:, orc.I_PX0], it[:, orc.I_PX1], it[:, orc.I_PY0], it[:, orc.I_PY1],
                   idx, tw, th, tiles_x)
    missing = np.setdiff1d(o, g, assume_unique=True)
    assert missing.size == 0, missing[:5]
    extra = np.setdiff1d(g, o, assume_unique=True)
    assert_pairs_harmless(orc, ref, cam, extra, tile)
    return int(o.size), int(extra.size)


def extra_pairs_harmless(orc, ref, rec, cam, v):
    return pair_set_check(orc, ref, rec, cam, v)[1]


_SCENES = {}


def scene_cached(name):
    """The full-size medium (1M, view 0) or large (6M) scene and camera,
    generated once per test process (read-only: do not modify)."""
    from paper_2512_08478_amd import scenes as S
    if name not in _SCENES:
        if len(_SCENES) >= 2:
            _SCENES.clear()
        _SCENES[name] = {"medium": S.medium_scene, "large": S.large_scene}[name]()
    return _SCENES[name]


def sampled_pixels(cam, n, seed):
    rng = np.random.default_rng(seed)
    pix = np.stack([rng.integers(0, cam.width, n), rng.integers(0, cam.height, n)], 1)
    corners = np.array([[0, 0], [cam.width - 1, cam.height - 1], [cam.width // 2, cam.height // 2],
                        [cam.width - 1, 0], [0, cam.height - 1]])
    return np.concatenate([pix, corners]).astype(np.int32)


def near_tie(x, h, scale=None):
    """True where float64 x lies within float64 rounding of the midpoint
    between binary16 h and a neighbour (either answer is then correct).
    The rounding of x is taken relative to max(|x|, scale): pass the
    magnitude of the terms x was summed from where they may cancel."""
    x = np.asarray(x, np.float64)
    hf = h.astype(np.float64)
    sp = np.spacing(np.abs(h)).astype(np.float64)
    mid = np.abs(np.abs(x) - np.abs(hf))
    mag = np.abs(x) if scale is None else np.maximum(np.abs(x), scale)
    return np.abs(mid - 0.5 * sp) <= 1e-12 * np.maximum(mag, 1e-30)
