"""Helpers for the GPU tests: run the HIP path through the C ABI and read
its outputs back as numpy."""
import numpy as np
import torch

SPLAT_DTYPE = np.dtype([("mx", "<f4"), ("my", "<f4"), ("qa", "<f4"), ("qb", "<f4"), ("qc", "<f4"),
                        ("op", "<f4"), ("r", "<f4"), ("g", "<f4"), ("b", "<f4"), ("depth", "<f4"),
                        ("px0", "<u2"), ("py0", "<u2"), ("px1", "<u2"), ("py1", "<u2")])
assert SPLAT_DTYPE.itemsize == 48
_TILED = np.dtype(SPLAT_DTYPE.descr + [("tx0", "<i8"), ("ty0", "<i8"), ("tx1", "<i8"), ("ty1", "<i8")])


def splats_np(splats_u8, n, tile=(16, 16)):
    """The records as a structured array, plus the tile rect (tx0, ty0,
    tx1, ty1) of each record's pixel bbox for tiles of `tile` pixels
    (culled records keep an empty rect, tx1 < tx0)."""
    raw = splats_u8[: n * 48].cpu().numpy().view(SPLAT_DTYPE)
    out = np.zeros(raw.shape, _TILED)
    for f in SPLAT_DTYPE.names:
        out[f] = raw[f]
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


def image_check(gpu_rgba, ref, tol=1e-4, flagged_tol=2e-2):
    """Compare a GPU image (P,4) to oracle outputs at the same pixels.

    Unflagged pixels (decision margin >= 1e-5, no depth tie, no ambiguous
    cull) must be within `tol`; flagged ones within the jump they straddle
    (bounded by `flagged_tol`).  Returns (max err unflagged, n flagged)."""
    err = np.abs(gpu_rgba.astype(np.float64) - ref["rgba"]).max(1)
    flagged = (ref["margin"] < 1e-5) | (ref["flags"] != 0)
    e_ok = err[~flagged].max() if (~flagged).any() else 0.0
    assert e_ok <= tol, (e_ok, np.argmax(np.where(flagged, 0, err)))
    if flagged.any():
        assert err[flagged].max() <= flagged_tol, err[flagged].max()
    return e_ok, int(flagged.sum())


def compare_records(orc, rec, ref, cam):
    """GPU per-Gaussian records vs oracle records (Eq. 1, colour, culls)."""
    vis_o = ref.visible
    vis_g = rec["tx1"] >= rec["tx0"]
    amb = ref.i[:, orc.I_AMBIG] == 1
    # The GPU widens the opacity-aware bbox by a rounding margin, so a
    # Gaussian whose exact footprint holds no pixel centre can keep a
    # non-empty bbox: allowed only where every pixel of its tiles has
    # weight below alpha_min (compositing then skips it everywhere).
    kept = vis_g & ~vis_o & ~amb & (ref.i[:, orc.I_CULL] == orc.C_OFFIMAGE)
    if kept.any():
        tx_n = (cam.width + 15) // 16
        gs, tiles = [], []
        for g in np.nonzero(kept)[0]:
            a = rec[g]
            for ty in range(a["ty0"], a["ty1"] + 1):
                for tx in range(a["tx0"], a["tx1"] + 1):
                    gs.append(g)
                    tiles.append(ty * tx_n + tx)
        w = orc.pair_max_weight(ref, cam, np.array(gs), np.array(tiles))
        assert w.max() < (1.0 / 255.0) * (1 + 1e-5), w.max()
    mismatch = (vis_o != vis_g) & ~amb & ~kept
    assert not mismatch.any(), np.nonzero(mismatch)[0][:10]
    v = vis_o & vis_g
    d = ref.d[v]
    r = rec[v]
    np.testing.assert_allclose(r["mx"], d[:, orc.D_MX], rtol=2e-6, atol=2e-3)
    np.testing.assert_allclose(r["my"], d[:, orc.D_MY], rtol=2e-6, atol=2e-3)
    np.testing.assert_allclose(r["depth"], d[:, orc.D_DEPTH], rtol=1e-6)
    np.testing.assert_allclose(r["op"], d[:, orc.D_OPAC], rtol=2e-6)
    np.testing.assert_allclose(np.stack([r["r"], r["g"], r["b"]], 1), d[:, orc.D_R:orc.D_B + 1], atol=2e-6)
    con = conic_from_whitened(r)
    ref_con = d[:, orc.D_CA:orc.D_CC + 1]
    scale = np.abs(ref_con).max(1, keepdims=True)
    np.testing.assert_allclose(con / scale, ref_con / scale, atol=2e-5)
    # pixel bboxes and tile rects: the GPU's may only be larger, by pixels
    # and tiles that hold no pixel with weight >= alpha_min
    it = ref.i[v]
    assert np.all(r["px0"] <= it[:, orc.I_PX0]) and np.all(r["px1"] >= it[:, orc.I_PX1])
    assert np.all(r["py0"] <= it[:, orc.I_PY0]) and np.all(r["py1"] >= it[:, orc.I_PY1])
    assert np.all(r["tx0"] <= it[:, orc.I_TX0]) and np.all(r["tx1"] >= it[:, orc.I_TX1])
    assert np.all(r["ty0"] <= it[:, orc.I_TY0]) and np.all(r["ty1"] >= it[:, orc.I_TY1])
    return v


def extra_pairs_harmless(orc, ref, rec, cam, v):
    tx_n = (cam.width + 15) // 16
    gs, tiles = [], []
    for g in np.nonzero(v)[0]:
        a, b = rec[g], ref.i[g]
        for ty in range(a["ty0"], a["ty1"] + 1):
            for tx in range(a["tx0"], a["tx1"] + 1):
                if not (b[orc.I_TX0] <= tx <= b[orc.I_TX1] and b[orc.I_TY0] <= ty <= b[orc.I_TY1]):
                    gs.append(g)
                    tiles.append(ty * tx_n + tx)
    if gs:
        w = orc.pair_max_weight(ref, cam, np.array(gs), np.array(tiles))
        assert w.max() < (1.0 / 255.0) * (1 + 1e-5)
    return len(gs)


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
