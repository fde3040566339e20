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
