"""Helpers for the GPU tests: run the HIP path through the C ABI and read
its outputs back as numpy."""
import numpy as np
import torch

SPLAT_DTYPE = np.dtype([("mx", "<f4"), ("my", "<f4"), ("qa", "<f4"), ("qb", "<f4"), ("qc", "<f4"),
                        ("op", "<f4"), ("r", "<f4"), ("g", "<f4"), ("b", "<f4"), ("depth", "<f4"),
                        ("tx0", "<u2"), ("ty0", "<u2"), ("tx1", "<u2"), ("ty1", "<u2")])
assert SPLAT_DTYPE.itemsize == 48


def splats_np(splats_u8, n):
    return splats_u8[: n * 48].cpu().numpy().view(SPLAT_DTYPE)


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
