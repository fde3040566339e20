"""Benchmark of the per-frame 3DGS render path on one MI355X.

Default workload: the 1,000,000-Gaussian clustered scene (SH degree 3) at
1920x1080, forward (preprocess -> keys + radix sort -> tile compositing),
inputs resident in HBM.  A step is one whole frame.  Prints ONE JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload medium|large|diff|tiny]
                  [--packed]

--packed renders from the FP16 pre-pack (Section 3.4): the Gaussians are
pre-packed once before timing, and every frame preprocesses the binary16
mean, opacity, upper covariance and SH (forward workloads only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frames/sec @1080p, 1M–6M Gaussians, fwd and fwd+bwd; sort Gkeys/s; % HBM peak"
HBM_PEAK_GBS = 8000.0

FP32_VECTOR_PEAK_TFLOPS = 157.3
# FP32 operations Eqs. 2-3 need per composited (pixel, Gaussian) pair:
# offset 2, quadratic form with the conic 7, o*exp(-Q/2) 3, clamp + skip
# test 2, T*alpha and the three colour FMAs 7, T *= 1 - alpha 2, stop test 1.
FLOPS_PER_BLEND = 24

SORT_KERNELS = ("sort_init", "radix_hist", "depth_pass", "kg_count", "kg_hist", "kg_scan", "keygen",
                "tile_pass", "tile_ranges", "tile_order")
HBM_KERNELS = ("preprocess", "preprocess_packed", "lbs", "depth_pass", "keygen", "kg_count", "kg_hist", "tile_pass",
               "tile_ranges", "preprocess_bwd")
ALU_KERNELS = ("raster", "raster_mesh", "raster_bwd")

WORKLOADS = {
    "tiny": "tiny: 4,096 Gaussians, SH degree 0, 256x256, forward",
    "medium": "medium: 1,000,000 Gaussians (64 clusters in [-5,5]^3), SH degree 3, 1920x1080, forward",
    "large": "large: 6,000,000 Gaussians (64 clusters in [-20,20]^3), SH degree 3, 1920x1080 eye inside, forward",
    "diff": "diff: 500,000 Gaussians, SH degree 3, 800x800, forward+backward (L1)",
    "avatar": "avatar: the medium scene skinned to 55 joints (4 influences each), FP16 "
              "pre-packed; every frame runs the linear-blend-skinning pre-decoder on a posed "
              "skeleton, then the packed forward",
    "mesh": "mesh: the medium scene composited with a mesh prepass (a plane through the "
            "scene centre facing the camera, 40% of its cells left out), forward",
    "sort32": "sort32: depth-only global sort of the 32-bit depth keys (culled = largest key) of "
              "the 6M-generator scene at 0.758/1.515/3.031/6.062 M Gaussians, 1920x1080 camera "
              "inside the cloud",
    "batched": "batched: 2M-Gaussian scene + 8 placed assets (50k-1M, 4.5M total), SH degree 3, "
               "32 views 512..1920 x 512..1080, forward+backward (L1), one graph launch, "
               "autotuned tile shape / digit width / sort mode",
}


# Launch configuration per workload (tile shape, digit width, compositing
# order), the fastest of an A/B over the autotuner's space (--tile auto
# searches it again) on MI355X.  Fixed by
# default so that the counter measurements of the timed kernels
# (profiles/pmc_traffic.json) belong to the configuration the bench times.
TUNED = {
    "tiny": ("16x16", 8, 1),
    "medium": ("32x16", 6, 1),
    "large": ("8x8", 8, 5),
    "diff": ("32x16", 6, 1),
    "avatar": ("32x16", 6, 1),
    "mesh": ("32x16", 6, 1),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="medium", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", default=None,
                    help="WxH; auto: the autotuner picks tile shape, digit width and "
                         "compositing order; default: the workload's tuned configuration")
    ap.add_argument("--radix-bits", type=int, default=None)
    ap.add_argument("--sort-mode", type=int, default=0)
    ap.add_argument("--raster-order", type=int, default=None,
                    help="bit 0: longest tile lists first (else spatial runs); "
                         "order >> 1 = s: forward quadrants in 2^s row bands")
    ap.add_argument("--packed", action="store_true",
                    help="forward from the FP16 pre-packed inputs (pre-packed once, untimed)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="medium only: skip the 6M forward and 500k forward+backward frames")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    ap.add_argument("--verbose", action="store_true")
    return ap.parse_args()


def make_workload(name):
    from paper_2512_08478_amd import scenes as S
    if name == "tiny":
        return S.tiny_scene()
    if name == "medium":
        return S.medium_scene()
    if name == "large":
        return S.large_scene()
    if name == "diff":
        return S.diff_scene()
    if name in ("mesh", "avatar"):
        return S.medium_scene()
    raise ValueError(name)


def make_mesh(cam):
    """The mesh workload's prepass: a plane through the origin, roughly
    facing the camera, with holes."""
    import numpy as np
    from paper_2512_08478_amd import scenes as S
    fwd = np.asarray(cam.viewmat, np.float64)[2, :3]
    return S.plane_mesh(cam, fwd + np.array([0.1, 0.3, 0.0]), 0.0, seed=8, occupancy=0.6)


def packed_sh_halves(K):
    return (3 * K + 3) // 4 * 4


def algorithmic_bytes(n, n_vis, inst, K, W, H, tiles, depth_passes=4):
    """Bytes each kernel must move (reads + writes), per launch."""
    return {
        # means 12 + log-scales 12 + quats 16 + logit 4 read, 48 B record + 4 B depth key
        # + 8 B tile rect written per Gaussian; SH 12K bytes read per visible one
        "preprocess": n * (44 + 60) + n_vis * 12 * K,
        # binary16 mean + opacity 8 + covariance 12 read, the same 60 B written per
        # Gaussian; the packed SH row (2 bytes a half) read per visible one
        "preprocess_packed": n * (20 + 60) + n_vis * 2 * packed_sh_halves(K),
        # canonical mean/opacity 8 + covariance 12 + joint indices 4 + weights 16 read,
        # deformed mean/opacity 8 + covariance 12 written per Gaussian
        "lbs": n * 60,
        # depth passes (upsweep, scan and downsweep together), averaged per pass:
        # the first reads every Gaussian's u32 key (values are positions) and
        # writes key + value of the visible ones; each later pass reads and
        # writes u32 key + u32 value per visible Gaussian
        "depth_pass": (n * 4 + n_vis * 8 + (depth_passes - 1) * n_vis * 16) / max(depth_passes, 1),
        # sorted index 4 read, tile rect 8 gathered and written in depth order per
        # visible Gaussian
        "kg_count": n_vis * 20,
        # the same, plus the first-tile-digit histogram of each slice (LDS only)
        "kg_hist": n_vis * 20,
        # sorted index 4 + sorted rect 8 read per visible Gaussian; tile key 4 +
        # value 4 written per instance (in the first tile pass's order when the
        # keygen is fused with that pass)
        "keygen": n_vis * 12 + inst * 8,
        # per tile pass: u32 key + u32 value read and written per instance
        "tile_pass": inst * 16,
        # sorted tile keys read, two u32 per tile written
        "tile_ranges": inst * 4 + tiles * 8,
        # value + 48 B record gathered per instance, RGBA + T + last written per pixel
        "raster": inst * (4 + 48) + tiles * 8 + W * H * 24,
        # parameters (44 B) + SH (12K) + 2-D gradient record (48) read and all
        # parameter gradients (44 + 12K) written per visible Gaussian
        "preprocess_bwd": n_vis * (44 + 12 * K + 48 + 44 + 12 * K),
    }


def traffic_key(workload, kernel, cfg):
    """Key of a counter measurement: the workload, the kernel and the launch
    configuration it was taken in (tile shape, digit width, sort mode and
    compositing order all change what a kernel reads)."""
    return (f"{workload}/{kernel}/{cfg['tile_w']}x{cfg['tile_h']}/b{cfg['radix_bits']}"
            f"/m{cfg['sort_mode']}/o{cfg['raster_order']}")


def profile_record(name, workload, kernel, cfg):
    """The record of profiles/<name> for `kernel` in exactly this launch
    configuration, or None when there is none or the kernel's sources
    changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    try:
        rec = json.load(open(path))[traffic_key(workload, kernel, cfg)]
    except (OSError, KeyError, ValueError):
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        with open(os.path.join(ROOT, "paper_2512_08478_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec["source_sha256_16"]:
        return None
    return rec


def measured_traffic(workload, kernel, cfg):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE + WRITE_SIZE passes (copy-calibrated), taken in exactly this
    launch configuration, or None when there are none or the kernel's
    sources changed since."""
    rec = profile_record("pmc_traffic.json", workload, kernel, cfg)
    return None if rec is None else int(rec["bytes_per_launch"])


def measured_counters(workload, kernel, cfg):
    """VALU-busy and issue fractions, resident waves per SIMD and vector
    instructions per wave of `kernel`, from the committed rocprofv3 SQ
    counter pass in exactly this launch configuration (same conditions as
    measured_traffic), or None."""
    rec = profile_record("pmc_counters.json", workload, kernel, cfg)
    if rec is None:
        return None
    return {k: rec[k] for k in ("valu_busy", "valu_issue", "waves_per_simd", "valu_insts_per_wave")
            if k in rec}


def evaluated_pairs(np, last, T_final, ranges, W, H, tw, th, t_eps):
    """(pixel, Gaussian) pairs Eq. 3 evaluates: each pixel walks its tile's
    list front to back up to the splat after which T fell below t_eps (`last`
    holds one past that splat's rank in the list), or to the list's end."""
    last = last.reshape(-1).view(np.uint32).astype(np.int64)
    T = T_final.reshape(-1)
    r = ranges.reshape(-1).view(np.uint32).astype(np.int64)
    tx = (W + tw - 1) // tw
    py, px = np.divmod(np.arange(W * H), W)
    tile = (py // th) * tx + px // tw
    length = r[2 * tile + 1] - r[2 * tile]
    walk = np.where(T < t_eps, last, length)
    return int(walk.sum())


# Frames timed one by one for the warm and cold medians and percentiles
# (at least this many, whatever --steps is).
PERCENTILE_FRAMES = 200


def frame_percentiles(torch, step, n, flush):
    """Median, p10 and p90 of n frame times (ms), each bracketed by events on
    the stream the frame runs on; with `flush`, that buffer (1 GiB) is read
    before every frame (outside the events)."""
    import numpy as np
    ev = []
    for _ in range(n):
        if flush is not None:
            flush.sum()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        step()
        b.record()
        ev.append((a, b))
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in ev])
    return {"median": round(float(np.median(t)), 4), "p10": round(float(np.percentile(t, 10)), 4),
            "p90": round(float(np.percentile(t, 90)), 4)}


def traced_stages(L, step, reps, flush):
    """Per-frame and per-launch kernel times (ms) over `reps` frames, from the
    HIP events libgs records around its own launches; with `flush`, that
    buffer (1 GiB) is read before every frame (not traced)."""
    L.trace_enable(True)
    acc, cnt = {}, {}
    for _ in range(reps):
        if flush is not None:
            flush.sum()
        step()
        for lab, ms in L.trace_read():
            acc[lab] = acc.get(lab, 0.0) + ms
            cnt[lab] = cnt.get(lab, 0) + 1
    L.trace_enable(False)
    return {k: acc[k] / reps for k in acc}, {k: acc[k] / cnt[k] for k in acc}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.packed and args.workload not in ("tiny", "medium", "large", "mesh"):
        print(json.dumps({"error": "--packed applies to the forward workloads tiny, medium, large, "
                                   "mesh"}))
        sys.exit(2)
    if args.workload == "batched":
        print(json.dumps(run_batched(args)), flush=True)
        return
    if args.workload == "sort32":
        return run_sort32(args)
    out = run_view(args, full=True)
    if args.workload == "medium" and not args.packed and not args.no_extra:
        # the metric's other frames (6M forward, 500k forward + backward),
        # autotuned and timed the same way
        import copy
        extra = {}
        for w in ("large", "diff"):
            a2 = copy.copy(args)
            a2.workload = w
            a2.calib_copy_mib = 0
            e = run_view(a2, full=False)
            extra[w] = {k: e[k] for k in ("value", "unit", "ms_per_step", "sort_ms", "sort_gkeys_per_s",
                                          "frame_ms", "roofline")}
            extra[w]["config"] = e["config"]
            extra[w]["stages"] = {k: {kk: vv for kk, vv in v.items()
                                      if kk in ("ms_per_frame", "gbs", "hbm_frac", "tflops", "alu_frac")}
                                  for k, v in e["stages"].items()}
        # the batched views (32 views x 4.5M Gaussians, forward + backward, one
        # graph launch per step)
        a2 = copy.copy(args)
        a2.workload = "batched"
        a2.steps, a2.warmup = min(args.steps, 10), min(args.warmup, 2)
        e = run_batched(a2, full=False)
        extra["batched"] = {k: e[k] for k in ("value", "unit", "ms_per_step", "plain_frames_per_s",
                                              "graph_speedup_vs_plain",
                                              "images_bitwise_equal_to_plain",
                                              "launches_per_batch", "roofline")}
        extra["batched"]["config"] = e["config"]
        out["extra_workloads"] = extra
    print(json.dumps(out), flush=True)


def run_view(args, full):
    """One single-view workload: autotune, time, trace; returns the result
    dict (with the CPU baseline when `full`)."""
    import numpy as np
    import torch
    from paper_2512_08478_amd import _lib as L
    from paper_2512_08478_amd.render import GaussianParams, Renderer

    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib * 2**20 // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sc, cam = make_workload(args.workload)
    p = GaussianParams.from_scene(sc)
    if args.packed or args.workload == "avatar":
        # the pre-pack runs once per asset, before any frame (Algorithm 1)
        p = Renderer().prepack(p)
        torch.cuda.synchronize()
    skin = skin_np = None
    if args.workload == "avatar":
        from paper_2512_08478_amd import scenes as S
        centres, jidx, jw = S.skinning(sc.means, n_joints=55, seed=0)
        dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
        skin_np = (jidx, jw, S.joint_pose(centres, seed=1))
        skin = tuple(dev(a) for a in skin_np)
        canon = p
        p = Renderer().lbs_deform(canon, *skin)   # the posed frame, for tuning and sizing
        torch.cuda.synchronize()
    backward = args.workload == "diff"
    mesh = make_mesh(cam) if args.workload == "mesh" else None
    H, W = cam.height, cam.width
    target = None
    if backward:
        from paper_2512_08478_amd import scenes as S
        target = torch.from_numpy(S.random_target(4, H, W)).cuda()
    tuned = None
    if args.tile == "auto":
        from paper_2512_08478_amd.batch import autotune_view
        best, table = autotune_view(p, cam, backward=backward, target=target,
                                    base_settings=dict(sort_mode=args.sort_mode), mesh=mesh)
        tw, th, bits = best["tile_w"], best["tile_h"], best["radix_bits"]
        order = best["raster_order"]
        tuned = [[f"{t[0]['tile_w']}x{t[0]['tile_h']}/{t[0]['radix_bits']}b/o{t[0]['raster_order']}",
                  round(t[1] * 1e3, 4)] for t in table]
    else:
        tile, bits, order = TUNED[args.workload]
        tw, th = map(int, (args.tile or tile).split("x"))
        bits = args.radix_bits if args.radix_bits is not None else bits
        order = args.raster_order if args.raster_order is not None else order
    R = Renderer(dict(tile_w=tw, tile_h=th, radix_bits=bits, sort_mode=args.sort_mode,
                      raster_order=order))

    # first frame: read the instance count once to size the sort buffers
    fr = R.forward(p, cam, mesh=mesh)
    torch.cuda.synchronize()
    inst = fr.capacity
    mesh = fr.mesh   # device buffers, uploaded once
    capacity = inst
    depth_bits = fr.depth_bits   # the visible depth key range of this (static) view

    def step():
        if skin is not None:
            R.lbs_deform(canon, *skin, out=p)   # the pre-decoder runs every frame
        f = R.forward(p, cam, capacity=capacity, mesh=mesh, depth_bits=depth_bits)
        if backward:
            # L1 loss gradient w.r.t. RGB (the caller's loss, not part of the method)
            G = torch.zeros((H, W, 4), device="cuda")
            G[..., :3] = torch.sign(f.image[..., :3] - target) / (3.0 * H * W)
            R.backward(p, cam, f, G)
        return f

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    flag = int(f.flag[0].item()) & 0xFFFFFFFF
    if flag & 1:
        raise RuntimeError("instance capacity exceeded during the timed steps")
    if flag & 2:
        raise RuntimeError("depth key range wider than planned during the timed steps")

    # Warm frames run back to back; a cold frame first reads 1 GiB, four
    # times the 256 MB last-level cache (MALL), so its inputs come from HBM.
    # A read leaves clean lines behind: a written flush buffer would make
    # the frame pay for writing the cache's dirty lines back.
    flush = torch.ones(2**28, dtype=torch.float32, device="cuda")
    frame_dist = {"warm": frame_percentiles(torch, step, max(args.steps, PERCENTILE_FRAMES), None),
                  "cold": frame_percentiles(torch, step, max(args.steps, PERCENTILE_FRAMES), flush)}

    # The same frames sized per frame, as for a scene that changes: the
    # instance count and depth key range are read back (one host sync) before
    # each sort, instead of the plan taken once from the first frame.
    def step_sized():
        if skin is not None:
            R.lbs_deform(canon, *skin, out=p)
        f = R.forward(p, cam, mesh=mesh)
        if backward:
            G = torch.zeros((H, W, 4), device="cuda")
            G[..., :3] = torch.sign(f.image[..., :3] - target) / (3.0 * H * W)
            R.backward(p, cam, f, G)
        return f

    for _ in range(args.warmup):
        step_sized()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_sized()
    torch.cuda.synchronize()
    ms_sized = (time.perf_counter() - t0) * 1e3 / args.steps

    # The 1M scene's whole 8-view orbit (the same launch configuration; each
    # view planned once from its first frame, like view 0 above)
    orbit = None
    if args.workload == "medium" and not args.packed:
        from paper_2512_08478_amd import scenes as S
        per_view = []
        for v in range(8):
            cv = S.orbit_camera(v, 8, 8.0, W, H)
            fv = R.forward(p, cv)
            torch.cuda.synchronize()
            cap_v, db_v = fv.capacity, fv.depth_bits
            for _ in range(args.warmup):
                R.forward(p, cv, capacity=cap_v, depth_bits=db_v)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fv = R.forward(p, cv, capacity=cap_v, depth_bits=db_v)
            torch.cuda.synchronize()
            ms_v = (time.perf_counter() - t0) * 1e3 / args.steps
            if int(fv.flag[0].item()) & 3:
                raise RuntimeError(f"orbit view {v}: plan exceeded during the timed steps")
            per_view.append((round(ms_v, 4), int(cap_v)))
        orbit = {"ms_per_view": [m for m, _ in per_view],
                 "instances_per_view": [c for _, c in per_view],
                 "frames_per_s": round(8000.0 / sum(m for m, _ in per_view), 2)}

    # per-kernel durations, measured with HIP events recorded by libgs on the
    # stream its kernels run on
    reps = max(5, min(20, args.steps))
    kern_ms, kern_avg = traced_stages(L, step, reps, None)
    cold_ms, cold_avg = traced_stages(L, step, reps, flush)
    del flush

    # composited (pixel, Gaussian) pairs of this frame, for the compositing
    # roofline, and the pairs Eq. 3 evaluates (each pixel walks its tile's
    # list up to its stop)
    nbl = torch.empty((H, W), dtype=torch.int32, device="cuda")
    R.rasterize(f.splats, f.values, f.ranges, cam, n_blend=nbl, mesh=f.mesh)
    blends = int(nbl.sum(dtype=torch.int64).item())
    del nbl
    evals = evaluated_pairs(np, f.last.cpu().numpy(), f.T_final.cpu().numpy(),
                            f.ranges.cpu().numpy(), W, H, tw, th, R.settings.t_eps)

    rec = f.splats[: sc.n * 48].cpu().numpy().view(np.uint16).reshape(sc.n, 24)
    n_vis = int(np.count_nonzero(rec[:, 22] >= rec[:, 20]))
    K = (sc.sh_degree + 1) ** 2
    tiles = R.tiles(cam)
    import ctypes
    key_bits = L.load().gs_sort_key_bits(ctypes.byref(L.make_camera(cam)), ctypes.byref(R.settings))
    if depth_bits > 0 and args.sort_mode == 0:
        depth_passes = -(-depth_bits // 9)
    else:
        depth_passes = -(-(depth_bits or 32) // bits)
    passes = [depth_passes, -(-(key_bits - 32) // bits)]
    ab = algorithmic_bytes(sc.n, n_vis, inst, K, W, H, tiles, depth_passes=passes[0])
    stages = {}
    for k, v in kern_avg.items():
        e = {"ms_per_launch": round(v, 5), "ms_per_frame": round(kern_ms[k], 5)}
        if k in ab:
            gbs = ab[k] / (v * 1e-3) / 1e9
            e.update(algo_bytes=int(ab[k]), gbs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
        stages[k] = e
    # compositing: blended pairs x FLOPS_PER_BLEND (the backward revisits
    # every blended pair once more, with roughly twice the arithmetic)
    flops = {"raster": blends * FLOPS_PER_BLEND, "raster_mesh": blends * FLOPS_PER_BLEND,
             "raster_bwd": blends * 2 * FLOPS_PER_BLEND}
    for k in ALU_KERNELS:
        if k in stages:
            tf = flops[k] / (kern_avg[k] * 1e-3) / 1e12
            stages[k].update(algo_flops=int(flops[k]), tflops=round(tf, 3),
                             alu_frac=round(tf / FP32_VECTOR_PEAK_TFLOPS, 4),
                             evaluated_pairs=evals,
                             gevals_per_s=round(evals / (kern_avg[k] * 1e-3) / 1e9, 2))
    stages_cold = {}
    for k, v in cold_avg.items():
        e = {"ms_per_launch": round(v, 5)}
        if k in ab:
            gbs = ab[k] / (v * 1e-3) / 1e9
            e.update(gbs=round(gbs, 1), hbm_frac=round(gbs / HBM_PEAK_GBS, 4))
        stages_cold[k] = e
    sort_ms = sum(kern_ms.get(k, 0.0) for k in SORT_KERNELS)
    # roofline of the kernel that takes the most time per frame
    dom = max(kern_ms, key=lambda k: kern_ms[k])
    if dom in ALU_KERNELS:
        tf = flops[dom] / (kern_avg[dom] * 1e-3) / 1e12
        roofline = {"kernel": dom, "bound": "alu", "achieved": round(tf, 3),
                    "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
                    "algo_flops_per_launch": int(flops[dom]), "blended_pairs": blends,
                    "evaluated_pairs": evals}
    else:
        dom_gbs = ab[dom] / (kern_avg[dom] * 1e-3) / 1e9
        roofline = {"kernel": dom, "bound": "hbm", "achieved": round(dom_gbs, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                    "traffic": None, "algo_bytes_per_launch": int(ab[dom])}
    roofline["ms_per_launch"] = round(kern_avg[dom], 5)
    dom_cfg = dict(tile_w=tw, tile_h=th, radix_bits=bits, sort_mode=args.sort_mode,
                   raster_order=order)
    roofline["traffic"] = measured_traffic(args.workload, dom, dom_cfg)
    if roofline["bound"] == "alu":
        # what the SQ counters say of the same kernel (an ALU fraction on
        # blended pairs' flops alone understates an issue-bound kernel)
        roofline["counters"] = measured_counters(args.workload, dom, dom_cfg)

    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms_per_step, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + (
                       ", FP16 pre-packed inputs" if args.packed and args.workload != "avatar"
                       else ""),
                   "n_gaussians": sc.n, "width": W, "raster_order": order,
                   "height": H, "tile": f"{tw}x{th}", "radix_bits": bits,
                   "visible": n_vis, "instances": inst, "key_bits": key_bits,
                   "depth_bits": depth_bits, "depth_passes": passes[0], "tile_passes": passes[1],
                   "first_tile_pass_fused_with_keygen": args.sort_mode == 0},
        "sort_gkeys_per_s": round(inst / (sort_ms * 1e-3) / 1e9, 3) if sort_ms > 0 else None,
        "sort_ms": round(sort_ms, 4),
        "stages": stages,
        "frame_ms": frame_dist,
        "ms_per_step_sized_per_frame": round(ms_sized, 4),
        "frames_per_s_sized_per_frame": round(1000.0 / ms_sized, 2),
        "orbit_8_views": orbit,
        "stages_cold": stages_cold,
        "roofline": roofline,
    }
    if tuned is not None:
        out["autotune_ms_per_frame"] = tuned

    if full and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(
            sc, cam, dict(tile_w=16, tile_h=16), packed=args.packed or skin_np is not None,
            mesh=make_mesh(cam) if args.workload == "mesh" else None, skin=skin_np)
    return out


# Table 1's Sort column (ms; an RTX 4090 in WebGPU), at its four Gaussian
# counts: context for the depth-only sort, not a target.
PAPER_SORT_MS = {758_000: 0.20, 1_515_000: 0.22, 3_031_000: 0.32, 6_062_000: 0.58}


def run_sort32(args):
    """Depth-only 32-bit key sort (the sort the paper times in Table 1) over
    the Table-1-shaped sweep of Gaussian counts."""
    import ctypes
    import torch
    from paper_2512_08478_amd import _lib as L
    from paper_2512_08478_amd import scenes as S
    from paper_2512_08478_amd.render import GaussianParams, Renderer

    sc, cam = S.large_scene(n=max(PAPER_SORT_MS))
    bits = args.radix_bits or 8
    R = Renderer(dict(radix_bits=bits, sort_mode=args.sort_mode))
    p = GaussianParams.from_scene(sc)
    _, dkeys, _, _ = R.preprocess(p, cam, reuse=False)
    torch.cuda.synchronize()
    flush = torch.ones(2**28, dtype=torch.float32, device="cuda")
    rows, ms_at_max = [], None
    for n in sorted(PAPER_SORT_MS):
        keys = dkeys[:n]  # the generator's draws are i.i.d., so a prefix is a random subset
        for _ in range(args.warmup):
            R.sort_pairs32(keys)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            R.sort_pairs32(keys)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        # cold: 1 GiB read before each sort, so the keys come from HBM
        cold = frame_percentiles(torch, lambda: R.sort_pairs32(keys), args.steps, flush)
        rows.append({"n": n, "ms": round(ms, 4), "gkeys_per_s": round(n / (ms * 1e-3) / 1e9, 3),
                     "cold_ms_median": cold["median"], "paper_ms_rtx4090": PAPER_SORT_MS[n]})
        ms_at_max = ms
    n = max(PAPER_SORT_MS)
    # per-kernel times at the largest size (HIP events on the library's stream)
    L.trace_enable(True)
    R.sort_pairs32(dkeys[:n])
    tr = L.trace_read(4096)
    L.trace_enable(False)
    pass_ms = [ms for lab, ms in tr if lab == "sort32_pass"]
    passes = len(pass_ms)
    # algorithmic bytes of one pass: key + value read and written per key
    gbs = 16 * n / (sum(pass_ms) / passes * 1e-3) / 1e9 if passes else 0.0
    out = {
        "metric": METRIC,
        "value": round(n / (ms_at_max * 1e-3) / 1e9, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_at_max, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["sort32"], "n_keys": n, "radix_bits": bits,
                   "passes": passes},
        "sweep": rows,
        "roofline": {"kernel": "sort32_pass", "bound": "hbm", "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": None, "algo_bytes_per_launch": 16 * n,
                     "ms_per_launch": round(sum(pass_ms) / passes, 5) if passes else None},
    }
    if not args.no_cpu_baseline:
        import numpy as np
        import oracle
        k = dkeys[:n].cpu().numpy().view(np.uint32).astype(np.uint64)
        t0 = time.perf_counter()
        oracle.stable_sort_pairs(k, np.arange(n, dtype=np.uint32))
        t = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(n / t / 1e9, 4), "unit": "Gkeys/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"std::stable_sort of the same {n} keys ({t:.2f} s)"}
    print(json.dumps(out), flush=True)


def run_batched(args, full=True):
    """All views' forward + backward (L1) as one HIP graph launch per step
    (the library's gs_batch_capture / gs_batch_launch); returns the result
    dict (with the CPU baseline when `full`)."""
    import torch
    from paper_2512_08478_amd import _lib as L
    from paper_2512_08478_amd import scenes as S
    from paper_2512_08478_amd.batch import BatchRenderer, autotune, plain_views
    from paper_2512_08478_amd.render import GaussianParams, Renderer

    assets, cams = S.batched_scenes()
    p = GaussianParams.concat([GaussianParams.from_scene(a) for a in assets])
    targets = [torch.from_numpy(S.random_target(100 + v, c.height, c.width)).cuda()
               for v, c in enumerate(cams)]
    log = (lambda m: print(m, file=sys.stderr, flush=True))
    best, tune_ms, tune_n = autotune(p, cams, targets, reps=2, log=log)
    br = BatchRenderer(p, cams, targets, best)
    cap = br.plan()
    br.capture()
    for _ in range(args.warmup):
        br.replay(check=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        br.replay(check=False)
    torch.cuda.synchronize()
    ms_per_step = (time.perf_counter() - t0) * 1e3 / args.steps
    br._check_flags()
    imgs = [im.clone() for im in br.images]
    grads = [g.clone() for g in br.grads]

    # the plain path: view by view, one count readback per view
    R = Renderer(best)
    plain_views(p, cams, targets, renderer=R)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 2
    for _ in range(reps):
        pimgs, pgrads = plain_views(p, cams, targets, renderer=R)
    torch.cuda.synchronize()
    plain_ms = (time.perf_counter() - t0) * 1e3 / reps
    equal = all(torch.equal(a, b) for a, b in zip(imgs, pimgs))
    grad_rel = max(float((a - b).norm() / b.norm().clamp_min(1e-30)) for a, b in zip(grads, pgrads))

    # per-kernel times of one eager batch (HIP events on the library's stream)
    br.run_eager()
    torch.cuda.synchronize()
    L.trace_enable(True)
    br.run_eager()
    tr = L.trace_read(4096)
    L.trace_enable(False)
    kern_ms, kern_n = {}, {}
    for lab, ms in tr:
        kern_ms[lab] = kern_ms.get(lab, 0.0) + ms
        kern_n[lab] = kern_n.get(lab, 0) + 1
    blends = 0
    for cam in cams:
        fr = R.forward(p, cam)
        nb = torch.empty((cam.height, cam.width), dtype=torch.int32, device="cuda")
        R.rasterize(fr.splats, fr.values, fr.ranges, cam, n_blend=nb)
        blends += int(nb.sum(dtype=torch.int64).item())
    flops = {"raster": blends * FLOPS_PER_BLEND, "raster_bwd": blends * 2 * FLOPS_PER_BLEND}
    dom = max(kern_ms, key=lambda k: kern_ms[k])
    stages = {k: {"ms_per_batch": round(v, 4), "launches": kern_n[k]} for k, v in kern_ms.items()}
    roofline = {"kernel": dom, "ms_per_launch": round(kern_ms[dom] / kern_n[dom], 5), "traffic": None}
    if dom in flops:
        tf = flops[dom] / (kern_ms[dom] * 1e-3) / 1e12
        roofline.update(bound="alu", achieved=round(tf, 3), peak=FP32_VECTOR_PEAK_TFLOPS,
                        unit="TFLOP/s", frac=round(tf / FP32_VECTOR_PEAK_TFLOPS, 4),
                        algo_flops_per_batch=int(flops[dom]), blended_pairs=blends)
    n_views = len(cams)
    out = {
        "metric": METRIC,
        "value": round(n_views * 1000.0 / ms_per_step, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["batched"], "n_gaussians": p.n,
                   "asset_sizes": [a.n for a in assets], "n_views": n_views,
                   "pixels": int(sum(c.width * c.height for c in cams)),
                   "instances_planned": cap, "autotuned": best},
        "plain_frames_per_s": round(n_views * 1000.0 / plain_ms, 2),
        "graph_speedup_vs_plain": round(plain_ms / ms_per_step, 3),
        "images_bitwise_equal_to_plain": bool(equal),
        "grads_rel_l2_vs_plain": grad_rel,
        "autotune": {"best_ms_per_batch": round(tune_ms, 4), "candidates_timed": tune_n},
        "launches_per_batch": sum(kern_n.values()),
        "stages": stages,
        "roofline": roofline,
    }
    if full and not args.no_cpu_baseline:
        cb = cpu_baseline(assets, cams[0], dict(tile_w=16, tile_h=16))
        cb["sample"] = "view 0 of the batch (all assets): " + cb["sample"]
        out["cpu_baseline"] = cb
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            return next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        return "unknown CPU"


def oracle_frame_stages(sc, cam, settings, pixels, packed=False, mesh=None, skin=None):
    """Times of the FP64 oracle's stages for one frame, in seconds: preprocess
    (Eq. 1 + colour + culls), keygen (the (tile, depth) key list),
    std::stable_sort of the keys, and the tiled composite (Eq. 3) of
    `pixels`.  The oracle as it stands; no tuning."""
    import oracle
    pk = oracle.prepack(sc) if packed else None
    t = [time.perf_counter()]
    if pk is not None:
        if skin is not None:
            pk = oracle.lbs_deform(pk, *skin)
        rec = oracle.preprocess_packed(pk, cam, settings)
    elif isinstance(sc, (list, tuple)):
        rec = oracle.preprocess_many(sc, cam, settings)
    else:
        rec = oracle.preprocess(sc, cam, settings)
    t.append(time.perf_counter())
    k, v = oracle.keys(rec, cam, settings)
    t.append(time.perf_counter())
    oracle.stable_sort_pairs(k, v)
    t.append(time.perf_counter())
    oracle.render_pixels(rec, cam, pixels, settings, mesh=mesh, tiled=True)
    t.append(time.perf_counter())
    return {"preprocess": t[1] - t[0], "keygen": t[2] - t[1], "stable_sort": t[3] - t[2],
            "composite": t[4] - t[3], "keys": int(k.size)}


def cpu_baseline(sc, cam, settings, packed=False, mesh=None, skin=None, one_core_rows=8):
    """The FP64 oracle, as it stands, timed by stage (preprocess, keygen,
    std::stable_sort, tiled composite) on all host threads over the whole
    frame, and on one thread with the composite over every `one_core_rows`-th
    tile row (scaled to the frame; the other stages whole).  `value` is the
    all-threads frame rate."""
    import numpy as np
    import oracle
    n_all = oracle.num_threads()
    pix = oracle.all_pixels(cam)
    st = dict(settings)
    allc = oracle_frame_stages(sc, cam, st, pix, packed, mesh, skin)
    th = st.get("tile_h", 16)
    rows = (pix[:, 1] // th) % one_core_rows == 0
    oracle.set_num_threads(1)
    try:
        one = oracle_frame_stages(sc, cam, st, pix[rows], packed, mesh, skin)
    finally:
        oracle.set_num_threads(n_all)
    one["composite"] *= pix.shape[0] / max(1, int(rows.sum()))
    frame_all = sum(allc[k] for k in ("preprocess", "keygen", "stable_sort", "composite"))
    frame_one = sum(one[k] for k in ("preprocess", "keygen", "stable_sort", "composite"))
    r = lambda d: {k: (round(v * 1e3, 2) if k != "keys" else v) for k, v in d.items()}
    return {"value": round(1.0 / frame_all, 4), "unit": "frames/s", "cores": n_all, "kind": "oracle",
            "cpu": cpu_model(),
            "stages_ms_all_threads": r(allc), "stages_ms_one_thread": r(one),
            "frames_per_s_one_thread": round(1.0 / frame_one, 5),
            "sort_mkeys_per_s_one_thread": round(one["keys"] / one["stable_sort"] / 1e6, 2),
            "sample": f"tiled FP64 oracle, forward only, by stage (preprocess, keygen, "
                      f"std::stable_sort of the {allc['keys']} keys, tiled composite): the whole "
                      f"{cam.width}x{cam.height} frame on {n_all} threads of {cpu_model()}; on one "
                      f"thread the composite of every {one_core_rows}th tile row ("
                      f"{int(rows.sum())} pixels) scaled to the frame"}


if __name__ == "__main__":
    main()
