"""Batched multi-view, multi-asset forward + backward: a marshaller over
the library's batch entry points (gs_batch_create / gs_batch_plan /
gs_batch_capture / gs_batch_launch, gs_autotune).

The library renders every view of a batch in one fixed sequence of
launches on one stream: one preprocess launch over every (view, asset,
Gaussian), one global sort whose tile keys cover every view (Algorithm 1
feeds every model's Gaussians to one sort; here every view's too), one
compositing launch over every view's tiles, then the L1 loss gradient, one
compositing-backward launch and the chain rule.  `BatchRenderer.capture()`
records that sequence into one HIP graph (stream capture inside the
library); a step is one graph launch with no host synchronisation.
Instance capacity and depth key bits are planned once from one counting
pass; a batch that outgrows them raises a bit of the status flag, which
`replay()` checks.

`autotune()` picks tile shape, digit width, sort mode and compositing order
with the library's gs_autotune (a coordinate search over whole batches).
Images do not depend on these choices, so tuning never changes results.
"""
from __future__ import annotations

import ctypes
import time

import torch

from . import _lib as L
from .render import GaussianParams, Renderer

TILE_SHAPES = ((16, 16), (16, 8), (32, 8), (8, 8), (32, 16), (32, 32), (64, 16), (64, 32))
RADIX_BITS = (8, 7, 6)
SORT_MODES = (0, 1)
RASTER_ORDERS = (1, 0, 3, 5, 2, 4)


def l1_grad(image, target):
    """dL/dRGBA of L = mean |RGB - target| over (H, W, 3); alpha gets none."""
    H, W = target.shape[:2]
    g = torch.zeros((H, W, 4), dtype=torch.float32, device=image.device)
    g[..., :3] = torch.sign(image[..., :3] - target) / (3.0 * H * W)
    return g


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class _Desc:
    """A gs_batch_desc and the host buffers it points to."""

    def __init__(self, params: GaussianParams, cams, targets):
        table = params.assets if params.assets is not None else [(0, params.n, params.model)]
        self.cams = (L.GsCamera * len(cams))(*[L.make_camera(c) for c in cams])
        self.assets, self._keep = L.asset_table(table)
        self.targets = targets
        d = L.GsBatchDesc()
        d.n_views = len(cams)
        d.cams = ctypes.cast(self.cams, ctypes.c_void_p)
        d.n_assets = len(table)
        d.assets = ctypes.cast(self.assets, ctypes.c_void_p)
        d.n = params.n
        d.means, d.log_scales, d.quats, d.opacity_logits, d.sh = [t.data_ptr() for t in params.tensors()]
        d.sh_degree = params.sh_degree
        d.targets = targets.data_ptr() if targets is not None else None
        self.desc = d


class BatchRenderer:
    """Views x assets forward (+ L1 backward with targets) as one batch."""

    def __init__(self, params: GaussianParams, cams, targets=None, settings=None, headroom=1.10,
                 device="cuda"):
        if targets is not None and len(cams) != len(targets):
            raise ValueError("one target image per view")
        self.lib = L.load()
        self.p = params
        self.cams = list(cams)
        self.settings = L.default_settings(**(settings or {}))
        self.headroom = headroom
        self.device = device
        tg = None
        if targets is not None:
            tg = torch.cat([t.to(device=device, dtype=torch.float32).reshape(-1) for t in targets])
        self._d = _Desc(params, self.cams, tg)
        h = ctypes.c_void_p()
        L.check(self.lib.gs_batch_create(ctypes.byref(self._d.desc), ctypes.byref(self.settings),
                                         ctypes.byref(h)), "gs_batch_create")
        self.h = h
        self.pixels = int(self.lib.gs_batch_pixels(h))
        self.offsets = [int(self.lib.gs_batch_pixel_offset(h, v)) for v in range(len(self.cams))]
        self.image_buf = torch.empty(self.pixels * 4, dtype=torch.float32, device=device)
        self.images = [self.image_buf[4 * o:4 * (o + c.width * c.height)].view(c.height, c.width, 4)
                       for o, c in zip(self.offsets, self.cams)]
        self.grads = tuple(torch.zeros_like(t) for t in params.tensors())
        self.flag = torch.zeros(1, dtype=torch.int32, device=device)
        self.ws = None
        self.capacity = None
        # the library's launches and captures run on a stream of their own
        # (a graph cannot be captured on the legacy default stream)
        self.stream = torch.cuda.Stream(device=device)
        self.captured = False

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.lib.gs_batch_destroy(h)
            self.h = None

    def _st(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _outs(self):
        g = self.grads if self._d.targets is not None else (None,) * 5
        return [_p(self.image_buf)] + [_p(t) for t in g] + [_p(self.flag)]

    def plan(self):
        """Instance capacity and depth key bits from one counting pass (one
        sync); sizes the workspace."""
        lib = self.lib
        need = lib.gs_batch_workspace_size(self.h, 0)
        ws = self.ws if self.ws is not None and self.ws.numel() >= need else \
            torch.empty(need, dtype=torch.uint8, device=self.device)
        cap = ctypes.c_int64(0)
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(lib.gs_batch_plan(self.h, ctypes.c_float(self.headroom), _p(ws), ws.numel(),
                                  ctypes.byref(cap), self._st()), "gs_batch_plan")
        self.capacity = int(cap.value)
        need = lib.gs_batch_workspace_size(self.h, self.capacity)
        if ws.numel() < need:
            del ws
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        self.ws = ws
        self.captured = False
        return self.capacity

    def run_eager(self):
        """One batch without a graph."""
        if self.capacity is None:
            self.plan()
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(self.lib.gs_batch_run(self.h, _p(self.ws), self.ws.numel(), *self._outs(), self._st()),
                "gs_batch_run")
        torch.cuda.current_stream().wait_stream(self.stream)
        return self.images

    def capture(self):
        """Record the whole batch into one HIP graph (inside the library)."""
        if self.capacity is None:
            self.plan()
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(self.lib.gs_batch_capture(self.h, _p(self.ws), self.ws.numel(), *self._outs(),
                                          self._st()), "gs_batch_capture")
        self.captured = True

    def replay(self, check=True):
        """One launch of the captured batch.  With check=True it waits for
        the stream and raises if the batch outgrew the planned instance
        capacity or depth key bits (parameters changed since plan(); plan()
        again).  With check=False nothing waits: when that happens the
        images and gradients of that step are wrong, and the status flag
        (self.flag, bits 0 and 1) says so."""
        if not self.captured:
            raise RuntimeError("capture() first")
        self.stream.wait_stream(torch.cuda.current_stream())
        L.check(self.lib.gs_batch_launch(self.h, self._st()), "gs_batch_launch")
        torch.cuda.current_stream().wait_stream(self.stream)
        if check:
            torch.cuda.synchronize()
            self._check_flags()
        return self.images

    def _check_flags(self):
        f = int(self.flag.item()) & 0xFFFFFFFF
        if f & 1:
            raise RuntimeError("instance capacity exceeded; plan() again with more headroom")
        if f & 2:
            raise RuntimeError("depth key range wider than planned; plan() again")


def plain_views(params: GaussianParams, cams, targets, settings=None, renderer=None):
    """The plain path: view by view, each reading its instance count back
    (one sync) before sorting, gradients accumulated over views."""
    R = renderer or Renderer(settings)
    grads = tuple(torch.zeros_like(t) for t in params.tensors())
    images = []
    for v, cam in enumerate(cams):
        fr = R.forward(params, cam)
        if targets is not None:
            g = l1_grad(fr.image, targets[v].to(device=fr.image.device, dtype=torch.float32))
            R.backward(params, cam, fr, g, out=grads, accumulate=v > 0)
        images.append(fr.image.clone())
    return images, grads


def autotune(params: GaussianParams, cams, targets=None, base_settings=None, reps=2,
             tiles=TILE_SHAPES, bits=RADIX_BITS, modes=SORT_MODES, orders=RASTER_ORDERS,
             headroom=1.10, log=None):
    """The library's batch autotuner (gs_autotune): a coordinate search over
    tile shape, digit width, sort mode and compositing order from
    `base_settings`, timing `reps` whole batches per candidate.  The
    workspace is sized for the largest candidate (one counting pass per
    tile shape).  Returns (settings dict, best ms per batch, candidates
    timed)."""
    lib = L.load()
    base = dict(base_settings or {})
    base.setdefault("tile_w", tiles[0][0])
    base.setdefault("tile_h", tiles[0][1])
    need = 0
    for tw, th in {(base["tile_w"], base["tile_h"]), *tiles}:
        br = BatchRenderer(params, cams, targets, dict(base, tile_w=tw, tile_h=th), headroom)
        br.plan()
        need = max(need, br.ws.numel())
        del br
    probe = BatchRenderer(params, cams, targets, base, headroom)
    ws = torch.empty(need, dtype=torch.uint8, device=probe.device)
    sp = L.GsAutotuneSpace()
    sp.n_tiles = len(tiles)
    for k, (tw, th) in enumerate(tiles):
        sp.tiles[2 * k], sp.tiles[2 * k + 1] = tw, th
    sp.n_bits = len(bits)
    for k, b in enumerate(bits):
        sp.bits[k] = b
    sp.n_modes = len(modes)
    for k, m in enumerate(modes):
        sp.modes[k] = m
    sp.n_orders = len(orders)
    for k, o in enumerate(orders):
        sp.orders[k] = o
    best = L.GsSettings()
    ms = ctypes.c_float(0)
    nev = ctypes.c_int32(0)
    probe.stream.wait_stream(torch.cuda.current_stream())
    L.check(lib.gs_autotune(ctypes.byref(probe._d.desc), ctypes.byref(probe.settings),
                            ctypes.byref(sp), reps, ctypes.c_float(headroom), _p(ws), ws.numel(),
                            *probe._outs(), ctypes.byref(best), ctypes.byref(ms),
                            ctypes.byref(nev), probe._st()), "gs_autotune")
    torch.cuda.current_stream().wait_stream(probe.stream)
    out = dict(base, tile_w=best.tile_w, tile_h=best.tile_h, radix_bits=best.radix_bits,
               sort_mode=best.sort_mode, raster_order=best.raster_order)
    if log:
        log(f"gs_autotune: {out} at {ms.value:.3f} ms per batch ({nev.value} candidates timed)")
    return out, float(ms.value), int(nev.value)


def autotune_view(params: GaussianParams, cam, backward=False, target=None, reps=3,
                  tiles=TILE_SHAPES, bits=RADIX_BITS, base_settings=None, log=None, mesh=None,
                  orders=RASTER_ORDERS):
    """Tile shape, then digit width, then the tiles' compositing order, for
    one view (forward, or forward +
    backward with an L1 loss against `target`; composited with `mesh` if
    given), by the wall time of `reps` frames each after one warm-up
    frame.  Returns (settings dict, table)."""
    base = dict(base_settings or {})
    table = []

    def measure(over):
        R = Renderer(dict(base, **over))
        fr = R.forward(params, cam, mesh=mesh)
        torch.cuda.synchronize()
        cap, m, db = fr.capacity, fr.mesh, fr.depth_bits

        def frame():
            f = R.forward(params, cam, capacity=cap, mesh=m, depth_bits=db)
            if backward:
                R.backward(params, cam, f, l1_grad(f.image, target))
        frame()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            frame()
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / reps
        table.append((dict(over), t))
        if log:
            log(f"autotune {over}: {t * 1e3:.3f} ms per frame")
        return t

    best = dict(tile_w=tiles[0][0], tile_h=tiles[0][1], radix_bits=bits[0],
                raster_order=orders[0])
    best_t = None
    for tw, th in tiles:
        t = measure(dict(best, tile_w=tw, tile_h=th))
        if best_t is None or t < best_t:
            best_t, best = t, dict(best, tile_w=tw, tile_h=th)
    for b in bits[1:]:
        t = measure(dict(best, radix_bits=b))
        if t < best_t:
            best_t, best = t, dict(best, radix_bits=b)
    for o in orders[1:]:
        t = measure(dict(best, raster_order=o))
        if t < best_t:
            best_t, best = t, dict(best, raster_order=o)
    return dict(base, **best), table
