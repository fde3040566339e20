"""Batched multi-view, multi-asset forward + backward in one HIP graph.

Every view renders all assets of the scene with one global depth order
(Algorithm 1 feeds every model's Gaussians to one sort), then runs the
hand-written backward; gradients of all views add up in one set of
parameter-gradient buffers.  Each view's compositing backward leaves a
48-byte 2-D gradient record per Gaussian; every 8 views, one multi-view
chain-rule pass turns those records into input gradients, reading and
writing each Gaussian's parameter gradient once for the 8 views instead of
once per view.  `BatchRenderer.capture()` records the whole batch -- every
view's preprocess, sort, compositing, loss gradient and backward -- into
one HIP graph (through torch's graph capture, on the library's stream), so
a step is a single graph launch with no host synchronisation.  Instance capacities are planned beforehand from one
counting pass; a view that exceeds its capacity raises its overflow flag,
which `replay()` checks.

Views of one 8-view chunk can run on several HIP streams at once (one
Renderer, with its own buffers, per stream; the chunk's chain rule joins
them): a view's sort is a chain of small latency-bound kernels, which
another view's compositing overlaps.  Captured, the streams become
parallel branches of the graph.

`autotune()` picks the tile shape and the radix digit width (and sort mode,
compositing order and stream count) by timing whole batches.  Images do
not depend on these choices (every tile shape composites the same pairs in
the same order with the same arithmetic), so tuning never changes results.
"""
from __future__ import annotations

import contextlib
import time

import torch

from . import _lib as L
from .render import GaussianParams, Renderer, depth_range_bits

TILE_SHAPES = ((16, 16), (16, 8), (32, 8), (8, 8), (32, 16), (32, 32), (64, 16), (64, 32))
RADIX_BITS = (8, 7, 6)
SORT_MODES = (0, 1)
RASTER_ORDERS = (1, 0)
STREAM_COUNTS = (1, 2, 4)


def l1_grad(image, target):
    """dL/dRGBA of L = mean |RGB - target| over (H, W, 3); alpha gets none."""
    H, W = target.shape[:2]
    g = torch.zeros((H, W, 4), dtype=torch.float32, device=image.device)
    g[..., :3] = torch.sign(image[..., :3] - target) / (3.0 * H * W)
    return g


class BatchRenderer:
    """Views x assets forward + backward with fixed per-view capacities."""

    def __init__(self, params: GaussianParams, cams, targets, settings=None, headroom=1.10,
                 device="cuda", streams=None):
        if len(cams) != len(targets):
            raise ValueError("one target image per view")
        settings = dict(settings or {})
        nst = int(settings.pop("streams", 1) if streams is None else streams)
        settings.pop("streams", None)
        if nst < 1:
            raise ValueError("streams must be >= 1")
        self.p = params
        self.cams = list(cams)
        self.targets = [t.to(device=device, dtype=torch.float32).contiguous() for t in targets]
        # one Renderer (its own reusable buffers) per stream; streams at the
        # default priority
        self.Rs = [Renderer(settings, device) for _ in range(nst)]
        self.R = self.Rs[0]
        self.streams = [torch.cuda.Stream(device=device) for _ in range(nst)] if nst > 1 else []
        self.headroom = headroom
        self.capacity = None
        self.depth_bits = None   # per view, from plan() (None: all 32 bits)
        self.graph = None
        self.images = None
        self.grads = tuple(torch.zeros_like(t) for t in params.tensors())
        self.flags = torch.zeros(len(self.cams), dtype=torch.int32, device=device)
        self.chunk = L.BWD_VIEWS_PER_LAUNCH
        self.g2d = [torch.empty((params.n, L.GRAD2D_STRIDE), dtype=torch.float32, device=device)
                    for _ in range(min(self.chunk, len(self.cams)))]

    @property
    def settings(self):
        s = self.R.settings
        return dict(tile_w=s.tile_w, tile_h=s.tile_h, radix_bits=s.radix_bits,
                    sort_mode=s.sort_mode, raster_order=s.raster_order, streams=len(self.Rs))

    def plan(self):
        """Per-view instance capacities and depth key bits from one counting
        pass (syncs once per view)."""
        caps, bits = [], []
        for cam in self.cams:
            _, _, _, counts = self.R.preprocess(self.p, cam)
            cn = [int(x) & 0xFFFFFFFF for x in counts[:4].tolist()]
            caps.append(cn[0])
            bits.append(depth_range_bits(cn))
        self.capacity = [max(256, int(c * self.headroom)) for c in caps]
        self.depth_bits = bits
        return list(caps)

    def _enqueue(self):
        """All views' forward + backward, forked from and joined back into
        the current stream per chunk; no host sync."""
        images = []
        main = torch.cuda.current_stream()
        nst = len(self.Rs)
        for v0 in range(0, len(self.cams), self.chunk):
            cams = self.cams[v0:v0 + self.chunk]
            for st in self.streams:
                st.wait_stream(main)
            for k, cam in enumerate(cams):
                v = v0 + k
                R = self.Rs[k % nst]
                ctx = torch.cuda.stream(self.streams[k % nst]) if self.streams else contextlib.nullcontext()
                with ctx:
                    fr = R.forward(self.p, cam, capacity=self.capacity[v],
                                   depth_bits=self.depth_bits[v] if self.depth_bits else None)
                    self.flags[v:v + 1].copy_(fr.flag)
                    g = l1_grad(fr.image, self.targets[v])
                    R.backward_2d(self.p, cam, fr, g, self.g2d[k])
                if self.streams:
                    fr.image.record_stream(main)
                images.append(fr.image)
            for st in self.streams:
                main.wait_stream(st)
            self.R.backward_views(self.p, cams, self.g2d[:len(cams)], out=self.grads,
                                  accumulate=v0 > 0)
        return images

    def run_eager(self):
        """One batch without a graph (sizes every reusable buffer)."""
        if self.capacity is None:
            self.plan()
        self.images = self._enqueue()
        return self.images

    def capture(self):
        """Record the whole batch into one HIP graph."""
        if self.capacity is None:
            self.plan()
        # an eager pass first: grows every reusable buffer to its final size,
        # so nothing is reallocated while capturing
        self.run_eager()
        torch.cuda.synchronize()
        self._check_flags()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.images = self._enqueue()
        self.graph = g
        return g

    def replay(self, check=True):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
        if check:
            torch.cuda.synchronize()
            self._check_flags()
        return self.images

    def _check_flags(self):
        bad = torch.nonzero(self.flags & 1).flatten().tolist()
        if bad:
            raise RuntimeError(f"instance capacity exceeded in views {bad}; plan() again "
                               f"with more headroom")
        bad = torch.nonzero(self.flags & 2).flatten().tolist()
        if bad:
            raise RuntimeError(f"depth key range wider than planned in views {bad}; plan() again")


def plain_views(params: GaussianParams, cams, targets, settings=None, renderer=None):
    """The plain path: view by view, each reading its instance count back
    (one sync) before sorting, gradients accumulated over views."""
    R = renderer or Renderer(settings)
    grads = tuple(torch.zeros_like(t) for t in params.tensors())
    images = []
    for v, cam in enumerate(cams):
        fr = R.forward(params, cam)
        g = l1_grad(fr.image, targets[v].to(device=fr.image.device, dtype=torch.float32))
        R.backward(params, cam, fr, g, out=grads, accumulate=v > 0)
        images.append(fr.image.clone())
    return images, grads


def _time_batch(br: BatchRenderer, reps: int):
    br.run_eager()
    torch.cuda.synchronize()
    br._check_flags()
    t0 = time.perf_counter()
    for _ in range(reps):
        br.run_eager()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def autotune(params: GaussianParams, cams, targets, base_settings=None, reps=2,
             tiles=TILE_SHAPES, bits=RADIX_BITS, modes=SORT_MODES, orders=RASTER_ORDERS,
             streams=STREAM_COUNTS, log=None):
    """Coordinate search: the number of streams (at the first tile shape,
    8-bit digits, mode 0), then tile shape, digit width, sort mode and the
    compositing order of the tiles, each by the wall time of whole eager
    batches.  Streams come first because they change what the other
    settings trade against (an overlapped sort costs less).  Returns
    (settings dict, [(settings, seconds)])."""
    base = dict(base_settings or {})
    table = []

    def measure(over):
        s = dict(base, **over)
        br = BatchRenderer(params, cams, targets, s)
        br.plan()
        t = _time_batch(br, reps)
        table.append((dict(over), t))
        if log:
            log(f"autotune {over}: {t * 1e3:.2f} ms per batch")
        del br
        return t

    best = dict(tile_w=tiles[0][0], tile_h=tiles[0][1], radix_bits=bits[0], sort_mode=modes[0],
                raster_order=orders[0], streams=streams[0])
    best_t = None
    for n in streams:
        t = measure(dict(best, streams=n))
        if best_t is None or t < best_t:
            best_t, best = t, dict(best, streams=n)
    for tw, th in tiles[1:]:
        t = measure(dict(best, tile_w=tw, tile_h=th))
        if t < best_t:
            best_t, best = t, dict(best, tile_w=tw, tile_h=th)
    for b in bits[1:]:
        t = measure(dict(best, radix_bits=b))
        if t < best_t:
            best_t, best = t, dict(best, radix_bits=b)
    for m in modes[1:]:
        t = measure(dict(best, sort_mode=m))
        if t < best_t:
            best_t, best = t, dict(best, sort_mode=m)
    for o in orders[1:]:
        t = measure(dict(best, raster_order=o))
        if t < best_t:
            best_t, best = t, dict(best, raster_order=o)
    return dict(base, **best), table


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
