"""Torch-facing wrapper of libgs: device buffers, streams and autograd.

PyTorch supplies device memory (tensor data pointers) and the current HIP
stream; every step of the render path runs in libgs's kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

__all__ = ["GaussianParams", "PackedParams", "Renderer", "Frame", "render", "GsRender",
           "mesh_buffers"]


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class GaussianParams:
    """Raw Gaussian parameters on the GPU (float32, contiguous)."""
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    opacity_logits: torch.Tensor
    sh: torch.Tensor
    sh_degree: int
    model: object = None  # 3x4 similarity transform or None
    # several assets concatenated: [(offset, count, model or None)] (None = one asset)
    assets: object = None

    @property
    def n(self):
        return int(self.means.shape[0])

    @staticmethod
    def concat(parts):
        """One parameter set holding several assets (each GaussianParams with
        its own model transform), for one global sort per view."""
        degs = {q.sh_degree for q in parts}
        if len(degs) != 1:
            raise ValueError("all assets must share one SH degree")
        table, off = [], 0
        for q in parts:
            table.append((off, q.n, q.model))
            off += q.n
        cat = lambda name: torch.cat([getattr(q, name) for q in parts]).contiguous()
        return GaussianParams(cat("means"), cat("log_scales"), cat("quats"),
                              cat("opacity_logits"), cat("sh"), degs.pop(), None, table)

    @staticmethod
    def from_scene(scene, device="cuda", requires_grad=False):
        f = lambda a: torch.as_tensor(a, dtype=torch.float32).to(device).contiguous().requires_grad_(requires_grad)
        return GaussianParams(f(scene.means), f(scene.log_scales), f(scene.quats),
                              f(scene.opacity_logits), f(scene.sh), int(scene.sh_degree),
                              None if scene.model is None else [list(map(float, r)) for r in scene.model])

    def tensors(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logits, self.sh)


@dataclass
class PackedParams:
    """The FP16 pre-packed form (int16 tensors holding binary16 bits):
    posop (n, 4) = mean, opacity; cov (n, 6) = upper covariance triangle;
    sh16 (n, S) = SH coefficients padded to S halves.  Forward only."""
    posop: torch.Tensor
    cov: torch.Tensor
    sh16: torch.Tensor
    sh_degree: int
    model: object = None
    assets: object = None

    @property
    def n(self):
        return int(self.posop.shape[0])

    def halves(self):
        """(posop, cov, sh16) viewed as float16."""
        return tuple(t.view(torch.float16) for t in (self.posop, self.cov, self.sh16))


@dataclass
class Frame:
    """Forward outputs plus the state the backward pass re-walks."""
    image: torch.Tensor      # (H, W, 4)
    T_final: torch.Tensor    # (H, W)
    last: torch.Tensor       # (H, W) int32 (u32 on the device)
    splats: torch.Tensor     # (n*48,) uint8
    depth_keys: torch.Tensor  # (n,) int32 (u32): depth sort keys
    rects: torch.Tensor      # (2n,) int32 (u32 pairs): tile rect per Gaussian
    counts: torch.Tensor     # (4,) int32 (u32), device: instances, visible, depth key range
    keys: torch.Tensor       # (capacity,) int64 (u64) or None
    values: torch.Tensor     # (capacity,) int32 (u32)
    ranges: torch.Tensor     # (2*tiles,) int32 (u32)
    flag: torch.Tensor       # (1,) int32: bit 0 = capacity exceeded, bit 1 = depth range
    capacity: int
    mesh: object = None      # the mesh prepass composited with (see Renderer.forward)
    depth_bits: int = 0      # depth key bits the sort ordered (0: all 32)


def mesh_buffers(mesh, cam, device="cuda"):
    """A mesh prepass {"depth": (H, W), "rgb": (H, W, 3) or None} (numpy or
    torch) as contiguous float32 device tensors of the camera's size."""
    H, W = cam.height, cam.width
    out = {}
    for k, shape in (("depth", (H, W)), ("rgb", (H, W, 3))):
        v = mesh.get(k)
        if v is None:
            out[k] = None
            continue
        t = torch.as_tensor(v).to(device=device, dtype=torch.float32).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError(f"mesh {k} must have shape {shape}, got {tuple(t.shape)}")
        out[k] = t
    return out


def depth_range_bits(counts, headroom_bits=0):
    """Depth key bits the sort must order for gs_preprocess counts
    (instances, visible, smallest and largest visible depth key): the bit
    length of the key range (at least 1), plus `headroom_bits` for later
    frames of a moving camera, at most 32; 0 (all bits) when nothing is
    visible."""
    if int(counts[1]) == 0:
        return 0
    r = (int(counts[3]) & 0xFFFFFFFF) - (int(counts[2]) & 0xFFFFFFFF)
    return min(32, max(1, r.bit_length()) + int(headroom_bits))


class Renderer:
    """Holds settings and reusable workspaces for one device."""

    def __init__(self, settings=None, device="cuda"):
        self.settings = L.default_settings(**(settings or {}))
        self.last_depth_bits = self.settings.depth_bits
        self.device = torch.device(device)
        self._bufs = {}
        L.load()

    # ------------------------------------------------------------ buffers
    def _buf(self, name, nbytes, reuse=True):
        nbytes = (max(int(nbytes), 256) + 255) // 256 * 256
        if not reuse:
            return torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        b = self._bufs.get(name)
        if b is None or b.numel() < nbytes:
            grown = (int(nbytes * 1.25) + 255) // 256 * 256
            b = torch.empty(grown, dtype=torch.uint8, device=self.device)
            self._bufs[name] = b
        return b

    def tiles(self, cam):
        s = self.settings
        return ((cam.width + s.tile_w - 1) // s.tile_w) * ((cam.height + s.tile_h - 1) // s.tile_h)

    # ------------------------------------------------------------ stages
    def prepack(self, p: GaussianParams) -> PackedParams:
        """The FP16 pre-pack of every Gaussian (once per asset set)."""
        lib = L.load()
        n, S = p.n, L.packed_sh_stride(p.sh_degree)
        dev = p.means.device
        posop = torch.empty((n, 4), dtype=torch.int16, device=dev)
        cov = torch.empty((n, 6), dtype=torch.int16, device=dev)
        sh16 = torch.empty((n, S), dtype=torch.int16, device=dev)
        st = lib.gs_prepack(n, *[_p(t) for t in p.tensors()], p.sh_degree, _p(posop), _p(cov),
                            _p(sh16), _stream())
        L.check(st, "gs_prepack")
        return PackedParams(posop, cov, sh16, p.sh_degree, p.model, p.assets)

    def lbs_deform(self, canon: PackedParams, joint_idx, joint_w, joints, out=None) -> PackedParams:
        """Linear blend skinning of the packed canonical Gaussians (the avatar
        pre-decoder): joint_idx (n, 4) uint8, joint_w (n, 4) float32, joints
        (K, 3, 4) float32 device tensors.  Returns the deformed PackedParams
        (new posop / cov, or those of `out`; SH shared with `canon`)."""
        lib = L.load()
        n = canon.n
        if out is None:
            out = PackedParams(torch.empty_like(canon.posop), torch.empty_like(canon.cov),
                               canon.sh16, canon.sh_degree, canon.model, canon.assets)
        idx = joint_idx.to(torch.uint8).contiguous()
        w = joint_w.to(torch.float32).contiguous()
        M = joints.to(torch.float32).contiguous()
        if idx.shape != (n, 4) or w.shape != (n, 4):
            raise ValueError("joint_idx and joint_w must be (n, 4)")
        st = lib.gs_lbs_deform(n, _p(canon.posop), _p(canon.cov), _p(idx), _p(w),
                               int(M.numel() // 12), _p(M), _p(out.posop), _p(out.cov), _stream())
        L.check(st, "gs_lbs_deform")
        return out

    def preprocess(self, p, cam, reuse=True):
        """Eq. 1 for every Gaussian of `p` (GaussianParams, or PackedParams
        for the pre-packed path): (splats, depth keys, tile rects, counts)."""
        lib = L.load()
        c, s = L.make_camera(cam), self.settings
        n = p.n
        splats = self._buf("splats", n * L.SPLAT_BYTES, reuse)[:n * L.SPLAT_BYTES]
        dkeys = self._buf("depth_keys", n * 4, reuse).view(torch.int32)[:n]
        rects = self._buf("rects", n * 8, reuse).view(torch.int32)[:2 * n]
        counts = self._buf("counts", 16, reuse).view(torch.int32)[:4]
        ws_bytes = lib.gs_workspace_size(L.GS_STAGE_PREPROCESS, n, 0, ctypes.byref(c), ctypes.byref(s))
        ws = self._buf("ws_pre", ws_bytes, reuse)
        if isinstance(p, PackedParams):
            table = p.assets if p.assets is not None else [(0, n, p.model)]
            tab, _keep = L.asset_table(table)
            st = lib.gs_preprocess_packed(len(table), tab, n, _p(p.posop), _p(p.cov),
                                          _p(p.sh16), p.sh_degree, ctypes.byref(c), ctypes.byref(s),
                                          _p(splats), _p(dkeys), _p(rects), _p(counts), _p(ws),
                                          ws.numel(), _stream())
            L.check(st, "gs_preprocess_packed")
        elif p.assets is not None:
            tab, _keep = L.asset_table(p.assets)
            st = lib.gs_preprocess_assets(len(p.assets), tab, n, *[_p(t) for t in p.tensors()],
                                          p.sh_degree, ctypes.byref(c), ctypes.byref(s), _p(splats),
                                          _p(dkeys), _p(rects), _p(counts), _p(ws), ws.numel(),
                                          _stream())
            L.check(st, "gs_preprocess_assets")
        else:
            st = lib.gs_preprocess(n, *[_p(t) for t in p.tensors()], p.sh_degree,
                                   L.model_array(p.model), ctypes.byref(c), ctypes.byref(s),
                                   _p(splats), _p(dkeys), _p(rects), _p(counts), _p(ws), ws.numel(),
                                   _stream())
            L.check(st, "gs_preprocess")
        return splats, dkeys, rects, counts

    def sort(self, n, splats, dkeys, rects, counts, cam, capacity=None, reuse=True,
             want_keys=False, depth_bits=None):
        """capacity=None reads the counts back (one sync): the instance
        count sizes the buffers, and the visible depth key range sets the
        depth bits to sort unless `depth_bits` is given (otherwise the
        settings' depth_bits)."""
        lib = L.load()
        c = L.make_camera(cam)
        if capacity is None:
            cn = [int(x) & 0xFFFFFFFF for x in counts[:4].tolist()]
            capacity = cn[0]
            if depth_bits is None:
                depth_bits = depth_range_bits(cn)
        capacity = int(capacity)
        s = self.settings
        if depth_bits is not None and int(depth_bits) != s.depth_bits:
            s = L.GsSettings.from_buffer_copy(s)
            s.depth_bits = int(depth_bits)
        keys = self._buf("keys", capacity * 8, reuse).view(torch.int64)[:capacity] if want_keys else None
        values = self._buf("values", capacity * 4, reuse).view(torch.int32)[:capacity]
        # [start, end) per tile, then the compositing order of the tiles
        ranges = self._buf("ranges", self.tiles(cam) * 12, reuse).view(torch.int32)[:3 * self.tiles(cam)]
        flag = self._buf("flag", 4, reuse).view(torch.int32)[:1]
        ws_bytes = lib.gs_workspace_size(L.GS_STAGE_SORT, n, capacity, ctypes.byref(c), ctypes.byref(s))
        if ws_bytes == 0:
            raise L.GsError(L.GS_ERR_INVALID_ARGUMENT, "gs_workspace_size(sort)")
        ws = self._buf("ws_sort", ws_bytes)
        st = lib.gs_sort(n, _p(splats), _p(dkeys), _p(rects), _p(counts), ctypes.byref(c),
                         ctypes.byref(s),
                         capacity, _p(keys), _p(values), _p(ranges), _p(flag), _p(ws), ws.numel(),
                         _stream())
        L.check(st, "gs_sort")
        self.last_depth_bits = s.depth_bits
        return keys, values, ranges, flag, capacity

    def sort_pairs32(self, keys, values=None, key_bits=32, want_keys=False):
        """Stable sort of 32-bit keys (int32 tensor holding u32 bit patterns)
        with u32 payloads (values=None: 0..n-1).  Returns (sorted keys or
        None, sorted values)."""
        lib = L.load()
        s = self.settings
        n = int(keys.numel())
        kout = self._buf("s32_keys", n * 4).view(torch.int32)[:n] if want_keys else None
        vout = self._buf("s32_vals", n * 4).view(torch.int32)[:n]
        ws_bytes = lib.gs_workspace_size(L.GS_STAGE_SORT_PAIRS, 0, n, None, ctypes.byref(s))
        ws = self._buf("ws_s32", ws_bytes)
        st = lib.gs_sort_pairs32(n, _p(keys), _p(values), key_bits, _p(kout), _p(vout),
                                 ctypes.byref(s), _p(ws), ws.numel(), _stream())
        L.check(st, "gs_sort_pairs32")
        return kout, vout

    def rasterize(self, splats, values, ranges, cam, n_blend=None, mesh=None):
        """Eqs. 2-3.  `n_blend`, if given, is an int32 (H, W) tensor that
        receives the number of splats blended into each pixel.  `mesh`
        (see mesh_buffers) composites with a mesh prepass."""
        lib = L.load()
        c, s = L.make_camera(cam), self.settings
        H, W = cam.height, cam.width
        image = torch.empty((H, W, 4), dtype=torch.float32, device=self.device)
        T = torch.empty((H, W), dtype=torch.float32, device=self.device)
        last = torch.empty((H, W), dtype=torch.int32, device=self.device)
        if n_blend is not None:
            assert n_blend.shape == (H, W) and n_blend.dtype == torch.int32 and n_blend.is_contiguous()
        nb = _p(n_blend) if n_blend is not None else None
        if mesh is not None:
            md, mr = mesh.get("depth"), mesh.get("rgb")
            st = lib.gs_rasterize_mesh(_p(splats), _p(values), _p(ranges), ctypes.byref(c),
                                       ctypes.byref(s), _p(md), _p(mr), _p(image), _p(T),
                                       _p(last), nb, _stream())
            L.check(st, "gs_rasterize_mesh")
        else:
            st = lib.gs_rasterize(_p(splats), _p(values), _p(ranges), ctypes.byref(c),
                                  ctypes.byref(s), _p(image), _p(T), _p(last), nb, _stream())
            L.check(st, "gs_rasterize")
        return image, T, last

    def forward(self, p, cam, capacity=None, reuse=True, want_keys=False, mesh=None,
                depth_bits=None) -> Frame:
        """One frame: preprocess, sort, composite (with a mesh prepass when
        `mesh` is given: {"depth": (H, W) float32 camera-space z, +inf where
        there is no mesh; "rgb": (H, W, 3) float32 or None}, device tensors,
        see mesh_buffers)."""
        if mesh is not None:
            mesh = mesh_buffers(mesh, cam, self.device)
        splats, dkeys, rects, counts = self.preprocess(p, cam, reuse)
        keys, values, ranges, flag, cap = self.sort(p.n, splats, dkeys, rects, counts, cam, capacity,
                                                    reuse, want_keys, depth_bits)
        image, T, last = self.rasterize(splats, values, ranges, cam, mesh=mesh)
        return Frame(image, T, last, splats, dkeys, rects, counts, keys, values, ranges, flag, cap,
                     mesh, self.last_depth_bits)

    def backward(self, p: GaussianParams, cam, fr: Frame, dL_dimage, out=None, accumulate=False):
        if fr.mesh is not None:
            # compositing backward against the mesh colour, then the chain rule
            g2d = self.backward_2d(p, cam, fr, dL_dimage)
            return self.backward_views(p, [cam], [g2d], out=out, accumulate=accumulate)
        lib = L.load()
        c, s = L.make_camera(cam), self.settings
        n = p.n
        if out is None:
            out = tuple(torch.zeros_like(t) for t in p.tensors())
        dL = dL_dimage.to(torch.float32).contiguous()
        ws_bytes = lib.gs_workspace_size(L.GS_STAGE_BACKWARD, n, 0, ctypes.byref(c), ctypes.byref(s))
        ws = self._buf("ws_bwd", ws_bytes)
        if p.assets is not None:
            tab, _keep = L.asset_table(p.assets)
            st = lib.gs_rasterize_backward_assets(
                len(p.assets), tab, n, *[_p(t) for t in p.tensors()], p.sh_degree, ctypes.byref(c),
                ctypes.byref(s), _p(fr.splats), _p(fr.values), _p(fr.ranges), _p(fr.T_final),
                _p(fr.last), _p(dL), *[_p(t) for t in out], int(bool(accumulate)), _p(ws),
                ws.numel(), _stream())
            L.check(st, "gs_rasterize_backward_assets")
        else:
            st = lib.gs_rasterize_backward(
                n, *[_p(t) for t in p.tensors()], p.sh_degree, L.model_array(p.model),
                ctypes.byref(c), ctypes.byref(s), _p(fr.splats), _p(fr.values), _p(fr.ranges),
                _p(fr.T_final), _p(fr.last), _p(dL), *[_p(t) for t in out], int(bool(accumulate)),
                _p(ws), ws.numel(), _stream())
            L.check(st, "gs_rasterize_backward")
        return out


    def backward_2d(self, p: GaussianParams, cam, fr: Frame, dL_dimage, grad2d=None):
        """The compositing backward only: per-Gaussian 2-D gradient records
        (n, 12) float32 of this view, for backward_views."""
        lib = L.load()
        c, s = L.make_camera(cam), self.settings
        n = p.n
        if grad2d is None:
            grad2d = torch.empty((n, L.GRAD2D_STRIDE), dtype=torch.float32, device=self.device)
        dL = dL_dimage.to(torch.float32).contiguous()
        if fr.mesh is not None:
            st = lib.gs_rasterize_backward_2d_mesh(
                _p(fr.splats), _p(fr.values), _p(fr.ranges), ctypes.byref(c), ctypes.byref(s),
                _p(fr.mesh.get("rgb")), _p(fr.T_final), _p(fr.last), _p(dL), n, _p(grad2d),
                _stream())
            L.check(st, "gs_rasterize_backward_2d_mesh")
        else:
            st = lib.gs_rasterize_backward_2d(_p(fr.splats), _p(fr.values), _p(fr.ranges),
                                              ctypes.byref(c), ctypes.byref(s), _p(fr.T_final),
                                              _p(fr.last), _p(dL), n, _p(grad2d), _stream())
            L.check(st, "gs_rasterize_backward_2d")
        return grad2d

    def backward_views(self, p: GaussianParams, cams, grad2ds, out=None, accumulate=False):
        """Input gradients summed over views from their 2-D gradient records."""
        lib = L.load()
        s = self.settings
        n = p.n
        if out is None:
            out = tuple(torch.zeros_like(t) for t in p.tensors())
        cam_arr = (L.GsCamera * len(cams))(*[L.make_camera(c) for c in cams])
        ptrs = (ctypes.c_void_p * len(grad2ds))(*[g.data_ptr() for g in grad2ds])
        assets = p.assets if p.assets is not None else [(0, n, p.model)]
        tab, _keep = L.asset_table(assets)
        st = lib.gs_preprocess_backward_views(
            len(cams), cam_arr, ptrs, len(assets), tab, n, *[_p(t) for t in p.tensors()],
            p.sh_degree, ctypes.byref(s), *[_p(t) for t in out], int(bool(accumulate)), _stream())
        L.check(st, "gs_preprocess_backward_views")
        return out


class GsRender(torch.autograd.Function):
    """image = render(params); backward through libgs's hand-written kernels."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, renderer, cam, sh_degree, model,
                assets=None, mesh=None):
        p = GaussianParams(means.detach(), log_scales.detach(), quats.detach(),
                           opacity_logits.detach(), sh.detach(), sh_degree, model, assets)
        fr = renderer.forward(p, cam, reuse=False, mesh=mesh)
        ctx.renderer, ctx.cam, ctx.p, ctx.frame = renderer, cam, p, fr
        return fr.image

    @staticmethod
    def backward(ctx, grad_image):
        g = ctx.renderer.backward(ctx.p, ctx.cam, ctx.frame, grad_image)
        return (*g, None, None, None, None, None, None)


def render(params: GaussianParams, cam, renderer: Renderer = None, mesh=None):
    """Differentiable render of ``params`` from ``cam``: (H, W, 4) RGBA,
    optionally composited with a mesh prepass (see Renderer.forward)."""
    renderer = renderer or Renderer()
    return GsRender.apply(params.means, params.log_scales, params.quats, params.opacity_logits,
                          params.sh, renderer, cam, params.sh_degree, params.model, params.assets,
                          mesh)
