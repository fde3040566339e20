"""Seeded synthetic inputs: Gaussian scenes, cameras and sort-key sets.

This module generates inputs only.  It holds none of the renderer's
arithmetic (no projection, colour, compositing or key construction), so the
GPU path and the independent CPU oracle can both be fed from it.

Everything is drawn with ``numpy.random.default_rng(seed)`` (PCG64) in float64
in the fixed order means -> log_scales -> quats -> opacity_logits -> sh, and
cast to float32 at the end.  Quaternions are normalised 4-D standard normals,
which makes them uniform on S^3; they are stored in (w, x, y, z) order.

The scene recipes stand in for the 3DGS "bicycle" asset that the paper
times (Section 4.2, Table 1), which is not available here:

* tiny     4,096 Gaussians, means U[-1,1]^3, log-scale N(-3.5,0.5),
           logit N(0,1), SH degree 0 with DC N(0,0.3); 256x256, 60 deg FoV,
           eye at distance 3.
* medium   1,000,000 Gaussians from a 64-cluster mixture (sigma 0.3) in
           [-5,5]^3, log-scale N(-4,0.7), logit N(0,1.5), SH degree 3 with
           DC N(0,0.3) and higher bands N(0,0.05); 1920x1080 on an azimuth
           orbit of radius 8.
* large    6,000,000 Gaussians as medium but in [-20,20]^3; 1920x1080 with
           the eye inside the cloud at (-12,-12,-16) (about 41% culled).
* diff     500,000 Gaussians as medium; 800x800, radius 8.
* fd       64 Gaussians, means U[-1,1]^3, log-scale N(-2,0.3); 32x32.
* batched  a 2M scene plus 8 assets of log-uniform size in [5e4, 1e6],
           each placed by a similarity transform; 32 views of uneven size.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "Camera", "Scene", "look_at", "pinhole_camera", "orbit_camera",
    "tiny_scene", "medium_scene", "large_scene", "diff_scene", "fd_scene",
    "batched_scenes", "random_target", "sort_keys", "SORT_KEY_KINDS",
    "sh_coeff_count",
]


def sh_coeff_count(degree: int) -> int:
    return (degree + 1) * (degree + 1)


@dataclass
class Camera:
    """Pinhole camera.  ``viewmat`` is the 4x4 row-major world->camera
    matrix in OpenCV axes (+x right, +y down, +z forward)."""
    viewmat: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    def as_dict(self):
        return dict(viewmat=self.viewmat.tolist(), fx=self.fx, fy=self.fy,
                    cx=self.cx, cy=self.cy, width=self.width,
                    height=self.height, znear=self.znear)


@dataclass
class Scene:
    """One asset: raw (pre-activation) Gaussian parameters, float32, C order.

    means (N,3), log_scales (N,3), quats (N,4) as (w,x,y,z),
    opacity_logits (N,), sh (N,K,3) with K=(degree+1)^2, coefficient-major
    and RGB innermost.  ``model`` is an optional 3x4 row-major similarity
    transform [s*R | t] placing the asset in the world (None = identity).
    """
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int
    model: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx):
        return Scene(self.means[idx].copy(), self.log_scales[idx].copy(),
                     self.quats[idx].copy(), self.opacity_logits[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree,
                     None if self.model is None else self.model.copy(),
                     dict(self.meta))


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World->camera 4x4 (row-major) with +z towards ``target`` and +y down."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    up = np.asarray(up, np.float64)
    z = target - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, up)
    nx = np.linalg.norm(x)
    if nx < 1e-9:                      # looking along the up axis
        x = np.cross(z, np.array([0.0, 0.0, 1.0]))
        nx = np.linalg.norm(x)
    x /= nx
    y = np.cross(z, x)
    R = np.stack([x, y, z], 0)
    V = np.eye(4)
    V[:3, :3] = R
    V[:3, 3] = -R @ eye
    return V.astype(np.float32)


def pinhole_camera(viewmat, width, height, fov_y_deg=60.0, znear=0.2) -> Camera:
    """Square-pixel pinhole with vertical FoV ``fov_y_deg``, centred
    principal point."""
    f = 0.5 * height / math.tan(math.radians(fov_y_deg) * 0.5)
    return Camera(np.asarray(viewmat, np.float32), float(np.float32(f)),
                  float(np.float32(f)), 0.5 * width, 0.5 * height,
                  int(width), int(height), float(znear))


def orbit_camera(view: int, n_views: int, radius: float, width: int,
                 height: int, fov_y_deg=60.0) -> Camera:
    """View ``view`` of ``n_views`` on a horizontal circle around the origin
    (view 0 sits on -z looking towards +z)."""
    az = 2.0 * math.pi * view / n_views
    eye = (radius * math.sin(az), 0.0, -radius * math.cos(az))
    return pinhole_camera(look_at(eye), width, height, fov_y_deg)


# --------------------------------------------------------------------------
# Gaussian parameter draws
# --------------------------------------------------------------------------

def _quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _cluster_means(rng, n, half_extent, n_clusters=64, sigma=0.3):
    centres = rng.uniform(-half_extent, half_extent, (n_clusters, 3))
    out = np.empty((n, 3))
    filled = 0
    while filled < n:
        need = n - filled
        k = rng.integers(0, n_clusters, need)
        p = centres[k] + sigma * rng.standard_normal((need, 3))
        ok = np.all(np.abs(p) <= half_extent, axis=1)
        p = p[ok]
        out[filled:filled + len(p)] = p
        filled += len(p)
    return out


def _sh(rng, n, degree, dc_sd, hi_sd):
    k = sh_coeff_count(degree)
    sh = np.empty((n, k, 3))
    sh[:, 0, :] = dc_sd * rng.standard_normal((n, 3))
    if k > 1:
        sh[:, 1:, :] = hi_sd * rng.standard_normal((n, k - 1, 3))
    return sh


def _pack(means, log_scales, quats, logits, sh, degree, model=None, **meta):
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f(means), f(log_scales), f(quats), f(logits), f(sh), degree,
                 None if model is None else f(model), dict(meta))


def _clustered(seed, n, half_extent, degree=3, rng=None):
    rng = np.random.default_rng(seed) if rng is None else rng
    means = _cluster_means(rng, n, half_extent)
    log_scales = rng.normal(-4.0, 0.7, (n, 3))
    quats = _quats(rng, n)
    logits = rng.normal(0.0, 1.5, n)
    sh = _sh(rng, n, degree, 0.3, 0.05)
    return means, log_scales, quats, logits, sh


def tiny_scene(seed=0, n=4096):
    """Tiny forward scene and its 256x256 camera."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    log_scales = rng.normal(-3.5, 0.5, (n, 3))
    quats = _quats(rng, n)
    logits = rng.normal(0.0, 1.0, n)
    sh = _sh(rng, n, 0, 0.3, 0.0)
    cam = pinhole_camera(look_at((0.0, 0.0, -3.0)), 256, 256, 60.0)
    return _pack(means, log_scales, quats, logits, sh, 0, name="tiny"), cam


def medium_scene(seed=1, n=1_000_000, view=0, width=1920, height=1080):
    """1M-Gaussian clustered scene and view ``view`` of its 8-view orbit."""
    s = _pack(*_clustered(seed, n, 5.0), 3, name="medium")
    return s, orbit_camera(view, 8, 8.0, width, height)


LARGE_EYE = (-12.0, -12.0, -16.0)


def large_scene(seed=2, n=6_000_000, width=1920, height=1080):
    """6M-Gaussian clustered scene in [-20,20]^3, eye inside the cloud at
    (-12,-12,-16) looking at the origin: about 41% of the Gaussians are
    culled (behind the near plane or with no pixel in their footprint)."""
    s = _pack(*_clustered(seed, n, 20.0), 3, name="large")
    cam = pinhole_camera(look_at(LARGE_EYE), width, height, 60.0)
    return s, cam


def diff_scene(seed=3, n=500_000, size=800):
    """Differentiable scene: 500k Gaussians, 800x800, radius 8."""
    s = _pack(*_clustered(seed, n, 5.0), 3, name="diff")
    return s, orbit_camera(0, 8, 8.0, size, size)


def fd_scene(seed=5, n=64, size=32, degree=3):
    """Finite-difference instance: footprints spanning several pixels."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, (n, 3))
    log_scales = rng.normal(-2.0, 0.3, (n, 3))
    quats = _quats(rng, n)
    logits = rng.normal(0.0, 1.0, n)
    sh = _sh(rng, n, degree, 0.3, 0.05)
    cam = pinhole_camera(look_at((0.0, 0.0, -3.0)), size, size, 60.0)
    return _pack(means, log_scales, quats, logits, sh, degree, name="fd"), cam


def random_target(seed, height, width):
    """Seeded L1 target image, U[0,1]^3, float32 (H,W,3)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, 1.0, (height, width, 3)).astype(np.float32)


def _random_rotation(rng):
    """Haar-uniform rotation: QR of a Gaussian matrix with the sign fix,
    then a column flip if needed so that det = +1."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def batched_scenes(seed=6, scene_n=2_000_000, n_assets=8, n_views=32,
                   size_range=(50_000, 1_000_000), max_wh=(1920, 1080),
                   min_wh=(512, 512), scale=1.0):
    """The batched workload: one scene (identity placement) plus
    ``n_assets`` assets placed by translate U[-10,10]^3 . rotation . scale
    U[0.25,1], and ``n_views`` cameras of uneven size on a sphere of radius
    16.  ``scale`` shrinks every Gaussian count (for small test versions)."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(size_range[0]),
                                       math.log(size_range[1]), n_assets)))
    sizes = np.maximum(1, np.rint(sizes * scale)).astype(np.int64)
    placements = []
    for _ in range(n_assets):
        t = rng.uniform(-10.0, 10.0, 3)
        R = _random_rotation(rng)
        s = rng.uniform(0.25, 1.0)
        placements.append(np.concatenate([s * R, t[:, None]], 1))
    views = []
    for _ in range(n_views):
        w = int(rng.integers(min_wh[0], max_wh[0] + 1))
        h = int(rng.integers(min_wh[1], max_wh[1] + 1))
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        views.append(pinhole_camera(look_at(16.0 * d), w, h, 60.0))
    assets = [_pack(*_clustered(seed * 1000 + 1, max(1, int(round(scene_n * scale))), 5.0),
                    3, name="scene")]
    for k in range(n_assets):
        a = _pack(*_clustered(seed * 1000 + 2 + k, int(sizes[k]), 5.0), 3,
                  model=placements[k], name=f"asset{k}")
        assets.append(a)
    return assets, views


# --------------------------------------------------------------------------
# Sort-key sets for the bit-exact sort contract
# --------------------------------------------------------------------------

SORT_KEY_KINDS = ("random64", "random45", "all_equal", "sorted", "reversed",
                  "two_unique", "tile_runs", "depth_like")


def skinning(means, n_joints=55, influences=4, seed=0):
    """Synthetic linear-blend-skinning data for an avatar-like asset:
    ``n_joints`` joint centres drawn (seeded) among the Gaussians' means;
    each Gaussian is bound to its ``influences`` nearest joints with
    weights proportional to 1 / (distance + 0.05)^2, normalised to sum to
    one in float64.  Returns (centres (K,3) float32, joint indices (N,J)
    uint8, weights (N,J) float32)."""
    if not 1 <= n_joints <= 256:
        raise ValueError("1..256 joints")
    rng = np.random.default_rng(seed)
    means = np.asarray(means, np.float64)
    n = means.shape[0]
    centres = means[rng.choice(n, n_joints, replace=n < n_joints)]
    J = min(influences, n_joints)
    idx = np.zeros((n, influences), np.uint8)
    w = np.zeros((n, influences), np.float64)
    for s0 in range(0, n, 65536):
        d = np.linalg.norm(means[s0:s0 + 65536, None, :] - centres[None], axis=2)
        near = np.argpartition(d, J - 1, axis=1)[:, :J] if J < n_joints else \
            np.tile(np.arange(n_joints), (d.shape[0], 1))
        dn = np.take_along_axis(d, near, 1)
        ww = 1.0 / (dn + 0.05) ** 2
        idx[s0:s0 + 65536, :J] = near
        w[s0:s0 + 65536, :J] = ww / ww.sum(1, keepdims=True)
    return centres.astype(np.float32), idx, w.astype(np.float32)


def joint_pose(centres, seed=0, angle=0.35, shift=0.2):
    """One pose: per joint a rigid motion about its centre c_k, rotation
    by a seeded angle up to ``angle`` radians about a random axis, then a
    shift up to ``shift``: M_k = [R_k | c_k - R_k c_k + d_k], float32
    (K,3,4).  seed=None gives the identity pose."""
    c = np.asarray(centres, np.float64)
    K = c.shape[0]
    M = np.zeros((K, 3, 4), np.float64)
    M[:, :, :3] = np.eye(3)
    if seed is None:
        return M.astype(np.float32)
    rng = np.random.default_rng(seed)
    for k in range(K):
        ax = rng.standard_normal(3)
        ax /= np.linalg.norm(ax)
        th = rng.uniform(-angle, angle)
        Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        R = np.eye(3) + math.sin(th) * Kx + (1 - math.cos(th)) * (Kx @ Kx)
        M[k, :, :3] = R
        M[k, :, 3] = c[k] - R @ c[k] + rng.uniform(-shift, shift, 3)
    return M.astype(np.float32)


def plane_mesh(cam: Camera, normal, offset, seed=0, cell=0.5, occupancy=1.0):
    """A mesh prepass stand-in: the per-pixel camera-space depth and colour
    of the world plane {X : normal . X = offset} seen through `cam` (pixel
    centres at +1/2), as float32 (H,W) depth (+inf where the ray misses the
    plane, or where a cell of the plane is left out) and (H,W,3) colour (a
    seeded random colour per `cell`-sized square of the plane).  With
    occupancy < 1 only that fraction of the cells is present (a wall with
    holes)."""
    rng = np.random.default_rng(seed)
    n = np.asarray(normal, np.float64)
    n = n / np.linalg.norm(n)
    V = np.asarray(cam.viewmat, np.float64).reshape(4, 4)
    Rv, tv = V[:3, :3], V[:3, 3]
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    dc = np.stack([(xs + 0.5 - cam.cx) / cam.fx, (ys + 0.5 - cam.cy) / cam.fy,
                   np.ones(xs.shape)], -1)                       # camera-space ray, z = 1
    nw = Rv @ n                                                  # plane normal in camera space
    h = offset + n @ (Rv.T @ tv)                                 # plane: nw . x_c = h
    den = dc @ nw
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(np.abs(den) > 1e-12, h / den, np.inf)
    z = np.where(z > 0, z, np.inf)
    Xw = (np.where(np.isfinite(z), z, 0.0)[..., None] * dc - tv) @ Rv   # world points
    # two in-plane axes for the cell pattern
    a = np.cross(n, [0.0, 0.0, 1.0] if abs(n[2]) < 0.9 else [1.0, 0.0, 0.0])
    a /= np.linalg.norm(a)
    b = np.cross(n, a)
    ci = np.floor(Xw @ a / cell).astype(np.int64)
    cj = np.floor(Xw @ b / cell).astype(np.int64)
    palette = rng.uniform(0.0, 1.0, (64, 3))
    keep = rng.uniform(0.0, 1.0, 64) < occupancy
    cid = (ci * 7 + cj * 13) % 64
    z = np.where(keep[cid], z, np.inf)
    rgb = np.where(np.isfinite(z)[..., None], palette[cid], 0.0)
    return dict(depth=z.astype(np.float32), rgb=rgb.astype(np.float32))


def sort_keys(kind: str, n: int, seed: int = 0, key_bits: int = 64):
    """Adversarial (keys uint64, values uint32) sets for the radix sort.

    Values are 0..n-1 so the result permutation is visible.  Keys use only
    the low ``key_bits`` bits."""
    rng = np.random.default_rng(seed)
    mask = np.uint64((1 << key_bits) - 1) if key_bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    if kind == "random64":
        k = rng.integers(0, 2**63, n, dtype=np.uint64) * np.uint64(2) + \
            rng.integers(0, 2, n, dtype=np.uint64)
    elif kind == "random45":
        k = rng.integers(0, 2**45, n, dtype=np.uint64)
    elif kind == "all_equal":
        k = np.full(n, 0x123456789A, dtype=np.uint64)
    elif kind == "sorted":
        k = np.sort(rng.integers(0, 2**40, n, dtype=np.uint64))
    elif kind == "reversed":
        k = np.sort(rng.integers(0, 2**40, n, dtype=np.uint64))[::-1].copy()
    elif kind == "two_unique":
        k = np.where(rng.integers(0, 2, n) == 1, np.uint64(7 << 33),
                     np.uint64(3)).astype(np.uint64)
    elif kind == "tile_runs":
        # long runs of one tile id with few distinct depths
        tiles = np.sort(rng.integers(0, 8160, n)).astype(np.uint64)
        depth = rng.integers(0, 16, n).astype(np.uint64) + np.uint64(0x3F000000)
        k = (tiles << np.uint64(32)) | depth
    elif kind == "depth_like":
        tiles = rng.integers(0, 8160, n).astype(np.uint64)
        d = rng.uniform(0.2, 40.0, n).astype(np.float32).view(np.uint32)
        k = (tiles << np.uint64(32)) | d.astype(np.uint64)
    else:
        raise ValueError(kind)
    k = (k & mask).astype(np.uint64)
    v = np.arange(n, dtype=np.uint32)
    return np.ascontiguousarray(k), v
