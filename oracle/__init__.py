"""FP64 CPU oracle for the 3DGS render path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It never imports the GPU library and
the GPU library never imports it; the two share only the seeded input
generator, which holds none of the method's arithmetic.

``gs_oracle.cpp`` (compiled to ``liboracle.so`` with g++, no fast-math)
implements the forward definition: the per-Gaussian projection of Eq. 1,
the SH colour, and the per-pixel compositing of Eqs. 2-3 by brute force in
ascending (depth, index) order, or (``tiled=True``) the same walk over
per-tile candidate lists, exactly equal and fast enough for whole frames;
each pixel's near decisions and the jump they straddle (the tolerance
protocol); plus the (tile, depth) key list and a library stable sort.  ``prepack`` / ``preprocess_packed`` give the FP16
pre-pack of Section 3.4 (one rounding of float64 values to binary16) and
the projection from the packed mean, opacity and upper covariance;
``lbs_deform`` the avatar pre-decoder's linear blend skinning (Section 3.3,
Eqs. 5-6); ``render_pixels(..., mesh=)`` the mesh depth composition of
Section 3.4.  ``grad.py`` gives reference gradients by float64
automatic differentiation of the same definition (Section 3.2: the
formulation is differentiable).

Pins (tests/test_oracle_*.py): closed forms for one isotropic Gaussian on
and off the optical axis, for its largest weight over a tile, for the jump
of every kind of near decision, tiled == brute force, two ordered Gaussians and n coincident Gaussians;
covariance eigen-invariants; the SH basis against SciPy's complex
harmonics and by quadrature; the sort against NumPy's stable argsort and a
brute-force sort; front-to-back against back-to-front compositing; and the
gradients against central finite differences of the C forward; the
covariance-input projection against the raw-parameter one at a SciPy
covariance, and the binary16 rounding against IEEE 754's ties-to-even
cases; mesh composition by walls behind, in front of and between
Gaussians; skinning by the identity pose, a single rigid joint against the
model transform, and closed-form blends of translations and rotations.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# Reading of the constants the paper leaves open (see the header of
# gs_oracle.cpp): 16x16 tiles, eps2d = 0.3 px^2, tau = 1/255,
# alpha_max = 0.99, t_eps = 1e-4, J clamp 1.3x the half-FoV tangent,
# black background.
DEFAULT_SETTINGS = dict(tile_w=16, tile_h=16, eps2d=0.3, tau=1.0 / 255.0,
                        alpha_max=0.99, t_eps=1e-4, clip=1.3,
                        bg=(0.0, 0.0, 0.0))

# record layout (must match the enums in gs_oracle.cpp)
D_MX, D_MY, D_SA, D_SB, D_SC, D_CA, D_CB, D_CC, D_DEPTH = range(9)
D_R, D_G, D_B, D_RR, D_RG, D_RB, D_OPAC, D_C3 = 9, 10, 11, 12, 13, 14, 15, 16
D_QMAX = 22
I_CULL, I_PX0, I_PX1, I_PY0, I_PY1, I_TX0, I_TY0, I_TX1, I_TY1, I_TILES, I_AMBIG = range(11)
C_VISIBLE, C_NEAR, C_INVALID, C_DET, C_OPACITY, C_OFFIMAGE = range(6)


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (OpenMP, -O2, IEEE semantics)."""
    global _lib
    with _lock:
        stale = (not os.path.exists(_LIB)
                 or os.path.getmtime(_LIB) < os.path.getmtime(_SRC))
        if force or stale:
            tmp = _LIB + ".tmp"
            cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fno-fast-math",
                   "-ffp-contract=off", "-shared", "-fPIC", _SRC, "-o", tmp]
            subprocess.run(cmd, check=True)
            os.replace(tmp, _LIB)
            _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.orc_preprocess.argtypes = [I64, P, P, P, P, P, ctypes.c_int, P, P, P, P, P]
        lib.orc_preprocess_f64.argtypes = [I64, P, P, P, P, P, ctypes.c_int, P, P, P, P, P]
        lib.orc_preprocess_cov.argtypes = [I64, P, P, P, P, ctypes.c_int, P, P, P, P, P]
        lib.orc_render_pixels.argtypes = [I64, P, P, P, P, I64, P, P, P, P, P, P, P, P, P]
        lib.orc_render_tiled.argtypes = [I64, P, P, P, P, I64, P, P, P, P, P, P, P, P, P]
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        lib.orc_keys.argtypes = [I64, P, P, ctypes.c_int, P, P]
        lib.orc_count_instances.argtypes = [I64, P]
        lib.orc_count_instances.restype = I64
        lib.orc_pair_max_weight.argtypes = [I64, P, P, P, P, P, P]
        lib.orc_stable_sort_pairs.argtypes = [I64, P, P]
        lib.orc_sh_basis.argtypes = [ctypes.c_int, I64, P, P]
        lib.orc_rec_layout.argtypes = [P]
        lib.orc_num_threads.restype = ctypes.c_int
        lay = np.zeros(2, np.int32)
        lib.orc_rec_layout(lay.ctypes.data)
        assert tuple(lay) == (24, 11), lay
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


def cam_array(cam) -> np.ndarray:
    v = np.asarray(cam.viewmat, np.float64).reshape(16)
    return np.concatenate([v, [cam.fx, cam.fy, cam.cx, cam.cy, cam.width,
                               cam.height, cam.znear]]).astype(np.float64)


def set_array(settings=None) -> np.ndarray:
    s = dict(DEFAULT_SETTINGS)
    if settings:
        s.update(settings)
    return np.array([s["tile_w"], s["tile_h"], s["eps2d"], s["tau"],
                     s["alpha_max"], s["t_eps"], s["clip"], *s["bg"]], np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(k: int) -> None:
    """Number of OpenMP threads the oracle's later calls use."""
    _load().orc_set_num_threads(int(k))


class Records:
    """Per-Gaussian float64 records of one or more concatenated assets."""

    def __init__(self, d: np.ndarray, i: np.ndarray):
        self.d = np.ascontiguousarray(d, np.float64)
        self.i = np.ascontiguousarray(i, np.int32)

    @property
    def n(self):
        return self.d.shape[0]

    @property
    def visible(self):
        return self.i[:, I_CULL] == C_VISIBLE

    def concat(self, other: "Records") -> "Records":
        return Records(np.concatenate([self.d, other.d]), np.concatenate([self.i, other.i]))


def preprocess(scene, cam, settings=None, f64_inputs=False) -> Records:
    """Eq. 1 + colour + culls for every Gaussian of ``scene`` (float64).

    Inputs are read as float32 (the library's type) unless ``f64_inputs``,
    which keeps them in float64 (for finite differences)."""
    lib = _load()
    n = scene.n
    d = np.zeros((n, 24), np.float64)
    iv = np.zeros((n, 11), np.int32)
    dt = np.float64 if f64_inputs else np.float32
    f = lambda a: np.ascontiguousarray(a, dt)
    arrs = [f(scene.means), f(scene.log_scales), f(scene.quats),
            f(scene.opacity_logits), f(scene.sh)]
    model = None if scene.model is None else np.ascontiguousarray(scene.model, np.float64)
    ca, sa = cam_array(cam), set_array(settings)
    fn = lib.orc_preprocess_f64 if f64_inputs else lib.orc_preprocess
    rc = fn(n, *[_p(a) for a in arrs], int(scene.sh_degree), _p(model),
            _p(ca), _p(sa), _p(d), _p(iv))
    if rc != 0:
        raise ValueError("orc_preprocess rejected its arguments")
    return Records(d, iv)


def covariance(scene) -> np.ndarray:
    """Sigma = R(q/|q|) diag(exp(log_s))^2 R^T per Gaussian (float64, (N,3,3))
    from the float32 inputs (Section 3.2; Algorithm 1, CovFromScaleRot)."""
    q = np.asarray(scene.quats, np.float32).astype(np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                  2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                  2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1)
    R = R.reshape(-1, 3, 3)
    s = np.exp(np.asarray(scene.log_scales, np.float32).astype(np.float64))
    M = R * s[:, None, :]
    return M @ np.transpose(M, (0, 2, 1))


def to_fp16(x) -> np.ndarray:
    """One rounding of float64 values to IEEE binary16, to nearest, ties to
    even (NumPy converts from the float64 bits directly)."""
    with np.errstate(over="ignore"):
        return np.asarray(x, np.float64).astype(np.float16)


def prepack(scene) -> dict:
    """The pre-pack of Algorithm 1 / Section 3.4: mean, activated opacity,
    the upper covariance triangle (xx, xy, xz, yy, yz, zz) and the SH
    coefficients, each computed in float64 from the float32 inputs and
    rounded once to binary16."""
    Sig = covariance(scene)
    iu = ([0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2])
    logit = np.asarray(scene.opacity_logits, np.float32).astype(np.float64)
    return dict(means=to_fp16(np.asarray(scene.means, np.float32)),
                opacity=to_fp16(1.0 / (1.0 + np.exp(-logit))),
                cov6=to_fp16(Sig[:, iu[0], iu[1]]),
                sh=to_fp16(np.asarray(scene.sh, np.float32)),
                sh_degree=int(scene.sh_degree), model=scene.model)


def preprocess_packed(packed, cam, settings=None) -> Records:
    """Eq. 1 + colour + culls from pre-packed values (any float dtype; they
    are used exactly, as float64)."""
    lib = _load()
    f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64))
    means, opac = f(packed["means"]), f(packed["opacity"]).reshape(-1)
    cov6, sh = f(packed["cov6"]).reshape(-1, 6), f(packed["sh"])
    n = means.shape[0]
    d = np.zeros((n, 24), np.float64)
    iv = np.zeros((n, 11), np.int32)
    model = packed.get("model")
    model = None if model is None else np.ascontiguousarray(model, np.float64)
    ca, sa = cam_array(cam), set_array(settings)
    rc = lib.orc_preprocess_cov(n, _p(means), _p(opac), _p(cov6), _p(sh), int(packed["sh_degree"]),
                                _p(model), _p(ca), _p(sa), _p(d), _p(iv))
    if rc != 0:
        raise ValueError("orc_preprocess_cov rejected its arguments")
    return Records(d, iv)


def lbs_deform(packed, joint_idx, joint_w, joints, rounded=True) -> dict:
    """Linear blend skinning of pre-packed canonical Gaussians (Section 3.3,
    Eqs. 5-6): T_i = sum_k w_ik M_k = [R_i | t_i], mu_i = R_i mu^_i + t_i,
    Sigma_i = R_i Sigma^_i R_i^T, in float64 from the decoded canonical
    values; with ``rounded`` the deformed mean and covariance are rounded
    once to binary16 (opacity and SH pass through)."""
    mu = np.asarray(packed["means"], np.float64)
    c6 = np.asarray(packed["cov6"], np.float64)
    Sig = np.stack([c6[:, [0, 1, 2]], c6[:, [1, 3, 4]], c6[:, [2, 4, 5]]], 1)
    M = np.asarray(joints, np.float64).reshape(-1, 3, 4)
    w = np.asarray(joint_w, np.float64)
    T = np.einsum("nk,nkij->nij", w, M[np.asarray(joint_idx, np.int64)])
    R, t = T[:, :, :3], T[:, :, 3]
    mu_d = np.einsum("nij,nj->ni", R, mu) + t
    Sig_d = R @ Sig @ np.transpose(R, (0, 2, 1))
    cov6 = Sig_d[:, [0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
    out = dict(packed)
    out["means"] = to_fp16(mu_d) if rounded else mu_d
    out["cov6"] = to_fp16(cov6) if rounded else cov6
    return out


def preprocess_many(scenes, cam, settings=None, f64_inputs=False) -> Records:
    """Records of several assets, concatenated in order (one global list)."""
    recs = None
    for s in scenes:
        r = preprocess(s, cam, settings, f64_inputs)
        recs = r if recs is None else recs.concat(r)
    return recs


def mesh_at(mesh, pix):
    """(depth (P,), rgb (P,3) or None) of a mesh prepass dict
    {depth: (H,W), rgb: (H,W,3) or None} at pixels (P,2) of x, y."""
    if mesh is None:
        return None, None
    pix = np.asarray(pix).reshape(-1, 2)
    md = mesh.get("depth")
    mr = mesh.get("rgb")
    d = None if md is None else np.ascontiguousarray(
        np.asarray(md, np.float64)[pix[:, 1], pix[:, 0]])
    r = None if mr is None else np.ascontiguousarray(
        np.asarray(mr, np.float64)[pix[:, 1], pix[:, 0]].reshape(-1, 3))
    return d, r


def render_pixels(recs: Records, cam, pix, settings=None, mesh=None, tiled=False):
    """Eq. 3 at the given pixels (int array (P,2) of x, y).

    By brute force (every pixel walks every visible Gaussian), or with
    ``tiled`` over per-tile candidate lists, which gives exactly the same
    outputs (pinned by the tests) at a fraction of the cost.
    ``mesh``: optional mesh prepass {depth: (H,W) camera-space z, +inf where
    no mesh; rgb: (H,W,3) or None}: Gaussians deeper than the mesh are
    hidden and the mesh colour replaces the background (Section 3.4).
    Returns dict(rgba (P,4), T (P,), n_blend (P,), margin (P,), flags (P,),
    jump (P,)): ``margin`` is the smallest relative distance of a decision
    to its threshold (capped at 1), ``flags`` marks depth near-ties (1),
    ambiguous culls (2), near mesh-depth tests (4) and any near decision
    (8: a weight within 3e-5 of tau, T within 1e-4 of t_eps, or one of the
    above), and ``jump`` is the largest change of the outputs that taking
    the pixel's near decisions the other way can cause, each re-walked."""
    lib = _load()
    pix = np.ascontiguousarray(pix, np.int32).reshape(-1, 2)
    P = pix.shape[0]
    out = dict(rgba=np.zeros((P, 4)), T=np.zeros(P), n_blend=np.zeros(P, np.int32),
               margin=np.zeros(P), flags=np.zeros(P, np.int32), jump=np.zeros(P))
    ca, sa = cam_array(cam), set_array(settings)
    md, mr = mesh_at(mesh, pix)
    fn = lib.orc_render_tiled if tiled else lib.orc_render_pixels
    fn(recs.n, _p(recs.d), _p(recs.i), _p(ca), _p(sa), P, _p(pix), _p(md), _p(mr),
       _p(out["rgba"]), _p(out["T"]), _p(out["n_blend"]), _p(out["margin"]),
       _p(out["flags"]), _p(out["jump"]))
    return out


def all_pixels(cam) -> np.ndarray:
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    return np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)


def render_image(recs: Records, cam, settings=None, mesh=None, tiled=False):
    """Full image (H,W,4) plus T, n_blend, margin, flags, jump as (H,W) maps."""
    o = render_pixels(recs, cam, all_pixels(cam), settings, mesh, tiled)
    H, W = cam.height, cam.width
    return dict(rgba=o["rgba"].reshape(H, W, 4),
                **{k: o[k].reshape(H, W) for k in ("T", "n_blend", "margin", "flags", "jump")})


def tiles_xy(cam, settings=None):
    s = dict(DEFAULT_SETTINGS)
    if settings:
        s.update(settings)
    return ((cam.width + s["tile_w"] - 1) // s["tile_w"],
            (cam.height + s["tile_h"] - 1) // s["tile_h"])


def keys(recs: Records, cam, settings=None):
    """(tile, depth) keys and Gaussian-index values, Gaussian-major order."""
    lib = _load()
    total = int(lib.orc_count_instances(recs.n, _p(recs.i)))
    k = np.zeros(total, np.uint64)
    v = np.zeros(total, np.uint32)
    tx, _ = tiles_xy(cam, settings)
    lib.orc_keys(recs.n, _p(recs.d), _p(recs.i), tx, _p(k), _p(v))
    return k, v


def stable_sort_pairs(keys_in, values_in):
    """Library stable sort (std::stable_sort) of (key, value) by key."""
    lib = _load()
    k = np.ascontiguousarray(keys_in, np.uint64).copy()
    v = np.ascontiguousarray(values_in, np.uint32).copy()
    lib.orc_stable_sort_pairs(k.shape[0], _p(k), _p(v))
    return k, v


def pair_max_weight(recs: Records, cam, g, tile, settings=None):
    """max over the pixel centres of ``tile`` of o*exp(-Q/2) for Gaussian g."""
    lib = _load()
    g = np.ascontiguousarray(g, np.uint32)
    tile = np.ascontiguousarray(tile, np.uint32)
    out = np.zeros(g.shape[0])
    ca, sa = cam_array(cam), set_array(settings)
    lib.orc_pair_max_weight(g.shape[0], _p(g), _p(tile), _p(recs.d), _p(ca), _p(sa), _p(out))
    return out


def sh_basis(degree, dirs):
    """Real SH basis (n,16) at unit directions (n,3)."""
    lib = _load()
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], 16))
    if lib.orc_sh_basis(int(degree), dirs.shape[0], _p(dirs), _p(out)) != 0:
        raise ValueError("degree must be 0..3")
    return out
