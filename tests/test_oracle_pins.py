"""Pins of the FP64 oracle against what the paper and mathematics fix.

Closed forms (Section 3.2, Eqs. 1-3), library routines (SciPy spherical
harmonics and rotations, NumPy stable argsort), invariants and brute force.
None of these re-types the oracle's own code path: each expected value comes
from a separate derivation or an outside routine.
"""
import math

import numpy as np
import pytest
import scipy.special as sps
from scipy.spatial.transform import Rotation

from paper_2512_08478_amd import scenes as S

TAU = 1.0 / 255.0


def one_scene(points, log_scale, logit, dc, quats=None, degree=0, sh=None):
    n = len(points)
    means = np.asarray(points, np.float32).reshape(n, 3)
    ls = np.broadcast_to(np.asarray(log_scale, np.float32), (n, 3)).copy()
    q = np.tile(np.array([1, 0, 0, 0], np.float32), (n, 1)) if quats is None else np.asarray(quats, np.float32)
    lg = np.broadcast_to(np.asarray(logit, np.float32), (n,)).copy()
    if sh is None:
        K = (degree + 1) ** 2
        sh = np.zeros((n, K, 3), np.float32)
        sh[:, 0, :] = np.asarray(dc, np.float32)
    return S.Scene(means, ls, q, lg, np.asarray(sh, np.float32), degree)


def axis_camera(W=32, H=32, f=40.0):
    return S.Camera(np.eye(4, dtype=np.float32), f, f, W / 2, H / 2, W, H, 0.2)


def f32(x):
    return float(np.float32(x))


# ---------------------------------------------------------------- P1, P2 (Eq. 1)

@pytest.mark.parametrize("eps", [0.0, 0.3])
def test_p1_isotropic_on_axis(orc, eps):
    sigma, d = f32(0.05), 2.5
    sc = one_scene([[0, 0, d]], math.log(sigma), 2.0, [0.1, 0.2, 0.3])
    cam = axis_camera()
    r = orc.preprocess(sc, cam, dict(eps2d=eps))
    sig = float(np.exp(np.float64(np.float32(math.log(sigma)))))
    expect = (cam.fx * sig / d) ** 2 + eps
    assert r.i[0, orc.I_CULL] == orc.C_VISIBLE
    np.testing.assert_allclose(r.d[0, [orc.D_MX, orc.D_MY]], [cam.cx, cam.cy], rtol=0, atol=1e-12)
    np.testing.assert_allclose(r.d[0, [orc.D_SA, orc.D_SB, orc.D_SC]], [expect, 0, expect], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(r.d[0, [orc.D_CA, orc.D_CB, orc.D_CC]], [1 / expect, 0, 1 / expect], rtol=1e-12)
    assert r.d[0, orc.D_DEPTH] == pytest.approx(d, abs=1e-12)


def test_p2_isotropic_off_axis(orc):
    sigma = float(np.exp(np.float64(np.float32(math.log(0.04)))))
    x0, d, eps = f32(0.3), 2.0, 0.3
    sc = one_scene([[x0, 0, d]], np.float32(math.log(0.04)), 2.0, [0, 0, 0])
    cam = axis_camera(64, 48, 50.0)
    r = orc.preprocess(sc, cam, dict(eps2d=eps))
    k = (cam.fx * sigma / d) ** 2
    np.testing.assert_allclose(r.d[0, orc.D_SA], k * (1 + x0 * x0 / (d * d)) + eps, rtol=1e-12)
    np.testing.assert_allclose(r.d[0, orc.D_SC], k + eps, rtol=1e-12)
    assert abs(r.d[0, orc.D_SB]) < 1e-12
    np.testing.assert_allclose(r.d[0, [orc.D_MX, orc.D_MY]], [cam.cx + cam.fx * x0 / d, cam.cy], rtol=1e-12)


def test_p2_jacobian_clamp(orc):
    # far off-axis: x/z is clamped to 1.3 * (W/2)/fx inside J only
    sigma = float(np.exp(np.float64(np.float32(math.log(0.05)))))
    x0, d = f32(3.0), 2.0
    sc = one_scene([[x0, 0, d]], np.float32(math.log(0.05)), 6.0, [0, 0, 0])
    cam = axis_camera(64, 64, 40.0)
    r = orc.preprocess(sc, cam, dict(eps2d=0.0))
    lim = 1.3 * 32 / 40.0
    k = (cam.fx * sigma / d) ** 2
    np.testing.assert_allclose(r.d[0, orc.D_SA], k * (1 + lim * lim), rtol=1e-12)
    np.testing.assert_allclose(r.d[0, orc.D_MX], cam.cx + cam.fx * x0 / d, rtol=1e-12)


# ---------------------------------------------------------------- P3-P5 (Eqs. 2-3)

def closed_form_weight(cam, mx, my, s2, o, x, y, amax=0.99):
    r2 = (x + 0.5 - mx) ** 2 + (y + 0.5 - my) ** 2
    return min(amax, o * math.exp(-r2 / (2 * s2)))


def test_p3_single_gaussian_image(orc):
    sigma_l = np.float32(math.log(0.06))
    sigma = float(np.exp(np.float64(sigma_l)))
    d, logit = 3.0, np.float32(1.5)
    dc = np.array([0.4, -0.2, 1.1], np.float32)
    sc = one_scene([[0, 0, d]], sigma_l, logit, dc)
    cam = axis_camera(24, 20, 60.0)
    r = orc.preprocess(sc, cam)
    img = orc.render_image(r, cam)
    o = 1 / (1 + math.exp(-float(logit)))
    s2 = (cam.fx * sigma / d) ** 2 + 0.3
    rgb = np.maximum(0.0, dc.astype(np.float64) / (2 * math.sqrt(math.pi)) + 0.5)
    for y in range(cam.height):
        for x in range(cam.width):
            a = closed_form_weight(cam, cam.cx, cam.cy, s2, o, x, y)
            if a < TAU:
                a = 0.0
            np.testing.assert_allclose(img["rgba"][y, x, :3], rgb * a, atol=1e-13)
            np.testing.assert_allclose(img["rgba"][y, x, 3], a, atol=1e-13)


def test_p4_two_gaussians_order(orc):
    # Gaussian 0 is behind Gaussian 1: the nearer one must be composited first.
    l = np.float32(math.log(0.08))
    sc = one_scene([[0, 0, 4.0], [0, 0, 2.0]], l, [0.5, 2.0], [[1.0, 0, 0], [0, 1.0, 0]])
    cam = axis_camera(16, 16, 30.0)
    r = orc.preprocess(sc, cam)
    o = [1 / (1 + math.exp(-0.5)), 1 / (1 + math.exp(-2.0))]
    sig = float(np.exp(np.float64(l)))
    s2 = [(cam.fx * sig / 4.0) ** 2 + 0.3, (cam.fx * sig / 2.0) ** 2 + 0.3]
    c = [np.array([1.0, 0, 0]) / (2 * math.sqrt(math.pi)) + 0.5,  # exact in f32
         np.array([0, 1.0, 0]) / (2 * math.sqrt(math.pi)) + 0.5]
    out = orc.render_pixels(r, cam, [[8, 8], [9, 7], [3, 12]])
    for p, (x, y) in enumerate([[8, 8], [9, 7], [3, 12]]):
        a_far = closed_form_weight(cam, 8, 8, s2[0], o[0], x, y)
        a_near = closed_form_weight(cam, 8, 8, s2[1], o[1], x, y)
        a_far = a_far if a_far >= TAU else 0.0
        a_near = a_near if a_near >= TAU else 0.0
        expect = c[1] * a_near + c[0] * a_far * (1 - a_near)
        np.testing.assert_allclose(out["rgba"][p, :3], expect, atol=1e-13)
        np.testing.assert_allclose(out["T"][p], (1 - a_near) * (1 - a_far), atol=1e-13)


@pytest.mark.parametrize("n,alpha_target", [(20, 0.5), (40, 0.3), (5, 0.9)])
def test_p5_coincident_stack_blend_then_stop(orc, n, alpha_target):
    # n identical Gaussians: T_k = (1-a)^k, blending stops right after T < t_eps.
    logit = np.float32(math.log(alpha_target / (1 - alpha_target)))
    sc = one_scene([[0, 0, 2.0]] * n, np.float32(math.log(0.2)), logit, [0.3, 0.1, -0.4])
    cam = axis_camera(8, 8, 10.0)
    r = orc.preprocess(sc, cam, dict(eps2d=0.0))
    out = orc.render_pixels(r, cam, [[4, 4]], dict(eps2d=0.0))
    o = 1 / (1 + math.exp(-float(logit)))
    s2 = (cam.fx * float(np.exp(np.float64(np.float32(math.log(0.2))))) / 2.0) ** 2
    a = min(0.99, o * math.exp(-0.5 / (2 * s2)))
    k = 0
    T = 1.0
    while k < n:
        T *= (1 - a)
        k += 1
        if T < 1e-4:
            break
    dc = np.array([0.3, 0.1, -0.4], np.float32).astype(np.float64)
    rgb = np.maximum(0, dc / (2 * math.sqrt(math.pi)) + 0.5)
    assert out["n_blend"][0] == k
    np.testing.assert_allclose(out["T"][0], (1 - a) ** k, rtol=1e-12)
    np.testing.assert_allclose(out["rgba"][0, :3], rgb * (1 - (1 - a) ** k), rtol=1e-12)


def test_alpha_clamp(orc):
    # opacity close to 1: the pixel weight is clamped at alpha_max = 0.99
    sc = one_scene([[0, 0, 2.0]], np.float32(math.log(5.0)), 12.0, [0, 0, 0])
    cam = axis_camera(8, 8, 10.0)
    r = orc.preprocess(sc, cam)
    out = orc.render_pixels(r, cam, [[4, 4]])
    assert out["rgba"][0, 3] == pytest.approx(0.99, abs=1e-15)


def test_background(orc):
    sc = one_scene([[0, 0, -2.0]], -3.0, 0.0, [0, 0, 0])  # behind the camera
    cam = axis_camera(8, 8, 10.0)
    r = orc.preprocess(sc, cam, dict(bg=(0.25, 0.5, 1.0)))
    assert r.i[0, orc.I_CULL] == orc.C_NEAR
    out = orc.render_pixels(r, cam, [[1, 1], [7, 0]], dict(bg=(0.25, 0.5, 1.0)))
    np.testing.assert_array_equal(out["rgba"], [[0.25, 0.5, 1.0, 0.0]] * 2)


def test_cull_codes(orc):
    pts = [[0, 0, 0.1], [0, 0, 3], [0, 0, 3], [50, 0, 3]]
    sc = one_scene(pts, -3.0, [0, 0, -10, 0], [0, 0, 0])
    sc.quats[1] = 0.0
    cam = axis_camera(16, 16, 10.0)
    r = orc.preprocess(sc, cam)
    assert list(r.i[:, orc.I_CULL]) == [orc.C_NEAR, orc.C_INVALID, orc.C_OPACITY, orc.C_OFFIMAGE]


# ---------------------------------------------------------------- Sigma (CovFromScaleRot)

def test_covariance_eigen_invariants(orc):
    sc, cam = S.tiny_scene(n=256)
    r = orc.preprocess(sc, cam)
    c = r.d[:, orc.D_C3:orc.D_C3 + 6]
    Sig = np.stack([c[:, [0, 1, 2]], c[:, [1, 3, 4]], c[:, [2, 4, 5]]], 1)
    s2 = np.exp(2 * sc.log_scales.astype(np.float64))
    ev = np.linalg.eigvalsh(Sig)
    np.testing.assert_allclose(ev, np.sort(s2, 1), rtol=1e-9)
    # eigenvectors: columns of the rotation of the (normalised) quaternion,
    # taken from SciPy (scalar-last order)
    q = sc.quats.astype(np.float64)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    for k in range(3):
        v = R[:, :, k]
        np.testing.assert_allclose(np.einsum("nij,nj->ni", Sig, v), s2[:, k:k + 1] * v, atol=1e-12)


def test_model_transform_similarity(orc):
    # A similarity-placed asset equals the same asset with its means and
    # covariances moved by hand (SciPy rotation), colour evaluated in the
    # asset frame: rotate the camera with the asset instead.
    sc, cam = S.tiny_scene(n=64)
    rot = Rotation.from_euler("xyz", [0.3, -0.7, 1.1])
    s, t = 0.6, np.array([0.2, -0.1, 0.4])
    model = np.concatenate([s * rot.as_matrix(), t[:, None]], 1)
    placed = S.Scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, sc.sh_degree, model)
    r1 = orc.preprocess(placed, cam)
    # equivalent camera: world->camera composed with the model transform,
    # with the scale folded into the Gaussians (means and log-scales)
    V = cam.viewmat.astype(np.float64)
    Mk = np.eye(4)
    Mk[:3, :3] = rot.as_matrix()
    Mk[:3, 3] = t
    cam2 = S.Camera((V @ Mk), cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, cam.znear)
    sc2 = S.Scene(sc.means.astype(np.float64) * s, sc.log_scales.astype(np.float64) + math.log(s),
                  sc.quats, sc.opacity_logits, sc.sh, sc.sh_degree)
    r2 = orc.preprocess(sc2, cam2)
    keep = [orc.D_MX, orc.D_MY, orc.D_SA, orc.D_SB, orc.D_SC, orc.D_DEPTH, orc.D_R, orc.D_G, orc.D_B]
    # inputs of the second form are rounded to float32, hence the tolerance
    np.testing.assert_allclose(r1.d[:, keep], r2.d[:, keep], rtol=1e-5, atol=1e-6)


# ---------------------------------------------------------------- SH colour

def real_sh_from_scipy(l, m, x, y, z):
    theta = np.arccos(np.clip(z, -1, 1))
    phi = np.arctan2(y, x)
    if m == 0:
        return sps.sph_harm_y(l, 0, theta, phi).real
    Y = sps.sph_harm_y(l, abs(m), theta, phi)
    return math.sqrt(2) * (Y.real if m > 0 else Y.imag)


def test_sh_basis_matches_scipy(orc):
    rng = np.random.default_rng(7)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    B = orc.sh_basis(3, d)
    for l in range(4):
        for m in range(-l, l + 1):
            k = l * l + l + m
            ref = real_sh_from_scipy(l, m, d[:, 0], d[:, 1], d[:, 2])
            np.testing.assert_allclose(B[:, k], ref, atol=1e-13, err_msg=f"l={l} m={m}")


def test_sh_orthonormal_by_quadrature(orc):
    # Gauss-Legendre in cos(theta) x uniform phi: exact for these degrees
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 24
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).reshape(-1)
    B = orc.sh_basis(3, d)
    G = (B * w[:, None]).T @ B
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_degree0_colour_closed_form(orc):
    sc, cam = S.tiny_scene(n=512)
    r = orc.preprocess(sc, cam)
    dc = sc.sh[:, 0, :].astype(np.float64)
    np.testing.assert_allclose(r.d[:, orc.D_R:orc.D_B + 1],
                               np.maximum(0, dc / (2 * math.sqrt(math.pi)) + 0.5), rtol=1e-13, atol=1e-15)


def test_sh_degree1_direction(orc):
    # degree-1 colour of a Gaussian straight ahead (d = +z): only Y_1^0 = c1 z
    sh = np.zeros((1, 4, 3), np.float32)
    sh[0, 2, :] = [0.2, -0.1, 0.05]
    sh[0, 1, :] = [5.0, 5.0, 5.0]  # Y_1^-1 ~ y: zero on the axis
    sc = one_scene([[0, 0, 3.0]], -3.0, 0.0, None, degree=1, sh=sh)
    cam = axis_camera()
    r = orc.preprocess(sc, cam)
    c1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(r.d[0, orc.D_R:orc.D_B + 1],
                               np.float64(sh[0, 2]) * c1 + 0.5, rtol=1e-12)


# ---------------------------------------------------------------- compositing invariants

def test_front_to_back_equals_back_to_front(orc):
    # With termination and skipping off, Eq. 3 (front-to-back) equals the
    # back-to-front "over" recursion the paper's draw uses.
    sc, cam = S.tiny_scene(n=200)
    st = dict(t_eps=0.0, tau=1e-300)
    r = orc.preprocess(sc, cam, st)
    pix = np.array([[128, 128], [100, 140], [60, 70], [200, 190]])
    out = orc.render_pixels(r, cam, pix, st)
    vis = np.where(r.visible)[0]
    order = vis[np.lexsort((vis, r.d[vis, orc.D_DEPTH]))]
    for p, (x, y) in enumerate(pix):
        C = np.zeros(3)
        for g in order[::-1]:
            d = r.d[g]
            dx, dy = x + 0.5 - d[orc.D_MX], y + 0.5 - d[orc.D_MY]
            Q = d[orc.D_CA] * dx * dx + 2 * d[orc.D_CB] * dx * dy + d[orc.D_CC] * dy * dy
            a = min(0.99, d[orc.D_OPAC] * math.exp(-0.5 * Q))
            C = a * d[orc.D_R:orc.D_B + 1] + (1 - a) * C
        np.testing.assert_allclose(out["rgba"][p, :3], C, atol=1e-12)


def test_shuffle_invariance(orc):
    sc, cam = S.tiny_scene(n=1024)
    pix = orc.all_pixels(cam)[::37]
    a = orc.render_pixels(orc.preprocess(sc, cam), cam, pix)
    perm = np.random.default_rng(3).permutation(sc.n)
    b = orc.render_pixels(orc.preprocess(sc.subset(perm), cam), cam, pix)
    np.testing.assert_array_equal(a["rgba"], b["rgba"])


def test_global_sort_equals_concatenation(orc):
    # Section 4.5: one global sort over all assets == the concatenated asset.
    sc, cam = S.tiny_scene(n=600)
    parts = [sc.subset(np.arange(0, 250)), sc.subset(np.arange(250, 600))]
    pix = orc.all_pixels(cam)[::29]
    a = orc.render_pixels(orc.preprocess(sc, cam), cam, pix)
    b = orc.render_pixels(orc.preprocess_many(parts, cam), cam, pix)
    np.testing.assert_array_equal(a["rgba"], b["rgba"])


def test_bbox_is_exact_support(orc):
    # Outside the tile rect every pixel weight is below tau; inside the pixel
    # bbox's edge pixels the weight can reach tau (the rect is not loose by
    # more than one pixel row of the ellipse's bbox).
    sc, cam = S.tiny_scene(n=300)
    r = orc.preprocess(sc, cam)
    tx, ty = orc.tiles_xy(cam)
    gs, tiles = [], []
    for g in np.where(r.visible)[0]:
        iv = r.i[g]
        for t in range(tx * ty):
            x, y = t % tx, t // tx
            if not (iv[orc.I_TX0] <= x <= iv[orc.I_TX1] and iv[orc.I_TY0] <= y <= iv[orc.I_TY1]):
                gs.append(g)
                tiles.append(t)
    w = orc.pair_max_weight(r, cam, np.array(gs), np.array(tiles))
    assert w.max() < TAU
    # per-pixel: weight below tau just outside the pixel bbox
    for g in np.where(r.visible)[0][:50]:
        iv, d = r.i[g], r.d[g]
        for x, y in [(iv[orc.I_PX0] - 1, int(d[orc.D_MY])), (iv[orc.I_PX1] + 1, int(d[orc.D_MY])),
                     (int(d[orc.D_MX]), iv[orc.I_PY0] - 1), (int(d[orc.D_MX]), iv[orc.I_PY1] + 1)]:
            dx, dy = x + 0.5 - d[orc.D_MX], y + 0.5 - d[orc.D_MY]
            Q = d[orc.D_CA] * dx * dx + 2 * d[orc.D_CB] * dx * dy + d[orc.D_CC] * dy * dy
            assert d[orc.D_OPAC] * math.exp(-0.5 * Q) < TAU


def test_stale_sort_differs(orc):
    # Section 4.4: an order taken from another camera gives a different image.
    sc, cam = S.tiny_scene(n=1500)
    cam2 = S.pinhole_camera(S.look_at((2.2, 0.0, -2.0)), 256, 256, 60.0)
    r_new = orc.preprocess(sc, cam2)
    r_old = orc.preprocess(sc, cam)
    stale = S.Scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, 0)  # noqa: F841
    rec = orc.Records(r_new.d.copy(), r_new.i.copy())
    rec.d[:, orc.D_DEPTH] = r_old.d[:, orc.D_DEPTH]  # order by the old camera's depths
    pix = orc.all_pixels(cam2)[::13]
    a = orc.render_pixels(r_new, cam2, pix)["rgba"]
    b = orc.render_pixels(rec, cam2, pix)["rgba"]
    assert np.abs(a - b).max() > 1e-2


# ---------------------------------------------------------------- keys + sort

@pytest.mark.parametrize("kind", S.SORT_KEY_KINDS)
def test_stable_sort_matches_numpy(orc, kind):
    k, v = S.sort_keys(kind, 5000, seed=11)
    ks, vs = orc.stable_sort_pairs(k, v)
    perm = np.argsort(k, kind="stable")
    np.testing.assert_array_equal(ks, k[perm])
    np.testing.assert_array_equal(vs, v[perm])


def test_stable_sort_brute_force_tiny(orc):
    rng = np.random.default_rng(1)
    for n in [0, 1, 2, 5, 17, 64]:
        k = rng.integers(0, 4, n).astype(np.uint64) << np.uint64(40)
        v = np.arange(n, dtype=np.uint32)
        ks, vs = orc.stable_sort_pairs(k, v)
        ref = sorted(zip(k.tolist(), v.tolist()), key=lambda t: t[0])
        assert [int(a) for a in ks] == [a for a, _ in ref]
        assert [int(b) for b in vs] == [b for _, b in ref]
        assert np.all(np.diff(ks.astype(np.float64)) >= 0)


def test_keys_structure(orc):
    sc, cam = S.tiny_scene()
    r = orc.preprocess(sc, cam)
    k, v = orc.keys(r, cam)
    assert len(k) == r.i[r.visible, orc.I_TILES].sum()
    tx, ty = orc.tiles_xy(cam)
    tile = (k >> np.uint64(32)).astype(np.int64)
    zb = (k & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    np.testing.assert_array_equal(zb.view(np.float32), r.d[v, orc.D_DEPTH].astype(np.float32))
    x, y = tile % tx, tile // tx
    iv = r.i[v]
    assert np.all((iv[:, orc.I_TX0] <= x) & (x <= iv[:, orc.I_TX1]))
    assert np.all((iv[:, orc.I_TY0] <= y) & (y <= iv[:, orc.I_TY1]))
    assert np.all(np.diff(v.astype(np.int64)) >= 0)  # Gaussian-major


# ---------------------------------------------------------------- Pre-pack (Section 3.4)

def _cov6_scipy(sc):
    """Upper triangle of R diag(s^2) R^T with R from SciPy (scalar-last)."""
    q = sc.quats.astype(np.float32).astype(np.float64)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    s2 = np.exp(2 * sc.log_scales.astype(np.float32).astype(np.float64))
    Sig = np.einsum("nik,nk,njk->nij", R, s2, R)
    return Sig[:, [0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]


def test_covariance_helper_matches_scipy(orc):
    sc, _ = S.tiny_scene(n=512)
    Sig = orc.covariance(sc)
    np.testing.assert_allclose(Sig[:, [0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]], _cov6_scipy(sc),
                               rtol=1e-12, atol=1e-18)


@pytest.mark.parametrize("with_model", [False, True])
def test_covariance_input_path_matches_raw_parameters(orc, with_model):
    # The pre-packed inputs without the fp16 rounding (mean, sigmoid of the
    # logit, SciPy covariance, SH, all float64) reproduce the raw-parameter
    # records: the two front ends meet at the same Sigma.
    sc, cam = S.medium_scene(n=3000)
    if with_model:
        rot = Rotation.from_euler("xyz", [0.2, 0.5, -0.3])
        model = np.concatenate([0.8 * rot.as_matrix(), np.array([[0.3], [-0.2], [0.1]])], 1)
        sc = S.Scene(sc.means, sc.log_scales, sc.quats, sc.opacity_logits, sc.sh, sc.sh_degree, model)
    r_raw = orc.preprocess(sc, cam)
    logit = sc.opacity_logits.astype(np.float32).astype(np.float64)
    packed = dict(means=sc.means.astype(np.float32), opacity=1 / (1 + np.exp(-logit)),
                  cov6=_cov6_scipy(sc), sh=sc.sh.astype(np.float32), sh_degree=sc.sh_degree,
                  model=sc.model)
    r_cov = orc.preprocess_packed(packed, cam)
    assert r_raw.visible.sum() > 500
    np.testing.assert_array_equal(r_cov.i[:, orc.I_CULL], r_raw.i[:, orc.I_CULL])
    v = r_raw.visible
    np.testing.assert_array_equal(r_cov.i[v], r_raw.i[v])
    np.testing.assert_allclose(r_cov.d[v], r_raw.d[v], rtol=1e-9, atol=1e-12)


def test_fp16_rounding_is_ieee_nearest_even(orc):
    # Round-to-nearest-even into binary16 (11-bit significand, subnormals
    # down to 2**-24, overflow past 65520), as IEEE 754 defines it.
    u = 2.0 ** -10
    cases = [(1 + u / 2, 1.0),                    # tie -> even
             (1 + 3 * u / 2, 1 + 2 * u),          # tie -> even (up)
             (1 + u / 2 + 2.0 ** -40, 1 + u),     # just past the tie
             (2.0 ** -25, 0.0),                   # tie at the smallest subnormal
             (2.0 ** -25 * 1.0000001, 2.0 ** -24),
             (3 * 2.0 ** -26, 2.0 ** -24),
             (65504.0, 65504.0), (65519.99, 65504.0), (65520.0, np.inf),
             (-(1 + 3 * u / 2), -(1 + 2 * u))]
    got = orc.to_fp16(np.array([x for x, _ in cases]))
    assert got.dtype == np.float16
    want = np.array([w for _, w in cases])
    np.testing.assert_array_equal(got.astype(np.float64), want)


def test_prepack_fields(orc):
    sc, _ = S.medium_scene(n=2000)
    p = orc.prepack(sc)
    assert all(p[k].dtype == np.float16 for k in ("means", "opacity", "cov6", "sh"))
    Sig = orc.covariance(sc)
    iu = ([0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2])
    exact = Sig[:, iu[0], iu[1]]
    # each packed covariance entry is the nearest binary16 value: within
    # half a spacing of the exact one
    got = p["cov6"].astype(np.float64)
    sp = np.spacing(np.abs(got).astype(np.float16)).astype(np.float64)
    assert np.all(np.abs(got - exact) <= 0.5 * sp * (1 + 1e-12))
    logit = sc.opacity_logits.astype(np.float32).astype(np.float64)
    o = p["opacity"].astype(np.float64)
    assert np.all(np.abs(o - 1 / (1 + np.exp(-logit))) <= 0.5 * np.spacing(p["opacity"]).astype(np.float64))
    np.testing.assert_array_equal(p["means"], sc.means.astype(np.float32).astype(np.float16))
    np.testing.assert_array_equal(p["sh"], sc.sh.astype(np.float32).astype(np.float16))


# ---------------------------------------------------------------- mesh depth composition (Section 3.4)

def _const_mesh(cam, depth, seed=3):
    rng = np.random.default_rng(seed)
    return dict(depth=np.full((cam.height, cam.width), depth, np.float32),
                rgb=rng.uniform(0, 1, (cam.height, cam.width, 3)).astype(np.float32))


def test_mesh_wall_behind_everything_is_a_background(orc):
    # A wall behind every Gaussian hides nothing: the image is the plain one
    # with the wall's colour in place of the background, C + T * rgb_mesh.
    sc, cam = S.tiny_scene(n=1024)
    r = orc.preprocess(sc, cam)
    pix = orc.all_pixels(cam)[::7]
    plain = orc.render_pixels(r, cam, pix)
    mesh = _const_mesh(cam, 1e4)
    m = orc.render_pixels(r, cam, pix, mesh=mesh)
    rgb = mesh["rgb"][pix[:, 1], pix[:, 0]].astype(np.float64)
    np.testing.assert_array_equal(m["T"], plain["T"])
    np.testing.assert_array_equal(m["n_blend"], plain["n_blend"])
    np.testing.assert_allclose(m["rgba"][:, :3], plain["rgba"][:, :3] + plain["T"][:, None] * rgb,
                               atol=1e-15)
    np.testing.assert_array_equal(m["rgba"][:, 3], plain["rgba"][:, 3])
    assert plain["n_blend"].max() > 0


def test_mesh_wall_in_front_hides_everything(orc):
    sc, cam = S.tiny_scene(n=1024)
    r = orc.preprocess(sc, cam)
    pix = orc.all_pixels(cam)[::5]
    mesh = _const_mesh(cam, 0.1)   # nearer than the near plane: every Gaussian is behind
    m = orc.render_pixels(r, cam, pix, mesh=mesh)
    np.testing.assert_array_equal(m["n_blend"], 0)
    np.testing.assert_array_equal(m["T"], 1.0)
    np.testing.assert_array_equal(m["rgba"][:, :3], mesh["rgb"][pix[:, 1], pix[:, 0]].astype(np.float64))
    np.testing.assert_array_equal(m["rgba"][:, 3], 0.0)


def test_mesh_wall_between_two_gaussians(orc):
    # The two-Gaussian scene of P4 (depths 2 and 4) with a wall at depth 3:
    # only the near Gaussian is composited, over the wall's colour.
    l = np.float32(math.log(0.08))
    sc = one_scene([[0, 0, 4.0], [0, 0, 2.0]], l, [0.5, 2.0], [[1.0, 0, 0], [0, 1.0, 0]])
    cam = axis_camera(16, 16, 30.0)
    r = orc.preprocess(sc, cam)
    o_near = 1 / (1 + math.exp(-2.0))
    sig = float(np.exp(np.float64(l)))
    s2 = (cam.fx * sig / 2.0) ** 2 + 0.3
    c_near = np.array([0, 1.0, 0]) / (2 * math.sqrt(math.pi)) + 0.5
    pts = [[8, 8], [9, 7], [3, 12]]
    for D in (3.0, 2.0):   # D = 2 exactly: a Gaussian at the mesh depth is kept
        mesh = _const_mesh(cam, D, seed=4)
        out = orc.render_pixels(r, cam, pts, mesh=mesh)
        for p, (x, y) in enumerate(pts):
            a = closed_form_weight(cam, 8, 8, s2, o_near, x, y)
            a = a if a >= TAU else 0.0
            wall = mesh["rgb"][y, x].astype(np.float64)
            np.testing.assert_allclose(out["rgba"][p, :3], c_near * a + wall * (1 - a), atol=1e-13)
            np.testing.assert_allclose(out["T"][p], 1 - a, atol=1e-13)
            assert out["n_blend"][p] == (1 if a > 0 else 0)
            # a blended Gaussian exactly at the mesh depth is flagged
            assert bool(out["flags"][p] & 4) == (D == 2.0 and a > 0)


def test_plane_mesh_depth_is_the_ray_plane_intersection(orc):
    # the input generator's wall: at each pixel, the camera-space point
    # z * ((x + 1/2 - cx)/fx, (y + 1/2 - cy)/fy, 1) lies on the world plane
    sc, cam = S.tiny_scene(n=4)
    n, h = np.array([0.3, 0.2, 1.0]), 0.2
    m = S.plane_mesh(cam, n, h)
    V = cam.viewmat.astype(np.float64)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    z = m["depth"].astype(np.float64)
    ok = np.isfinite(z)
    assert ok.mean() > 0.5
    xc = np.stack([(xs + 0.5 - cam.cx) / cam.fx * z, (ys + 0.5 - cam.cy) / cam.fy * z, z], -1)[ok]
    Xw = (xc - V[:3, 3]) @ V[:3, :3]
    np.testing.assert_allclose(Xw @ (n / np.linalg.norm(n)), h, atol=1e-5)


# ---------------------------------------------------------------- LBS pre-decoder (Section 3.3, Eqs. 5-6)

def _skin_one(n, joints_of, weights_of):
    idx = np.zeros((n, 4), np.uint8)
    w = np.zeros((n, 4), np.float32)
    idx[:, :len(joints_of)] = joints_of
    w[:, :len(weights_of)] = weights_of
    return idx, w


def test_lbs_identity_pose_is_exact(orc):
    sc, _ = S.medium_scene(n=3000)
    pk = orc.prepack(sc)
    centres, idx, w = S.skinning(sc.means, n_joints=20, seed=1)
    out = orc.lbs_deform(pk, idx, w, S.joint_pose(centres, seed=None))
    # the same binary16 numbers (a -0 may come back as +0)
    np.testing.assert_array_equal(out["means"], pk["means"])
    np.testing.assert_array_equal(out["cov6"], pk["cov6"])
    assert out["opacity"] is pk["opacity"] and out["sh"] is pk["sh"]


def test_lbs_single_joint_equals_model_transform(orc):
    # all weight on one rigid joint: the same records as rendering the
    # canonical asset placed by that transform (colour is view-independent
    # at SH degree 0, so it agrees too)
    sc, cam = S.tiny_scene(n=2000)
    pk = orc.prepack(sc)
    R = Rotation.from_euler("xyz", [0.3, -0.5, 0.2]).as_matrix()
    M = np.concatenate([R, np.array([[0.2], [-0.1], [0.3]])], 1)
    joints = np.stack([np.eye(3, 4), M]).astype(np.float64)
    idx, w = _skin_one(sc.n, [1], [1.0])
    d = orc.lbs_deform(pk, idx, w, joints, rounded=False)
    r_lbs = orc.preprocess_packed(dict(d, model=None), cam)
    r_mod = orc.preprocess_packed(dict(pk, model=M), cam)
    assert r_mod.visible.sum() > 500
    np.testing.assert_array_equal(r_lbs.i[:, orc.I_CULL], r_mod.i[:, orc.I_CULL])
    v = r_mod.visible
    keep = [orc.D_MX, orc.D_MY, orc.D_SA, orc.D_SB, orc.D_SC, orc.D_DEPTH, orc.D_R, orc.D_G, orc.D_B]
    np.testing.assert_allclose(r_lbs.d[v][:, keep], r_mod.d[v][:, keep], rtol=1e-10, atol=1e-12)


def test_lbs_translation_blend_closed_form(orc):
    sc, _ = S.tiny_scene(n=64)
    pk = orc.prepack(sc)
    a, b = np.array([1.0, 0.0, 0.5]), np.array([0.0, 2.0, -1.0])
    joints = np.zeros((2, 3, 4))
    joints[:, :, :3] = np.eye(3)
    joints[0, :, 3], joints[1, :, 3] = a, b
    idx, w = _skin_one(sc.n, [0, 1], [0.25, 0.75])   # exact in float32
    d = orc.lbs_deform(pk, idx, w, joints, rounded=False)
    np.testing.assert_allclose(d["means"], pk["means"].astype(np.float64) + 0.25 * a + 0.75 * b,
                               rtol=0, atol=1e-15)
    np.testing.assert_array_equal(d["cov6"], pk["cov6"].astype(np.float64))


def test_lbs_rotation_blend_shrinks_closed_form(orc):
    # Blending a rotation about z by theta with the identity shrinks the
    # xy-plane: R = w1 Rz + w2 I, R R^T = diag(a^2 + b^2, a^2 + b^2, 1) with
    # a = w1 cos(theta) + w2, b = w1 sin(theta) (the LBS "candy wrapper").
    th, w1, w2 = 1.1, 0.5, 0.5
    pk = dict(means=np.array([[0.5, -0.25, 1.0]], np.float16), opacity=np.array([0.5], np.float16),
              cov6=np.array([[0.25, 0, 0, 0.25, 0, 0.25]], np.float16),
              sh=np.zeros((1, 1, 3), np.float16), sh_degree=0, model=None)
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    joints = np.stack([np.concatenate([Rz, np.zeros((3, 1))], 1), np.eye(3, 4)])
    d = orc.lbs_deform(pk, np.array([[0, 1, 0, 0]], np.uint8), np.array([[w1, w2, 0, 0]], np.float32),
                       joints, rounded=False)
    a, b = w1 * math.cos(th) + w2, w1 * math.sin(th)
    np.testing.assert_allclose(d["cov6"][0], 0.25 * np.array([a * a + b * b, 0, 0, a * a + b * b, 0, 1]),
                               atol=1e-15)
    mu = np.array([0.5, -0.25, 1.0])
    np.testing.assert_allclose(d["means"][0], [a * mu[0] - b * mu[1], b * mu[0] + a * mu[1], mu[2]],
                               atol=1e-15)


def test_skinning_generator(orc):
    sc, _ = S.medium_scene(n=5000)
    centres, idx, w = S.skinning(sc.means, n_joints=55, seed=3)
    assert centres.shape == (55, 3) and idx.shape == (5000, 4) and w.dtype == np.float32
    np.testing.assert_allclose(w.astype(np.float64).sum(1), 1.0, atol=1e-6)
    assert idx.max() < 55 and (w > 0).all()
    # the first influence is a nearest joint
    d = np.linalg.norm(sc.means[:, None, :].astype(np.float64) - centres[None].astype(np.float64), axis=2)
    dsel = np.take_along_axis(d, idx.astype(np.int64), 1)
    assert np.all(dsel.min(1) <= d.min(1) + 1e-6)
