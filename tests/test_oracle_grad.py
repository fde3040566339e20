"""Pin of the reference gradients (float64 autograd of the definition)
against central finite differences of the separate C forward."""
import math

import numpy as np
import pytest

from paper_2512_08478_amd import scenes as S


def _loss_c(orc, scene, cam, pix, G, settings=None):
    r = orc.preprocess(scene, cam, settings, f64_inputs=True)
    out = orc.render_pixels(r, cam, pix, settings)
    return float((out["rgba"] * G).sum()), out


def _f64(scene):
    return S.Scene(*(np.asarray(a, np.float64).copy() for a in
                     (scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh)),
                   scene.sh_degree, scene.model)


def test_autograd_forward_matches_c_forward(orc):
    from oracle import grad as og
    sc, cam = S.tiny_scene(n=512)
    pix = orc.all_pixels(cam)[::97]
    G = np.zeros((len(pix), 4))
    rgba, _ = og.render_and_grad(sc, cam, pix, G)
    ref = orc.render_pixels(orc.preprocess(sc, cam), cam, pix)["rgba"]
    np.testing.assert_allclose(rgba, ref, atol=1e-12)


@pytest.mark.parametrize("with_model", [False, True])
def test_gradients_match_central_differences(orc, with_model):
    from oracle import grad as og
    sc, cam = S.fd_scene()
    if with_model:
        from scipy.spatial.transform import Rotation
        A = 0.8 * Rotation.from_euler("xyz", [0.2, 0.5, -0.3]).as_matrix()
        sc.model = np.concatenate([A, np.array([[0.1], [-0.2], [0.3]])], 1)
    sc = _f64(sc)
    pix = orc.all_pixels(cam)
    r0 = orc.preprocess(sc, cam, f64_inputs=True)
    base = orc.render_pixels(r0, cam, pix)
    rng = np.random.default_rng(21)
    G = rng.standard_normal((len(pix), 4))
    # finite differences are only valid where no discrete decision is near
    safe = (base["margin"] > 1e-3) & (base["flags"] == 0)
    G[~safe] = 0.0
    assert safe.mean() > 0.95
    _, g_ad = og.render_and_grad(sc, cam, pix, G)
    h = 1e-6
    names = ["means", "log_scales", "quats", "opacity_logits", "sh"]
    for nm in names:
        arr = getattr(sc, nm)
        fd = np.zeros(arr.shape)
        flat = arr.reshape(-1)
        idx = np.arange(flat.size)
        if nm == "sh":  # linear in sh: a sample of entries suffices
            idx = rng.choice(flat.size, 300, replace=False)
        for k in idx:
            v = flat[k]
            flat[k] = v + h
            lp, _ = _loss_c(orc, sc, cam, pix, G)
            flat[k] = v - h
            lm, _ = _loss_c(orc, sc, cam, pix, G)
            flat[k] = v
            fd.reshape(-1)[k] = (lp - lm) / (2 * h)
        ad = g_ad[nm].reshape(-1)[idx]
        fdv = fd.reshape(-1)[idx]
        scale = np.abs(fdv).max()
        assert scale > 0, nm
        np.testing.assert_allclose(ad, fdv, rtol=1e-5, atol=1e-6 * scale, err_msg=nm)


def test_single_gaussian_opacity_derivative_closed_form(orc):
    # dA/dlogit = o(1-o) exp(-r^2 / 2 s^2) when the alpha clamp does not bind
    from oracle import grad as og
    sc = S.Scene(np.array([[0, 0, 2.0]]), np.full((1, 3), math.log(0.1)), np.array([[1.0, 0, 0, 0]]),
                 np.array([0.3]), np.zeros((1, 1, 3)), 0)
    cam = S.Camera(np.eye(4, dtype=np.float32), 20.0, 20.0, 8.0, 8.0, 16, 16, 0.2)
    pix = np.array([[8, 8], [10, 7]])
    G = np.zeros((2, 4))
    G[:, 3] = 1.0
    _, g = og.render_and_grad(sc, cam, pix, G)
    o = 1 / (1 + math.exp(-0.3))
    s2 = (20 * 0.1 / 2.0) ** 2 + 0.3
    expect = sum(o * (1 - o) * math.exp(-((x + 0.5 - 8) ** 2 + (y + 0.5 - 8) ** 2) / (2 * s2)) for x, y in pix)
    assert g["opacity_logits"][0] == pytest.approx(expect, rel=1e-12)


def _two_assets(orc):
    """The FD instance split into two assets, the second placed by a
    similarity transform, so their Gaussians interleave in depth."""
    from scipy.spatial.transform import Rotation
    sc, cam = S.fd_scene()
    sc = _f64(sc)
    A = 0.9 * Rotation.from_euler("xyz", [0.1, -0.4, 0.25]).as_matrix()
    model = np.concatenate([A, np.array([[0.05], [0.1], [-0.2]])], 1)
    h = sc.n // 2
    part = lambda sl, m: S.Scene(*(np.ascontiguousarray(getattr(sc, k)[sl]) for k in
                                   ("means", "log_scales", "quats", "opacity_logits", "sh")),
                                 sc.sh_degree, m)
    return [part(slice(0, h), None), part(slice(h, None), model)], cam


def test_multi_asset_autograd_forward_matches_c_forward(orc):
    from oracle import grad as og
    assets, cam = _two_assets(orc)
    pix = orc.all_pixels(cam)
    rgba, _ = og.render_and_grad_assets(assets, cam, pix, np.zeros((len(pix), 4)))
    ref = orc.render_pixels(orc.preprocess_many(assets, cam, f64_inputs=True), cam, pix)["rgba"]
    np.testing.assert_allclose(rgba, ref, atol=1e-12)
    # both assets contribute, so the global order really interleaves them
    solo = [orc.render_pixels(orc.preprocess(a, cam, f64_inputs=True), cam, pix)["rgba"] for a in assets]
    assert all(np.abs(s[:, 3]).max() > 0.05 for s in solo)
    assert np.abs(ref - solo[0]).max() > 1e-3 and np.abs(ref - solo[1]).max() > 1e-3


def test_multi_asset_gradients_match_central_differences(orc):
    from oracle import grad as og
    assets, cam = _two_assets(orc)
    pix = orc.all_pixels(cam)
    base = orc.render_pixels(orc.preprocess_many(assets, cam, f64_inputs=True), cam, pix)
    rng = np.random.default_rng(31)
    G = rng.standard_normal((len(pix), 4))
    G[~((base["margin"] > 1e-3) & (base["flags"] == 0))] = 0.0
    _, g_ad = og.render_and_grad_assets(assets, cam, pix, G)
    h = 1e-6

    def loss():
        out = orc.render_pixels(orc.preprocess_many(assets, cam, f64_inputs=True), cam, pix)
        return float((out["rgba"] * G).sum())
    for a, sc in enumerate(assets):
        for nm in ("means", "log_scales", "quats", "opacity_logits", "sh"):
            flat = getattr(sc, nm).reshape(-1)
            idx = rng.choice(flat.size, min(flat.size, 40), replace=False)
            fd = np.zeros(len(idx))
            for j, k in enumerate(idx):
                v = flat[k]
                flat[k] = v + h
                lp = loss()
                flat[k] = v - h
                lm = loss()
                flat[k] = v
                fd[j] = (lp - lm) / (2 * h)
            ad = g_ad[a][nm].reshape(-1)[idx]
            scale = max(np.abs(fd).max(), 1e-12)
            np.testing.assert_allclose(ad, fd, rtol=1e-5, atol=1e-6 * scale, err_msg=f"asset {a} {nm}")


def test_mesh_autograd_forward_matches_c_forward(orc):
    from oracle import grad as og
    sc, cam = S.tiny_scene(n=512)
    mesh = S.plane_mesh(cam, (0.3, 0.2, 1.0), 0.1, seed=2, occupancy=0.6)
    pix = orc.all_pixels(cam)[::53]
    G = np.zeros((len(pix), 4))
    rgba, _ = og.render_and_grad(sc, cam, pix, G, mesh=mesh)
    ref = orc.render_pixels(orc.preprocess(sc, cam), cam, pix, mesh=mesh)
    np.testing.assert_allclose(rgba, ref["rgba"], atol=1e-12)
    plain = orc.render_pixels(orc.preprocess(sc, cam), cam, pix)
    assert (ref["n_blend"] < plain["n_blend"]).sum() > 10   # the wall hides something


def test_mesh_gradients_match_central_differences(orc):
    from oracle import grad as og
    sc, cam = S.fd_scene()
    sc = _f64(sc)
    pix = orc.all_pixels(cam)
    r0 = orc.preprocess(sc, cam, f64_inputs=True)
    depth = r0.d[r0.visible, orc.D_DEPTH]
    mesh = S.plane_mesh(cam, (0.2, -0.1, 1.0), 0.0, seed=9, occupancy=0.7)
    # move the wall into the middle of the Gaussians' depth range
    fin = np.isfinite(mesh["depth"])
    mesh["depth"][fin] += np.float32(np.median(depth) - np.median(mesh["depth"][fin]))
    base = orc.render_pixels(r0, cam, pix, mesh=mesh)
    plain = orc.render_pixels(r0, cam, pix)
    assert (base["n_blend"] < plain["n_blend"]).sum() > 20
    rng = np.random.default_rng(22)
    G = rng.standard_normal((len(pix), 4))
    safe = (base["margin"] > 1e-3) & (base["flags"] == 0)
    G[~safe] = 0.0
    assert safe.mean() > 0.9
    _, g_ad = og.render_and_grad(sc, cam, pix, G, mesh=mesh)

    def loss(s):
        out = orc.render_pixels(orc.preprocess(s, cam, f64_inputs=True), cam, pix, mesh=mesh)
        return float((out["rgba"] * G).sum())
    h = 1e-6
    for nm in ["means", "log_scales", "opacity_logits", "sh"]:
        arr = getattr(sc, nm)
        flat = arr.reshape(-1)
        idx = rng.choice(flat.size, min(flat.size, 120), replace=False)
        fd = np.zeros(len(idx))
        for j, k in enumerate(idx):
            v = flat[k]
            flat[k] = v + h
            lp = loss(sc)
            flat[k] = v - h
            lm = loss(sc)
            flat[k] = v
            fd[j] = (lp - lm) / (2 * h)
        ad = g_ad[nm].reshape(-1)[idx]
        scale = np.abs(fd).max()
        assert scale > 0, nm
        np.testing.assert_allclose(ad, fd, rtol=1e-5, atol=1e-6 * scale, err_msg=nm)


def test_tiled_gradients_equal_whole_image(orc):
    """The per-tile autograd (each tile's candidates only, gradients summed)
    equals autograd of the whole image at once: the same definition."""
    from oracle import grad as og
    sc, cam = S.fd_scene()
    rng = np.random.default_rng(31)
    G = rng.standard_normal((cam.height, cam.width, 4))
    pix = orc.all_pixels(cam)
    rgba_a, ga = og.render_and_grad(sc, cam, pix, G.reshape(-1, 4))
    for tile in ((16, 16), (8, 8), (32, 8)):
        rgba_b, gb = og.render_and_grad_tiled(sc, cam, G, tile=tile)
        np.testing.assert_allclose(rgba_b.reshape(-1, 4), rgba_a, rtol=0, atol=1e-14)
        for nm in ga:
            scale = max(np.abs(ga[nm]).max(), 1e-300)
            np.testing.assert_allclose(gb[nm] / scale, ga[nm] / scale, rtol=0, atol=1e-12,
                                       err_msg=f"{nm} {tile}")
