"""GPU tests of mesh depth composition (Algorithm 1's mesh depth prepass
and DrawSplatsWithMeshDepth; Section 3.4).

The mesh prepass is a seeded plane (with holes) seen through the camera;
images are compared with the FP64 oracle composited against the same
depth and colour buffers, gradients with its autograd.
"""
import numpy as np
import pytest
import torch

from paper_2512_08478_amd import scenes as S
from gpu_util import image_check, print_case, sampled_pixels

pytestmark = pytest.mark.gpu
NAMES = ["means", "log_scales", "quats", "opacity_logits", "sh"]


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_08478_amd.render import Renderer
    return Renderer()


def gp(scene):
    from paper_2512_08478_amd.render import GaussianParams
    return GaussianParams.from_scene(scene)


def wall(cam, depths, normal=(0.25, -0.15, 1.0), seed=5, occupancy=0.65):
    """A plane with holes whose median depth is the median Gaussian depth."""
    m = S.plane_mesh(cam, normal, 0.0, seed=seed, occupancy=occupancy)
    fin = np.isfinite(m["depth"])
    m["depth"][fin] += np.float32(np.median(depths) - np.median(m["depth"][fin]))
    return m


def test_mesh_tiny_whole_image(R, orc):
    print_case("mesh composition tiny 256x256 vs brute force")
    sc, cam = S.tiny_scene()
    rec = orc.preprocess(sc, cam)
    mesh = wall(cam, rec.d[rec.visible, orc.D_DEPTH])
    fr = R.forward(gp(sc), cam, mesh=mesh)
    img = fr.image.cpu().numpy().reshape(-1, 4)
    ref = orc.render_image(rec, cam, mesh=mesh)
    flat = {k: v.reshape(-1, 4) if k == "rgba" else v.reshape(-1) for k, v in ref.items()}
    e, nflag, nloose = image_check(img, flat, max_flagged=0.01, max_loosened=0.005,
                                   T=fr.T_final.cpu().numpy().reshape(-1))
    plain = orc.render_image(rec, cam)
    hidden = int((plain["n_blend"] > ref["n_blend"]).sum())
    print(f"tiny mesh max err {e:.2e}, flagged {nflag}, jump above 1e-4 {nloose}, "
          f"pixels with hidden splats {hidden}")
    assert hidden > 1000


def test_mesh_absent_is_bitwise_plain(R):
    print_case("mesh at +inf with the background colour == plain raster, bitwise")
    sc, cam = S.tiny_scene()
    p = gp(sc)
    plain = R.forward(p, cam, reuse=False)
    bg = np.asarray(list(R.settings.bg), np.float32)
    mesh = dict(depth=np.full((cam.height, cam.width), np.inf, np.float32),
                rgb=np.broadcast_to(bg, (cam.height, cam.width, 3)).copy())
    for m in (mesh, dict(depth=mesh["depth"], rgb=None)):
        fr = R.forward(p, cam, reuse=False, mesh=m)
        assert torch.equal(fr.image, plain.image)
        assert torch.equal(fr.last, plain.last)
        assert torch.equal(fr.T_final, plain.T_final)


@pytest.mark.parametrize("shape", [(16, 16, 8), (32, 16, 7), (8, 8, 8)])
def test_mesh_1m_1080p_whole_image(R, orc, shape):
    print_case(f"mesh composition 1M 1920x1080 whole image, tiles {shape[0]}x{shape[1]}")
    from paper_2512_08478_amd.render import Renderer
    from gpu_util import scene_cached
    Rs = Renderer(dict(tile_w=shape[0], tile_h=shape[1], radix_bits=shape[2]))
    sc, cam = scene_cached("medium")
    rec = orc.preprocess(sc, cam)
    mesh = wall(cam, rec.d[rec.visible, orc.D_DEPTH], normal=(0.1, 0.3, 1.0), seed=8)
    fr = Rs.forward(gp(sc), cam, mesh=mesh)
    img = fr.image.cpu().numpy().reshape(-1, 4)
    ref = orc.render_pixels(rec, cam, orc.all_pixels(cam), mesh=mesh, tiled=True)
    e, nflag, nloose = image_check(img, ref, T=fr.T_final.cpu().numpy().reshape(-1))
    nb = torch.empty((cam.height, cam.width), dtype=torch.int32, device="cuda")
    Rs.rasterize(fr.splats, fr.values, fr.ranges, cam, n_blend=nb, mesh=fr.mesh)
    got = nb.cpu().numpy().reshape(-1)
    ok = (ref["margin"] >= 1e-5) & (ref["flags"] == 0)
    np.testing.assert_array_equal(got[ok], ref["n_blend"][ok])
    print(f"1M mesh max err {e:.2e}, flagged {nflag}, jump above 1e-4 {nloose}, "
          f"blended pairs {int(nb.sum())}")


@pytest.mark.parametrize("order", [2, 3, 4, 5])
def test_mesh_row_bands_bitwise(R, orc, order):
    """Mesh composition with each 8x8 quadrant taken in row bands: image,
    T_final, last and blend counts bitwise those of whole quadrants (the
    mesh depth hides splats per pixel, so a band must read its own rows'
    depths)."""
    print_case(f"mesh composition in row bands (raster_order {order}) == whole quadrants")
    from paper_2512_08478_amd.render import Renderer
    sc, _ = S.medium_scene(n=200_000)
    cam = S.orbit_camera(2, 8, 8.0, 1920, 1080)
    rec = orc.preprocess(sc, cam)
    mesh = wall(cam, rec.d[rec.visible, orc.D_DEPTH], normal=(0.1, 0.3, 1.0), seed=8)
    out = []
    for o in (order & 1, order):
        Rs = Renderer(dict(tile_w=8, tile_h=8, raster_order=o))
        fr = Rs.forward(gp(sc), cam, mesh=mesh)
        nb = torch.zeros((cam.height, cam.width), dtype=torch.int32, device="cuda")
        Rs.rasterize(fr.splats, fr.values, fr.ranges, cam, n_blend=nb, mesh=fr.mesh)
        out.append((fr.image, fr.T_final, fr.last, nb))
    for a, b, name in zip(out[0], out[1], ("image", "T_final", "last", "n_blend")):
        assert torch.equal(a, b), name
    assert int(out[0][3].sum()) > 0


def test_mesh_backward_vs_oracle(R, orc):
    print_case("mesh composition backward vs autograd oracle")
    from oracle import grad as og
    sc, cam = S.fd_scene()
    rec = orc.preprocess(sc, cam)
    mesh = wall(cam, rec.d[rec.visible, orc.D_DEPTH], seed=9, occupancy=0.7)
    pix = orc.all_pixels(cam)
    ref = orc.render_pixels(rec, cam, pix, mesh=mesh)
    plain = orc.render_pixels(rec, cam, pix)
    assert (plain["n_blend"] > ref["n_blend"]).sum() > 20
    rng = np.random.default_rng(31)
    G = rng.standard_normal((len(pix), 4))
    G[(ref["margin"] < 1e-4) | (ref["flags"] != 0)] = 0.0
    _, g_ref = og.render_and_grad(sc, cam, pix, G, mesh=mesh)
    p = gp(sc)
    fr = R.forward(p, cam, reuse=False, mesh=mesh)
    g = R.backward(p, cam, fr, torch.from_numpy(G.reshape(cam.height, cam.width, 4)).float().cuda())
    for k, nm in enumerate(NAMES):
        got = g[k].cpu().numpy().astype(np.float64)
        e = np.linalg.norm(got - g_ref[nm]) / max(np.linalg.norm(g_ref[nm]), 1e-30)
        print(f"{nm}: rel L2 {e:.2e}")
        assert e <= 1e-3, (nm, e)


def test_mesh_autograd_function(R):
    print_case("torch.autograd.Function with a mesh prepass")
    from paper_2512_08478_amd.render import GaussianParams, render
    sc, cam = S.fd_scene(n=200, size=48)
    p = GaussianParams.from_scene(sc, requires_grad=True)
    mesh = S.plane_mesh(cam, (0.0, 0.0, 1.0), 0.0, seed=2, occupancy=0.5)
    target = torch.from_numpy(S.random_target(4, cam.height, cam.width)).cuda()
    img = render(p, cam, R, mesh=mesh)
    loss = (img[..., :3] - target).abs().mean()
    loss.backward()
    for t in p.tensors():
        assert t.grad is not None and torch.isfinite(t.grad).all()
    assert float(p.means.grad.abs().sum()) > 0
