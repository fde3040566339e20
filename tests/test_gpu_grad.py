"""GPU backward (hand-written kernels) against the FP64 autograd oracle,
which is itself pinned to central finite differences of the C forward."""
import numpy as np
import pytest
import torch

from paper_2512_08478_amd import scenes as S
from gpu_util import print_case

pytestmark = pytest.mark.gpu
NAMES = ["means", "log_scales", "quats", "opacity_logits", "sh"]


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_08478_amd.render import Renderer
    return Renderer()


def gpu_grads(R, sc, cam, G_img):
    from paper_2512_08478_amd.render import GaussianParams
    p = GaussianParams.from_scene(sc)
    fr = R.forward(p, cam, reuse=False)
    g = R.backward(p, cam, fr, torch.from_numpy(G_img.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return fr, {nm: t.cpu().numpy().astype(np.float64) for nm, t in zip(NAMES, g)}


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def test_backward_fd_instance(R, orc):
    print_case("backward 64 Gaussians 32x32 vs autograd oracle")
    from oracle import grad as og
    sc, cam = S.fd_scene()
    pix = orc.all_pixels(cam)
    ref = orc.render_pixels(orc.preprocess(sc, cam), cam, pix)
    rng = np.random.default_rng(8)
    G = rng.standard_normal((len(pix), 4))
    G[(ref["margin"] < 1e-4) | (ref["flags"] != 0)] = 0.0
    _, g_ref = og.render_and_grad(sc, cam, pix, G)
    G_img = G.reshape(cam.height, cam.width, 4)
    fr, g = gpu_grads(R, sc, cam, G_img)
    for nm in NAMES:
        e = rel_l2(g[nm], g_ref[nm])
        print(f"{nm}: rel L2 {e:.2e}")
        assert e <= 1e-3, (nm, e)


def test_backward_diff_scene_sampled(R, orc):
    print_case("backward 500k 800x800, sparse upstream gradient")
    from oracle import grad as og
    sc, cam = S.diff_scene()
    rng = np.random.default_rng(9)
    pix = np.stack([rng.integers(0, cam.width, 48), rng.integers(0, cam.height, 48)], 1).astype(np.int32)
    pix = np.unique(pix, axis=0)
    ref = orc.render_pixels(orc.preprocess(sc, cam), cam, pix)
    G = rng.standard_normal((len(pix), 4))
    G[(ref["margin"] < 1e-4) | (ref["flags"] != 0)] = 0.0
    G_img = np.zeros((cam.height, cam.width, 4))
    G_img[pix[:, 1], pix[:, 0]] = G
    fr, g = gpu_grads(R, sc, cam, G_img)
    _, g_ref = og.render_and_grad(sc, cam, pix, G)
    for nm in NAMES:
        e = rel_l2(g[nm], g_ref[nm])
        print(f"{nm}: rel L2 {e:.2e}, nonzero rows {np.count_nonzero(np.abs(g_ref[nm]).reshape(sc.n, -1).sum(1))}")
        assert e <= 1e-3, (nm, e)


@pytest.mark.parametrize("shape", [(16, 16, 8, 1), (32, 16, 6, 1), (8, 8, 8, 0)])
def test_backward_dense_upstream(orc, shape):
    """Every pixel of a 256x256 frame of 50k Gaussians carries an upstream
    gradient (except the few whose decisions are near a threshold, where
    the gradient is not defined): many pixels accumulate into each Gaussian
    through the backward's atomics.  Against the per-tile FP64 autograd
    oracle (equal to autograd of the whole image), with the default launch
    configuration, the fwd+bwd benchmark's (32x16 tiles, 6-bit digits) and
    8x8 tiles in spatial order."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_08478_amd.render import Renderer
    R = Renderer(dict(tile_w=shape[0], tile_h=shape[1], radix_bits=shape[2],
                      raster_order=shape[3]))
    print_case(f"backward 50k 256x256, dense upstream gradient, tiles {shape[0]}x{shape[1]}")
    from oracle import grad as og
    sc, cam = S.diff_scene(n=50_000, size=256)
    ref = orc.render_image(orc.preprocess(sc, cam), cam, tiled=True)
    rng = np.random.default_rng(12)
    G = rng.standard_normal((cam.height, cam.width, 4))
    near = (ref["margin"] < 1e-4) | (ref["flags"] != 0)
    G[near] = 0.0
    assert near.mean() < 0.06
    fr, g = gpu_grads(R, sc, cam, G)
    rgba, g_ref = og.render_and_grad_tiled(sc, cam, G, tile=(32, 32))
    np.testing.assert_allclose(rgba, ref["rgba"], rtol=0, atol=1e-12)
    for nm in NAMES:
        e = rel_l2(g[nm], g_ref[nm])
        rows = np.count_nonzero(np.abs(g_ref[nm]).reshape(sc.n, -1).sum(1))
        print(f"{nm}: rel L2 {e:.2e}, Gaussians with a gradient {rows}")
        assert e <= 1e-3, (nm, e)


def test_autograd_function_l1(R):
    print_case("torch.autograd.Function with an L1 loss")
    from paper_2512_08478_amd.render import GaussianParams, render
    sc, cam = S.fd_scene(n=200, size=48)
    p = GaussianParams.from_scene(sc, requires_grad=True)
    target = torch.from_numpy(S.random_target(4, cam.height, cam.width)).cuda()
    img = render(p, cam, R)
    loss = (img[..., :3] - target).abs().mean()
    loss.backward()
    # same gradient through the plain entry points
    G = (torch.sign(img[..., :3] - target) / (3 * cam.height * cam.width)).detach()
    G4 = torch.cat([G, torch.zeros_like(G[..., :1])], -1)
    p2 = GaussianParams.from_scene(sc)
    fr = R.forward(p2, cam, reuse=False)
    g2 = R.backward(p2, cam, fr, G4)
    for a, b in zip(p.tensors(), g2):
        np.testing.assert_allclose(a.grad.cpu().numpy(), b.cpu().numpy(), rtol=1e-5, atol=1e-9)


def test_backward_accumulate(R):
    print_case("backward accumulate flag")
    from paper_2512_08478_amd.render import GaussianParams
    sc, cam = S.fd_scene()
    p = GaussianParams.from_scene(sc)
    fr = R.forward(p, cam, reuse=False)
    G = torch.randn(cam.height, cam.width, 4, device="cuda")
    g1 = R.backward(p, cam, fr, G)
    g1 = [t.clone() for t in g1]
    g2 = R.backward(p, cam, fr, G, out=[t.clone() for t in g1], accumulate=True)
    # the second pass adds a fresh backward whose float atomics may sum in
    # another order, so compare against the magnitude of each gradient
    for name, a, b in zip(("means", "log_scales", "quats", "opacity", "sh"), g1, g2):
        a, b = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
        scale = max(np.abs(a).max(), 1e-30)
        d = np.abs(b - 2 * a).max() / scale
        print(f"{name}: max |g2 - 2 g1| / max |g1| = {d:.2e}")
        assert d <= 1e-5, (name, d)
