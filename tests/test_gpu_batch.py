"""GPU tests of the multi-asset entry points and the batch path.

Multi-asset frames are checked against the FP64 oracle (records, pixels
and gradients).  The batch (gs_batch_*: every view in one preprocess
launch, one global sort, one compositing launch, captured into one HIP
graph) against the plain view-by-view path: images bitwise equal on every
replay, gradients equal up to the order of float atomics; the full batched
workload (4.5M Gaussians, 32 views) also against the oracle; the
autotuner's choice leaves images unchanged.
"""
import numpy as np
import pytest
import torch

from paper_2512_08478_amd import scenes as S
from gpu_util import image_check, print_case, splats_np

pytestmark = pytest.mark.gpu

NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_08478_amd.render import Renderer
    return Renderer()


def small_batch(n_views=4, scale=0.01, seed=6):
    return S.batched_scenes(seed=seed, scale=scale, n_views=n_views, max_wh=(480, 320),
                            min_wh=(160, 128))


def concat_params(assets):
    from paper_2512_08478_amd.render import GaussianParams
    return GaussianParams.concat([GaussianParams.from_scene(a) for a in assets])


def targets_for(cams):
    return [torch.from_numpy(S.random_target(100 + v, c.height, c.width)).cuda()
            for v, c in enumerate(cams)]


def test_multi_asset_records_equal_single_asset_records(R):
    print_case("multi-asset preprocess == per-asset preprocess")
    from paper_2512_08478_amd.render import GaussianParams
    assets, cams = small_batch(n_views=1)
    p = concat_params(assets)
    cam = cams[0]
    splats, _, _, counts = R.preprocess(p, cam, reuse=False)
    rec = splats_np(splats, p.n)
    c_all = counts.cpu().numpy().view(np.uint32)
    tot = np.zeros(2, np.int64)
    kmin, kmax = 0xFFFFFFFF, 0
    off = 0
    for a in assets:
        s1, _, _, c1 = R.preprocess(GaussianParams.from_scene(a), cam, reuse=False)
        r1 = splats_np(s1, a.n)
        assert r1.tobytes() == rec[off:off + a.n].tobytes()
        c1 = c1.cpu().numpy().view(np.uint32)
        tot += c1[:2]
        kmin, kmax = min(kmin, int(c1[2])), max(kmax, int(c1[3]))
        off += a.n
    assert list(tot) == list(c_all[:2])
    assert (kmin, kmax) == (int(c_all[2]), int(c_all[3]))
    print(f"{len(assets)} assets, {p.n} Gaussians, instances {c_all[0]}, visible {c_all[1]}")


def test_multi_asset_view_vs_oracle(R, orc):
    print_case("multi-asset view vs oracle, whole images")
    assets, cams = small_batch(n_views=2)
    p = concat_params(assets)
    for cam in cams:
        fr = R.forward(p, cam)
        img = fr.image.cpu().numpy()
        ref = orc.render_pixels(orc.preprocess_many(assets, cam), cam, orc.all_pixels(cam),
                                tiled=True)
        e, nflag, nloose = image_check(img.reshape(-1, 4), ref,
                                       T=fr.T_final.cpu().numpy().reshape(-1))
        assert ref["rgba"][:, 3].max() > 0.1
        print(f"{cam.width}x{cam.height}: max err {e:.2e}, flagged {nflag}, jump above 1e-4 {nloose}")


def test_multi_asset_backward_vs_oracle(R, orc):
    print_case("multi-asset backward vs autograd oracle")
    from scipy.spatial.transform import Rotation
    from oracle import grad as og
    from paper_2512_08478_amd.render import GaussianParams
    sc, cam = S.fd_scene()
    A = 0.9 * Rotation.from_euler("xyz", [0.1, -0.4, 0.25]).as_matrix()
    model = np.concatenate([A, np.array([[0.05], [0.1], [-0.2]])], 1)
    h = sc.n // 2
    part = lambda sl, m: S.Scene(*(np.ascontiguousarray(getattr(sc, k)[sl]) for k in NAMES),
                                 sc.sh_degree, m)
    assets = [part(slice(0, h), None), part(slice(h, None), model)]
    pix = orc.all_pixels(cam)
    ref = orc.render_pixels(orc.preprocess_many(assets, cam), cam, pix)
    rng = np.random.default_rng(12)
    G = rng.standard_normal((len(pix), 4))
    G[(ref["margin"] < 1e-4) | (ref["flags"] != 0)] = 0.0
    _, g_ref = og.render_and_grad_assets(assets, cam, pix, G)
    p = GaussianParams.concat([GaussianParams.from_scene(a) for a in assets])
    fr = R.forward(p, cam, reuse=False)
    g = R.backward(p, cam, fr, torch.from_numpy(G.reshape(cam.height, cam.width, 4)).float().cuda())
    for k, nm in enumerate(NAMES):
        got = g[k].cpu().numpy().astype(np.float64)
        want = np.concatenate([g_ref[0][nm], g_ref[1][nm]])
        e = np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-30)
        print(f"{nm}: rel L2 {e:.2e}")
        assert e <= 1e-3, (nm, e)


def _rel_max(a, b):
    a, b = a.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)


def test_graph_batch_matches_plain_views_on_every_replay(R):
    print_case("graph-captured batch vs plain views, 3 replays")
    from paper_2512_08478_amd.batch import BatchRenderer, plain_views
    assets, cams = small_batch(n_views=4)
    p = concat_params(assets)
    tg = targets_for(cams)
    imgs_ref, grads_ref = plain_views(p, cams, tg)
    br = BatchRenderer(p, cams, tg)
    br.capture()
    noise = torch.randn(512, 512, device="cuda")
    for rep in range(3):
        imgs = br.replay()
        for v in range(len(cams)):
            assert torch.equal(imgs[v], imgs_ref[v]), (rep, v)
        for k, nm in enumerate(NAMES):
            d = _rel_max(br.grads[k], grads_ref[k])
            assert d <= 1e-5, (rep, nm, d)
        # the program's own eager work between replays
        noise = (noise @ noise.T).tanh_()
        torch.cuda.synchronize()
    # the eager run gives the same images
    again = [im.clone() for im in br.run_eager()]
    for v in range(len(cams)):
        assert torch.equal(again[v], imgs_ref[v])
    print(f"{len(cams)} views, {p.n} Gaussians, capacity {br.capacity}")


@pytest.mark.parametrize("shape", [(8, 8, 8, 0, 1), (32, 16, 6, 1, 0), (64, 32, 7, 0, 1),
                                   (16, 8, 8, 0, 3), (32, 16, 7, 1, 2)])
def test_batch_settings_forward_only(R, shape):
    """A forward-only batch (no targets) in several tile shapes, digit
    widths, sort modes and orders: images bitwise equal to plain views."""
    tw, th, bits, mode, order = shape
    print_case(f"forward-only batch, tiles {tw}x{th}, {bits}-bit, mode {mode}, order {order}")
    from paper_2512_08478_amd.batch import BatchRenderer, plain_views
    from paper_2512_08478_amd.render import Renderer
    st = dict(tile_w=tw, tile_h=th, radix_bits=bits, sort_mode=mode, raster_order=order)
    assets, cams = small_batch(n_views=5, seed=9)
    p = concat_params(assets)
    imgs_ref, _ = plain_views(p, cams, None, renderer=Renderer(st))
    br = BatchRenderer(p, cams, None, st)
    br.capture()
    imgs = br.replay()
    for v in range(len(cams)):
        assert torch.equal(imgs[v], imgs_ref[v]), v


def test_batch_capacity_overflow_is_reported(R):
    """Parameters updated after planning so that the batch needs more
    instances than planned: the status flag reports it."""
    print_case("batched capacity overflow flag")
    from paper_2512_08478_amd.batch import BatchRenderer
    assets, cams = small_batch(n_views=2)
    p = concat_params(assets)
    br = BatchRenderer(p, cams, targets_for(cams), headroom=1.0)
    br.plan()
    br.run_eager()
    torch.cuda.synchronize()
    br._check_flags()
    with torch.no_grad():
        p.log_scales.add_(1.5)     # every footprint grows: more tiles per Gaussian
    br.run_eager()
    torch.cuda.synchronize()
    with pytest.raises(RuntimeError, match="capacity"):
        br._check_flags()
    br.plan()                      # planned again: fits
    br.run_eager()
    torch.cuda.synchronize()
    br._check_flags()


def test_autotuned_settings_leave_images_unchanged(R):
    print_case("gs_autotune: tile shape / digit width / sort mode / order choice keeps images")
    from paper_2512_08478_amd.batch import BatchRenderer, autotune
    assets, cams = small_batch(n_views=2)
    p = concat_params(assets)
    tg = targets_for(cams)
    best, ms, nev = autotune(p, cams, tg, reps=1, tiles=((16, 16), (8, 8), (32, 8)), bits=(8, 6),
                             modes=(0, 1), orders=(1, 0))
    assert nev == 1 + 2 + 1 + 1 + 1 and ms > 0
    ref = BatchRenderer(p, cams, tg)
    ref_imgs = [im.clone() for im in ref.run_eager()]
    tuned = BatchRenderer(p, cams, tg, best)
    imgs = tuned.run_eager()
    for a, b in zip(imgs, ref_imgs):
        assert torch.equal(a, b)
    print(f"autotune picked {best} at {ms:.3f} ms per batch")


def test_full_batched_workload(R, orc):
    """The batched workload itself (2M scene + 8 placed assets, 4.5M
    Gaussians; 32 views of uneven size): the graph-captured batch equals
    the plain view-by-view path (images bitwise, gradients up to the order
    of float atomics), and two views against the tiled FP64 oracle, every
    pixel."""
    print_case("full batch: 4.5M Gaussians x 32 views, graph vs plain views and oracle")
    from paper_2512_08478_amd.batch import BatchRenderer, plain_views
    from paper_2512_08478_amd.render import Renderer
    assets, cams = S.batched_scenes()
    p = concat_params(assets)
    tg = targets_for(cams)
    st = dict(tile_w=16, tile_h=16, radix_bits=8)
    br = BatchRenderer(p, cams, tg, st)
    br.capture()
    imgs = [im.clone() for im in br.replay()]
    grads = [g.clone() for g in br.grads]
    imgs_ref, grads_ref = plain_views(p, cams, tg, renderer=Renderer(st))
    for v in range(len(cams)):
        assert torch.equal(imgs[v], imgs_ref[v]), v
    for k, nm in enumerate(NAMES):
        d = _rel_max(grads[k], grads_ref[k])
        print(f"{nm}: max |batch - plain| / max |plain| = {d:.2e}")
        assert d <= 1e-5, (nm, d)
    for v in (0, 17):
        cam = cams[v]
        ref = orc.render_pixels(orc.preprocess_many(assets, cam), cam, orc.all_pixels(cam),
                                tiled=True)
        e, nflag, nloose = image_check(imgs[v].cpu().numpy().reshape(-1, 4), ref)
        print(f"view {v} {cam.width}x{cam.height}: max err {e:.2e}, flagged {nflag}, "
              f"jump above 1e-4 {nloose}")
    print(f"{len(cams)} views, {p.n} Gaussians, {br.pixels} pixels, capacity {br.capacity}")


def test_multi_view_backward_matches_per_view_backward(R):
    print_case("multi-view chain rule (10 views, two launches) vs per-view backward")
    from paper_2512_08478_amd.batch import l1_grad
    assets, cams = S.batched_scenes(seed=7, scale=0.004, n_views=10, max_wh=(200, 160),
                                    min_wh=(96, 80))
    p = concat_params(assets)
    tg = targets_for(cams)
    ref = tuple(torch.zeros_like(t) for t in p.tensors())
    g2d = []
    for v, cam in enumerate(cams):
        fr = R.forward(p, cam, reuse=False)
        g = l1_grad(fr.image, tg[v])
        R.backward(p, cam, fr, g, out=ref, accumulate=v > 0)
        g2d.append(R.backward_2d(p, cam, fr, g))
    got = R.backward_views(p, cams, g2d)
    for k, nm in enumerate(NAMES):
        d = _rel_max(got[k], ref[k])
        print(f"{nm}: max |views - per view| / max |per view| = {d:.2e}")
        assert d <= 1e-5, (nm, d)
    # accumulate adds onto what is there
    again = R.backward_views(p, cams, g2d, out=tuple(t.clone() for t in got), accumulate=True)
    for k in range(5):
        assert _rel_max(again[k], 2 * got[k]) <= 1e-6
