"""GPU tests of the linear-blend-skinning pre-decoder (Section 3.3,
Eqs. 5-6) on pre-packed Gaussians: bit-exact against the oracle's single
float64 -> binary16 rounding, the identity pose leaves the packed data and
the rendered image bit-identical, and a posed frame matches the oracle."""
import numpy as np
import pytest
import torch

from paper_2512_08478_amd import scenes as S
from gpu_util import image_check, near_tie, print_case, sampled_pixels, scene_cached

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_08478_amd.render import Renderer
    return Renderer()


def halves(t):
    return t.cpu().numpy().view(np.float16)


def decoded(pk):
    K3 = 3 * (pk.sh_degree + 1) ** 2
    return dict(means=halves(pk.posop)[:, :3], opacity=halves(pk.posop)[:, 3],
                cov6=halves(pk.cov), sh=halves(pk.sh16)[:, :K3].reshape(pk.n, -1, 3),
                sh_degree=pk.sh_degree, model=None)


def avatar(n, n_joints=55, seed=0, pose_seed=1, R=None):
    from paper_2512_08478_amd.render import GaussianParams
    sc, cam = S.medium_scene(n=n)
    centres, idx, w = S.skinning(sc.means, n_joints=n_joints, seed=seed)
    joints = S.joint_pose(centres, seed=pose_seed)
    canon = R.prepack(GaussianParams.from_scene(sc))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return sc, cam, canon, (dev(idx), dev(w), dev(joints)), (idx, w, joints)


def test_lbs_bitexact_vs_oracle(R, orc):
    print_case("lbs deform 100k Gaussians, 55 joints, bit-exact")
    sc, cam, canon, (di, dw, dj), (idx, w, joints) = avatar(100_003, R=R)
    out = R.lbs_deform(canon, di, dw, dj)
    torch.cuda.synchronize()
    c = decoded(canon)
    ref = orc.lbs_deform(c, idx, w, joints)
    exact = orc.lbs_deform(c, idx, w, joints, rounded=False)
    rowmax = lambda a: np.abs(np.asarray(a, np.float64)).max(1, keepdims=True)
    mscale = rowmax(c["means"]) + np.abs(joints[:, :, 3]).max()
    for got, want, x, sc_, nm in (
            (halves(out.posop)[:, :3], ref["means"], exact["means"], mscale, "means"),
            (halves(out.cov), ref["cov6"], exact["cov6"], rowmax(exact["cov6"]), "cov")):
        diff = got.view(np.uint16) != want.view(np.uint16)
        tie = near_tie(x, want, sc_)
        assert not (diff & ~tie).any(), (nm, np.argwhere(diff & ~tie)[:5])
        print(f"{nm}: differing {int(diff.sum())}, float64 ties {int(tie.sum())}")
    # opacity bits copied
    np.testing.assert_array_equal(halves(out.posop)[:, 3].view(np.uint16),
                                  halves(canon.posop)[:, 3].view(np.uint16))
    moved = np.abs(halves(out.posop)[:, :3].astype(np.float64) - c["means"].astype(np.float64)).max()
    assert moved > 0.05


def test_lbs_identity_pose_bit_identical(R):
    print_case("lbs identity pose: packed data and image bit-identical")
    sc, cam, canon, (di, dw, dj), _ = avatar(200_000, pose_seed=None, R=R)
    out = R.lbs_deform(canon, di, dw, dj)
    # equal as numbers: a canonical -0 may come back as +0 (sums of zeros)
    for a, b in ((out.posop, canon.posop), (out.cov, canon.cov)):
        x, y = halves(a), halves(b)
        assert np.array_equal(x, y)
        assert np.array_equal(x.view(np.uint16)[x != 0], y.view(np.uint16)[y != 0])
    a = R.forward(canon, cam, reuse=False).image
    b = R.forward(out, cam, reuse=False).image
    assert torch.equal(a, b)


def test_lbs_index_past_last_joint_contributes_nothing(R, orc):
    print_case("lbs: joint index >= n_joints contributes nothing")
    sc, cam, canon, (di, dw, dj), (idx, w, joints) = avatar(20_000, n_joints=30, R=R)
    idx = idx.copy()
    idx[::3, 3] = 200                       # past the 30 joints
    out = R.lbs_deform(canon, torch.from_numpy(idx).cuda(), dw, dj)
    w0 = w.copy()
    w0[::3, 3] = 0.0
    ref = orc.lbs_deform(decoded(canon), np.minimum(idx, 29), w0, joints)
    exact = orc.lbs_deform(decoded(canon), np.minimum(idx, 29), w0, joints, rounded=False)
    diff = halves(out.posop)[:, :3].view(np.uint16) != ref["means"].view(np.uint16)
    scale = np.abs(decoded(canon)["means"].astype(np.float64)).max(1, keepdims=True) + 1.0
    assert not (diff & ~near_tie(exact["means"], ref["means"], scale)).any()


@pytest.mark.parametrize("n", [20_000, 1_000_000])
def test_lbs_posed_frame_vs_oracle(R, orc, n):
    # camera in general position (binary16 means seen along an axis give
    # exactly equal depths; see the packed end-to-end test)
    print_case(f"lbs posed frame, {n} Gaussians, 1920x1080, sampled pixels")
    sc, _, canon, (di, dw, dj), _ = avatar(n, R=R)
    cam = S.pinhole_camera(S.look_at((2.3, 1.7, -8.1)), 1920, 1080, 60.0)
    out = R.lbs_deform(canon, di, dw, dj)
    fr = R.forward(out, cam)
    img = fr.image.cpu().numpy()
    pix = sampled_pixels(cam, 256, 23)
    ref = orc.render_pixels(orc.preprocess_packed(decoded(out), cam), cam, pix)
    e, nflag, _ = image_check(img[pix[:, 1], pix[:, 0]], ref, max_flagged=0.15, max_loosened=0.05)
    assert ref["rgba"][:, 3].max() > 0.1
    print(f"posed max err {e:.2e}, flagged {nflag}")


def test_lbs_posed_frame_end_to_end(R, orc):
    """The avatar frame, every pixel, against the oracle's own chain:
    oracle pre-pack -> oracle skinning (Eqs. 5-6, float64, one rounding) ->
    projection from the posed packed values -> tiled Eq. 3.  The GPU's
    posed bits must equal the oracle's.  Camera in general position (see
    the packed end-to-end test)."""
    print_case("lbs posed 1M frame end to end, whole image")
    from paper_2512_08478_amd.render import GaussianParams
    sc, _ = scene_cached("medium")
    cam = S.pinhole_camera(S.look_at((2.3, 1.7, -8.1)), 1920, 1080, 60.0)
    centres, idx, w = S.skinning(sc.means, n_joints=55, seed=0)
    joints = S.joint_pose(centres, seed=1)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    canon = R.prepack(GaussianParams.from_scene(sc))
    out = R.lbs_deform(canon, dev(idx), dev(w), dev(joints))
    fr = R.forward(out, cam)
    img = fr.image.cpu().numpy().reshape(-1, 4)
    posed = orc.lbs_deform(orc.prepack(sc), idx, w, joints)
    got = decoded(out)
    for k in ("means", "opacity", "cov6", "sh"):
        a = np.asarray(got[k]).reshape(-1).view(np.uint16)
        b = np.asarray(posed[k]).reshape(-1).view(np.uint16)
        assert np.array_equal(a, b), (k, int((a != b).sum()))
    ref = orc.render_pixels(orc.preprocess_packed(posed, cam), cam, orc.all_pixels(cam), tiled=True)
    e, nflag, nloose = image_check(img, ref, T=fr.T_final.cpu().numpy().reshape(-1))
    print(f"avatar end to end: max err {e:.2e}, flagged {nflag}, jump above 1e-4 {nloose}")
