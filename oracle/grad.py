"""Reference gradients by float64 automatic differentiation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper notes that the splatting formulation of Eqs. 1-3 is
differentiable (Section 3.2).  This module writes the same forward
definition as ``gs_oracle.cpp`` with plain PyTorch CPU float64 tensor ops
and lets autograd differentiate it.  Every discrete decision (culls, the
pixel skip alpha < tau, the stop at T < t_eps) is taken in a no-grad pass
and then held fixed, so the result is the gradient of the piecewise-smooth
forward at the given point; the clamps (alpha_max, the J clamp, colour at
0) pass zero gradient where they bind.  Tests pin it against central finite
differences of the C forward, which is a separate implementation.

Only the Gaussians that blend into at least one requested pixel enter the
autograd graph; every other Gaussian has an exactly zero gradient for
those pixels.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import DEFAULT_SETTINGS

_F = torch.float64


def _settings(settings):
    s = dict(DEFAULT_SETTINGS)
    if settings:
        s.update(settings)
    return s


def sh_basis_t(degree: int, d: torch.Tensor) -> torch.Tensor:
    """Real SH basis (same convention as the C oracle) on unit rows of d."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    out = [torch.full_like(x, 0.5 * math.sqrt(1.0 / math.pi))]
    if degree >= 1:
        c1 = math.sqrt(3.0 / (4.0 * math.pi))
        out += [-c1 * y, c1 * z, -c1 * x]
    if degree >= 2:
        a, b, c = 0.5 * math.sqrt(15 / math.pi), 0.25 * math.sqrt(5 / math.pi), 0.25 * math.sqrt(15 / math.pi)
        out += [a * x * y, -a * y * z, b * (2 * z * z - x * x - y * y), -a * x * z, c * (x * x - y * y)]
    if degree >= 3:
        a = 0.25 * math.sqrt(35 / (2 * math.pi))
        b = 0.5 * math.sqrt(105 / math.pi)
        c = 0.25 * math.sqrt(21 / (2 * math.pi))
        e = 0.25 * math.sqrt(7 / math.pi)
        f = 0.25 * math.sqrt(105 / math.pi)
        out += [-a * y * (3 * x * x - y * y), b * x * y * z, -c * y * (4 * z * z - x * x - y * y),
                e * z * (2 * z * z - 3 * x * x - 3 * y * y), -c * x * (4 * z * z - x * x - y * y),
                f * z * (x * x - y * y), -a * x * (x * x - 3 * y * y)]
    return torch.stack(out, 1)


def _rot(q):
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    return torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], 1).reshape(-1, 3, 3)


def project(means, log_scales, quats, logits, sh, degree, model, cam, settings=None):
    """Eq. 1 and the colour for a set of Gaussians (float64 tensors).

    Returns mean2d (N,2), conic (N,3) = (A, B, C) of S^-1, opacity (N,),
    rgb (N,3), depth (N,), and a bool mask of the culls that change the
    image (near plane, opacity, degenerate or non-finite values)."""
    st = _settings(settings)
    V = torch.as_tensor(np.asarray(cam.viewmat, np.float64).reshape(4, 4), dtype=_F)
    s = torch.exp(log_scales)
    qn = quats / torch.linalg.norm(quats, dim=1, keepdim=True)
    o = torch.sigmoid(logits)
    R = _rot(qn)
    M = R * s[:, None, :]
    Sig = M @ M.transpose(1, 2)
    if model is not None:
        Mk = torch.as_tensor(np.asarray(model, np.float64), dtype=_F)
        A, tk = Mk[:, :3], Mk[:, 3]
        sk = torch.linalg.det(A) ** (1.0 / 3.0)
        Rk = A / sk
    else:
        A, tk, Rk = torch.eye(3, dtype=_F), torch.zeros(3, dtype=_F), torch.eye(3, dtype=_F)
    muw = means @ A.T + tk
    Sigw = A @ Sig @ A.T
    W, Vt = V[:3, :3], V[:3, 3]
    t = muw @ W.T + Vt
    tz = t[:, 2]
    limx = st["clip"] * (0.5 * cam.width) / cam.fx
    limy = st["clip"] * (0.5 * cam.height) / cam.fy
    xt = torch.clamp(t[:, 0] / tz, -limx, limx)
    yt = torch.clamp(t[:, 1] / tz, -limy, limy)
    zero = torch.zeros_like(tz)
    J = torch.stack([torch.stack([cam.fx / tz, zero, -cam.fx * xt / tz], 1),
                     torch.stack([zero, cam.fy / tz, -cam.fy * yt / tz], 1)], 1)
    Sc = W @ Sigw @ W.T
    S2 = J @ Sc @ J.transpose(1, 2)
    a = S2[:, 0, 0] + st["eps2d"]
    b = 0.5 * (S2[:, 0, 1] + S2[:, 1, 0])
    c = S2[:, 1, 1] + st["eps2d"]
    det = a * c - b * b
    conic = torch.stack([c / det, -b / det, a / det], 1)
    mean2d = torch.stack([cam.fx * t[:, 0] / tz + cam.cx, cam.fy * t[:, 1] / tz + cam.cy], 1)
    campos = -(W.T @ Vt)
    dvec = muw - campos
    dvec = dvec / torch.linalg.norm(dvec, dim=1, keepdim=True)
    dl = dvec @ Rk  # R_k^T d per row
    Y = sh_basis_t(degree, dl)
    rgb = torch.clamp(torch.einsum("nk,nkc->nc", Y, sh) + 0.5, min=0.0)
    with torch.no_grad():
        ok = (tz > cam.znear) & (o >= st["tau"]) & (det > 0)
        ok &= torch.isfinite(conic).all(1) & torch.isfinite(mean2d).all(1) & torch.isfinite(rgb).all(1)
    return dict(mean2d=mean2d, conic=conic, opacity=o, rgb=rgb, depth=tz, ok=ok)


def _weights(p, px, py):
    dx = px[:, None] - p["mean2d"][None, :, 0]
    dy = py[:, None] - p["mean2d"][None, :, 1]
    cA, cB, cC = p["conic"][:, 0], p["conic"][:, 1], p["conic"][:, 2]
    Q = cA[None] * dx * dx + 2 * cB[None] * dx * dy + cC[None] * dy * dy
    return p["opacity"][None] * torch.exp(-0.5 * Q)


def _blend_masks(g, st):
    """Which (pixel, Gaussian) pairs blend, Gaussians in blend order."""
    a = torch.clamp(g, max=st["alpha_max"])
    m = a >= st["tau"]
    Tafter = torch.cumprod(1.0 - a * m, dim=1)
    stopped = Tafter < st["t_eps"]
    # blended up to and including the first entry with T < t_eps
    before_stop = torch.cumsum(stopped.to(torch.int64), 1) - stopped.to(torch.int64) == 0
    return m & before_stop


def scene_tensors(scene, requires_grad=True):
    f = lambda a: torch.tensor(np.asarray(a, np.float64), dtype=_F, requires_grad=requires_grad)
    return [f(scene.means), f(scene.log_scales), f(scene.quats), f(scene.opacity_logits),
            f(scene.sh)]


def render_and_grad(scene, cam, pix, dL_drgba, settings=None, chunk=64, mesh=None):
    """rgba at ``pix`` (P,4) and d(sum dL_drgba * rgba)/d(inputs).

    Returns (rgba numpy (P,4), dict of float64 numpy gradients with keys
    means, log_scales, quats, opacity_logits, sh)."""
    rgba, grads = render_and_grad_assets([scene], cam, pix, dL_drgba, settings, chunk, mesh)
    return rgba, grads[0]


def render_and_grad_assets(scenes, cam, pix, dL_drgba, settings=None, chunk=64, mesh=None):
    """As render_and_grad for several assets rendered together: every asset
    is projected with its own model transform and all visible Gaussians are
    composited in one global (depth, global index) order, the global index
    running over the assets in list order (Algorithm 1's single sort over
    all models).  ``mesh`` ({depth: (H,W), rgb: (H,W,3) or None}) hides the
    Gaussians deeper than the mesh at each pixel and puts the mesh colour
    behind the rest (Section 3.4); the mesh itself is not differentiated.
    Returns (rgba (P,4), [gradient dict per asset])."""
    from . import mesh_at
    st = _settings(settings)
    pix = np.asarray(pix, np.int64).reshape(-1, 2)
    md, mr = mesh_at(mesh, pix)
    if md is None:
        md = np.full(len(pix), np.inf)
    G = torch.as_tensor(np.asarray(dL_drgba, np.float64).reshape(-1, 4), dtype=_F)
    params = [scene_tensors(sc) for sc in scenes]
    offs = np.cumsum([0] + [sc.n for sc in scenes])
    with torch.no_grad():
        ps = [project(*params[a], sc.sh_degree, sc.model, cam, st) for a, sc in enumerate(scenes)]
        p = {k: torch.cat([q[k] for q in ps]) for k in ps[0]}
        vis = torch.nonzero(p["ok"]).flatten().numpy()
        depth = p["depth"].numpy()
        order = vis[np.lexsort((vis, depth[vis]))]
        pord = {k: v[order] for k, v in p.items() if k != "ok"}
        masks = []
        used = np.zeros(len(order), bool)
        for s0 in range(0, len(pix), chunk):
            pp = torch.as_tensor(pix[s0:s0 + chunk] + 0.5, dtype=_F)
            # in front of (or at) the mesh; in depth order, so the first
            # hidden Gaussian hides every later one
            front = pord["depth"][None, :] <= torch.as_tensor(md[s0:s0 + chunk], dtype=_F)[:, None]
            m = _blend_masks(_weights(pord, pp[:, 0], pp[:, 1]) * front, st)
            masks.append(m)
            used |= m.any(0).numpy()
        cols = np.nonzero(used)[0]
        mask = torch.cat(masks, 0)[:, torch.as_tensor(cols)] if len(cols) else torch.zeros((len(pix), 0), dtype=torch.bool)
    gsel = order[cols]  # global indices of the blending Gaussians, in blend order
    parts = []
    for a, sc in enumerate(scenes):
        loc = gsel[(gsel >= offs[a]) & (gsel < offs[a + 1])] - offs[a]
        if len(loc) == 0:
            continue
        sel = torch.as_tensor(loc, dtype=torch.int64)
        sub = [t.index_select(0, sel) for t in params[a]]
        parts.append((offs[a] + loc, project(*sub, sc.sh_degree, sc.model, cam, st)))
    if parts:
        # back to blend order
        gidx = np.concatenate([g for g, _ in parts])
        q = {k: torch.cat([d[k] for _, d in parts]) for k in ("mean2d", "conic", "opacity", "rgb")}
        where = {int(g): i for i, g in enumerate(gidx)}
        perm = torch.as_tensor([where[int(g)] for g in gsel], dtype=torch.int64)
        q = {k: v.index_select(0, perm) for k, v in q.items()}
    else:
        q = {"mean2d": torch.zeros((0, 2), dtype=_F), "conic": torch.zeros((0, 3), dtype=_F),
             "opacity": torch.zeros(0, dtype=_F), "rgb": torch.zeros((0, 3), dtype=_F)}
    pp = torch.as_tensor(pix + 0.5, dtype=_F)
    a = torch.clamp(_weights(q, pp[:, 0], pp[:, 1]), max=st["alpha_max"]) * mask
    one_m = 1.0 - a
    Tb = torch.cat([torch.ones((len(pix), 1), dtype=_F), torch.cumprod(one_m, 1)[:, :-1]], 1)
    C = torch.einsum("pn,nc->pc", a * Tb, q["rgb"])
    Tf = torch.prod(one_m, 1)
    if mr is None:
        bg = torch.as_tensor(np.asarray(st["bg"], np.float64), dtype=_F)[None]
    else:
        bg = torch.as_tensor(mr, dtype=_F)
    rgba = torch.cat([C + Tf[:, None] * bg, (1.0 - Tf)[:, None]], 1)
    L = (G * rgba).sum()
    flat = [t for ts in params for t in ts]
    grads = torch.autograd.grad(L, flat, allow_unused=True) if L.requires_grad else [None] * len(flat)
    names = ["means", "log_scales", "quats", "opacity_logits", "sh"]
    out = []
    for a in range(len(scenes)):
        d = {}
        for k, nm in enumerate(names):
            g, t = grads[5 * a + k], params[a][k]
            d[nm] = np.zeros(t.shape) if g is None else g.detach().numpy()
        out.append(d)
    return rgba.detach().numpy(), out


def render_and_grad_tiled(scene, cam, dL_dimage, settings=None, tile=(16, 16)):
    """render_and_grad over the whole image, one tile at a time.

    ``dL_dimage`` is the (H,W,4) upstream gradient.  A pixel's composite
    involves only Gaussians whose weight reaches tau there, i.e. whose exact
    support bbox (the oracle's pixel bbox) overlaps the pixel's tile; every
    other Gaussian is skipped by the definition and receives no gradient
    from that pixel.  So each tile is render_and_grad of its candidates
    (kept in global index order, so equal depths still break ties by
    index), and the loss gradient is the sum of the tiles' gradients.
    Returns (rgba (H,W,4), gradient dict) like render_and_grad."""
    from . import I_PX0, I_PX1, I_PY0, I_PY1, all_pixels, preprocess
    tw, th = tile
    H, W = cam.height, cam.width
    G = np.asarray(dL_dimage, np.float64).reshape(H, W, 4)
    recs = preprocess(scene, cam, settings)
    vis = np.nonzero(recs.visible)[0]
    iv = recs.i[vis]
    tx0, tx1 = iv[:, I_PX0] // tw, iv[:, I_PX1] // tw
    ty0, ty1 = iv[:, I_PY0] // th, iv[:, I_PY1] // th
    grads = {nm: np.zeros(np.asarray(a).shape) for nm, a in
             zip(("means", "log_scales", "quats", "opacity_logits", "sh"),
                 (scene.means, scene.log_scales, scene.quats, scene.opacity_logits, scene.sh))}
    rgba = np.zeros((H, W, 4))
    st = _settings(settings)
    pix_all = all_pixels(cam).reshape(H, W, 2)
    for ty in range(-(-H // th)):
        for tx in range(-(-W // tw)):
            ys, xs = slice(ty * th, min(H, (ty + 1) * th)), slice(tx * tw, min(W, (tx + 1) * tw))
            pix = pix_all[ys, xs].reshape(-1, 2)
            cand = vis[(tx0 <= tx) & (tx <= tx1) & (ty0 <= ty) & (ty <= ty1)]
            if cand.size == 0:
                rgba[ys, xs, :3] = st["bg"]
                continue
            sub = scene.subset(cand)
            out, g = render_and_grad(sub, cam, pix, G[ys, xs].reshape(-1, 4), settings)
            rgba[ys, xs] = out.reshape(ys.stop - ys.start, xs.stop - xs.start, 4)
            for nm in grads:
                np.add.at(grads[nm], cand, g[nm])
    return rgba, grads
