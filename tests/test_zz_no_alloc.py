"""The allocation-free preprocess (gs_preprocess_noalloc, its scratch in a
static device array inside the library) against the workspace variant
(gs_preprocess) through the C ABI: bitwise equal records, depth keys, tile
rects and counts, on two calls in a row, the second with a smaller input
(the scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2512_08478_amd import _lib as L
from paper_2512_08478_amd import scenes as S

pytestmark = pytest.mark.gpu


def run(lib, sc, cam, noalloc):
    from paper_2512_08478_amd.render import GaussianParams
    p = GaussianParams.from_scene(sc)
    n = p.n
    s = L.default_settings()
    c = L.make_camera(cam)
    dev = dict(device="cuda")
    splats = torch.full((max(n, 1) * L.SPLAT_BYTES,), 0x5A, dtype=torch.uint8, **dev)
    dkeys = torch.full((max(n, 1),), -1, dtype=torch.int32, **dev)
    rects = torch.full((max(2 * n, 2),), -1, dtype=torch.int32, **dev)
    counts = torch.full((4,), -1, dtype=torch.int32, **dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    ins = [ptr(t) for t in p.tensors()]
    if noalloc:
        st = lib.gs_preprocess_noalloc(n, *ins, p.sh_degree, L.model_array(p.model), ctypes.byref(c),
                                       ctypes.byref(s), ptr(splats), ptr(dkeys), ptr(rects),
                                       ptr(counts), stream)
    else:
        wsb = lib.gs_workspace_size(L.GS_STAGE_PREPROCESS, n, 0, ctypes.byref(c), ctypes.byref(s))
        ws = torch.empty(wsb, dtype=torch.uint8, **dev)
        st = lib.gs_preprocess(n, *ins, p.sh_degree, L.model_array(p.model), ctypes.byref(c),
                               ctypes.byref(s), ptr(splats), ptr(dkeys), ptr(rects), ptr(counts),
                               ptr(ws), wsb, stream)
    L.check(st, "gs_preprocess_noalloc" if noalloc else "gs_preprocess")
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in (splats, dkeys, rects, counts)]


def test_noalloc_equals_workspace_variant():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = L.load()
    big = S.medium_scene(n=1_000_000)
    small = S.tiny_scene()
    for (sc, cam), name in ((big, "1M, 1920x1080"), (small, "4096, 256x256")):
        print(f"[gpu case] gs_preprocess_noalloc vs gs_preprocess, {name}", flush=True)
        want = run(lib, sc, cam, noalloc=False)
        got = run(lib, sc, cam, noalloc=True)
        for a, b, what in zip(got, want, ("records", "depth keys", "tile rects", "counts")):
            np.testing.assert_array_equal(a, b, err_msg=what)
        c = got[3].view(np.uint32)
        assert c[1] > 0 and c[0] >= c[1]
        print(f"instances {c[0]}, visible {c[1]}", flush=True)
