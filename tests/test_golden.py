"""The oracle still reproduces its stored regression fixture, and the
paper's Table 1 figures are internally consistent (Total ~ Sort + Prep.+Draw)."""
import json
import os

import numpy as np

from paper_2512_08478_amd import scenes as S

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_oracle_matches_golden(orc):
    g = json.load(open(os.path.join(HERE, "tiny_oracle.json")))
    sc, cam = S.tiny_scene()
    rec = orc.preprocess(sc, cam)
    out = orc.render_pixels(rec, cam, np.array(g["pixels"]))
    np.testing.assert_allclose(out["rgba"], g["rgba"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["T"], g["T"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(out["n_blend"], g["n_blend"])
    gid = np.array(g["gaussians"])
    np.testing.assert_allclose(rec.d[gid][:, [orc.D_MX, orc.D_MY]], g["mean2d"], atol=1e-10)
    np.testing.assert_allclose(rec.d[gid][:, [orc.D_SA, orc.D_SB, orc.D_SC]], g["cov2d"], rtol=1e-10)
    assert int(rec.i[rec.visible, orc.I_TILES].sum()) == g["instances"]


def test_paper_table1_consistent():
    t = json.load(open(os.path.join(HERE, "paper_table1.json")))
    for s, d, tot in zip(t["visionary_sort_ms"], t["visionary_prep_draw_ms"], t["visionary_total_ms"]):
        assert abs(s + d - tot) <= 0.011  # the paper's rounding
