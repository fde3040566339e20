"""Write the oracle regression fixtures in this folder.

Calls only the oracle and the seeded input generator.  The stored values
pin the oracle against silent drift: a later change to its arithmetic
must also regenerate these files, in a commit that names the passage of
the paper (or the reading of it) that justifies the change.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2512_08478_amd import scenes as S  # noqa: E402


def main():
    sc, cam = S.tiny_scene()
    rec = oracle.preprocess(sc, cam)
    rng = np.random.default_rng(2024)
    pix = np.stack([rng.integers(0, cam.width, 64), rng.integers(0, cam.height, 64)], 1)
    out = oracle.render_pixels(rec, cam, pix)
    gid = rng.choice(np.nonzero(rec.visible)[0], 32, replace=False)
    data = {
        "what": "FP64 oracle on the tiny scene (seed 0, 4096 Gaussians, 256x256): "
                "Eq. 3 at 64 pixels and Eq. 1 records of 32 Gaussians",
        "pixels": pix.tolist(),
        "rgba": out["rgba"].tolist(),
        "T": out["T"].tolist(),
        "n_blend": out["n_blend"].tolist(),
        "gaussians": gid.tolist(),
        "mean2d": rec.d[gid][:, [oracle.D_MX, oracle.D_MY]].tolist(),
        "cov2d": rec.d[gid][:, [oracle.D_SA, oracle.D_SB, oracle.D_SC]].tolist(),
        "rgb": rec.d[gid][:, [oracle.D_R, oracle.D_G, oracle.D_B]].tolist(),
        "depth": rec.d[gid][:, oracle.D_DEPTH].tolist(),
        "instances": int(rec.i[rec.visible, oracle.I_TILES].sum()),
    }
    with open(os.path.join(HERE, "tiny_oracle.json"), "w") as f:
        json.dump(data, f, indent=1)
    print("wrote tiny_oracle.json")


if __name__ == "__main__":
    main()
