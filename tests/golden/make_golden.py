"""Write the oracle regression fixtures in this folder (calls only ``oracle`` and ``sims``).

The paper prints no worked numeric example, so these fixtures are oracle
outputs on a tiny seeded instance; they freeze the oracle so that a later
change to its arithmetic shows up as a failing regression test.

Usage: python tests/golden/make_golden.py
"""

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as ref  # noqa: E402
from sims import configs  # noqa: E402


def tiny_c1():
    """C1 geometry scaled down: 16 antennas in the 2 km disk, 24^2 pixels over 5 deg, 2+1 levels."""
    w = configs.c1(n_ant=16, n_side=24, n_src=3, n_pos_levels=2)
    inst = w.instance(0)
    G = ref.gram(inst.x, inst.wl)
    lam, A = ref.geneig(inst.V, G)
    import sims
    iv = sims.kmeans1d_intervals(lam, 2, negative_level=True)
    img, lam_k, W, member = ref.collect(inst.V, inst.x, inst.wl, w.pix, 16, iv)
    sel = list(range(0, w.n_pix, 37)) + [int(j) for j in w.source_pixels()]
    return {
        "description": "oracle Bluebild LSQ level images, C1 geometry scaled to L=16, 24x24 pixels, "
                       "2 positive k-means levels + 1 negative level (Sections 2.3-2.6, Algorithm 1)",
        "generator": "tests/golden/make_golden.py (oracle.collect on sims.configs.c1(n_ant=16, n_side=24, n_src=3, n_pos_levels=2))",
        "intervals": iv.tolist(),
        "eigenvalues_desc": lam_k.tolist(),
        "pixels": sel,
        "images": img[:, sel].tolist(),
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "tiny_c1_images.json"), "w") as f:
        json.dump(tiny_c1(), f, indent=1)
    print("wrote tiny_c1_images.json")
