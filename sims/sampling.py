"""Pixel samples for checking full-size images on the CPU.

Evaluating the FP64 reference at every pixel of a 1024^2 or 2048^2 image over
all epochs would take hours; the checks use every ``stride``-th row and column
of the grid, the (2 halo + 1)^2 neighbourhood of every point source (where the
images have their largest values and steepest gradients), and the grid's last
pixel (the ragged end of the last pixel tile).  No imaging arithmetic here.
"""

import numpy as np


def sample_pixels(n_side, src_pixels, stride=8, halo=4):
    """Sorted flat indices (row-major, n_side x n_side grid) of the sample."""
    iy, ix = np.meshgrid(np.arange(0, n_side, stride), np.arange(0, n_side, stride), indexing="ij")
    sel = [(iy * n_side + ix).ravel()]
    for p in np.asarray(src_pixels, np.int64).ravel():
        cy, cx = divmod(int(p), n_side)
        ys = np.arange(max(cy - halo, 0), min(cy + halo, n_side - 1) + 1)
        xs = np.arange(max(cx - halo, 0), min(cx + halo, n_side - 1) + 1)
        sel.append((ys[:, None] * n_side + xs[None, :]).ravel())
    sel.append(np.array([n_side * n_side - 1]))
    return np.unique(np.concatenate(sel)).astype(np.int64)
