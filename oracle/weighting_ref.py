"""Uniform image weighting of the visibilities (test infrastructure only).

Natural weighting leaves the visibilities alone; uniform weighting divides
each visibility by the sampling density of its baseline, counted on a uv grid
with cells 1/FoV wide, before the eigendecomposition (Section 3.5).

Readings (the paper gives only the cell size):
  * the uv coordinates of baseline (p, q) are the projections of
    (x_p - x_q) / lambda_w on the two image-plane axes e_u, e_v at the phase
    centre (the first two axes of the pixel grid's basis);
  * the cell of a coordinate a = u * FoV is round(a) with halves rounded away
    from zero, so that (p, q) and (q, p) fall in mirrored cells and the
    weighted matrix stays Hermitian;
  * the density is the number of the instance's own L^2 ordered antenna pairs,
    autocorrelations included, that fall in the cell;
  * the weight of a visibility is 1 / density, applied to its real and
    imaginary parts separately.

The arithmetic order below (differences, the two products summed before the
third, then one product with fov / lambda_w) is the definition: where a
coordinate lands exactly on a cell edge, that order decides the cell.
"""

import numpy as np

__all__ = ["uv_cells", "cell_counts", "uniform_weights", "apply_uniform_weighting"]


def _round_half_away(a):
    t = np.trunc(a)
    frac = a - t                                        # exact
    return (t + np.where(np.abs(frac) >= 0.5, np.sign(a), 0.0)).astype(np.int64)


def uv_cells(x, wl, e_u, e_v, fov_rad):
    """(iu, iv): int64 (L, L) uv cell of every ordered antenna pair (p, q)."""
    x = np.asarray(x, np.float64)
    d = x[:, None, :] - x[None, :, :]                   # x_p - x_q
    s = float(fov_rad) / float(wl)
    out = []
    for e in (np.asarray(e_u, np.float64), np.asarray(e_v, np.float64)):
        raw = (d[..., 0] * e[0] + d[..., 1] * e[1]) + d[..., 2] * e[2]
        out.append(_round_half_away(raw * s))
    return out[0], out[1]


def cell_counts(iu, iv):
    """Number of ordered pairs sharing each pair's cell, as an (L, L) int64 array."""
    keys = list(zip(iu.ravel().tolist(), iv.ravel().tolist()))
    tally = {}
    for key in keys:
        tally[key] = tally.get(key, 0) + 1
    return np.array([tally[key] for key in keys], np.int64).reshape(iu.shape)


def uniform_weights(x, wl, e_u, e_v, fov_rad):
    """w_pq = 1 / (number of pairs in the uv cell of (p, q)), float64 (L, L)."""
    iu, iv = uv_cells(x, wl, e_u, e_v, fov_rad)
    return 1.0 / cell_counts(iu, iv)


def apply_uniform_weighting(V, x, wl, e_u, e_v, fov_rad):
    """V_pq / density_pq, real and imaginary parts divided separately."""
    V = np.asarray(V, np.complex128)
    iu, iv = uv_cells(x, wl, e_u, e_v, fov_rad)
    cnt = cell_counts(iu, iv).astype(np.float64)
    out = np.empty_like(V)
    out.real = V.real / cnt
    out.imag = V.imag / cnt
    return out
