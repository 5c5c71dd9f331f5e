"""Shared test helpers: oracle-side expected images and error metrics (tests only)."""

import numpy as np

import oracle as ref
import sims


def eig_inputs(V, x, wl, n_eig, n_pos_levels, negative_level=True):
    """Oracle eigenpairs (top n_eig), LSQ weights and level ids from k-means intervals."""
    lam, A = ref.geneig(V, ref.gram(x, wl))
    lam, W = ref.select_top(lam, A, n_eig)
    iv = sims.kmeans1d_intervals(lam, n_pos_levels, negative_level=negative_level)
    lev = sims.levels_from_intervals(lam, iv)
    return lam, W, iv, lev


def oracle_images(W, d, lev, x, wl, pix, n_levels):
    member = ref.membership_from_level_of(lev, n_levels)
    return ref.synthesize_blas(W, d, member, x, pix, wl)


def level_errors(got, want):
    """Per-level (max-normalised max error, rms-normalised rms error), skipping empty levels."""
    out = []
    for a, b in zip(np.asarray(got, np.float64), np.asarray(want, np.float64)):
        if np.max(np.abs(b)) == 0:
            assert np.max(np.abs(a)) == 0
            continue
        out.append((np.max(np.abs(a - b)) / np.max(np.abs(b)), np.sqrt(np.mean((a - b) ** 2) / np.mean(b * b))))
    return np.array(out)
