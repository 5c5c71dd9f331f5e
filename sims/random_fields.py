"""Random stand-ins for eigenpairs, for workloads where an eigensolve per instance is not needed.

The synthesis step accepts any (W, lambda); these draws have the magnitudes of
G-normalised eigenvectors of the synthetic visibility matrices (entries of
order 1/sqrt(L)) and a spread of positive and a few negative eigenvalues.
"""

import numpy as np


def random_eigvecs(L, K, g, dtype=np.complex128):
    """(L, K) complex matrix with i.i.d. CN(0, 1/L) entries."""
    W = (g.standard_normal((L, K)) + 1j * g.standard_normal((L, K))) / np.sqrt(2.0 * L)
    return W.astype(dtype)


def random_eigvals(K, g, frac_neg=0.1):
    """K eigenvalues sorted descending: log-normal positives and a few small negatives."""
    n_neg = int(round(frac_neg * K))
    pos = np.exp(g.normal(0.0, 1.5, K - n_neg))
    neg = -np.abs(g.normal(0.0, 0.05, n_neg)) * np.median(pos)
    return np.sort(np.concatenate([pos, neg]))[::-1].copy()
