"""Energy-level partitions: exact 1-D k-means on eigenvalues -> [min, max] intervals.

The paper lets levels come from k-means on the eigenvalues or from
user-given intervals (Section 2.6) and, in its validation, clusters the
positive eigenvalues into 1/2/4/8 levels plus one level holding every negative
eigenvalue (Section 4.2).  Here the clustering is the optimal 1-D k-means by
dynamic programming over the sorted values (deterministic; a textbook method),
and interval bounds sit at the midpoints of the gaps between clusters, with
open outer bounds, so that ~1e-13 relative differences between two
eigensolvers cannot move an eigenvalue across a bound.
"""

import numpy as np


def _kmeans1d_sorted(v, k):
    """Optimal partition of sorted ``v`` into ``k`` contiguous clusters; returns cluster starts."""
    n = v.size
    k = min(k, n)
    s1 = np.concatenate([[0.0], np.cumsum(v)])
    s2 = np.concatenate([[0.0], np.cumsum(v * v)])

    def cost(i, j):  # SSE of v[i..j] inclusive; i, j arrays broadcastable
        cnt = j - i + 1
        sm = s1[j + 1] - s1[i]
        return (s2[j + 1] - s2[i]) - sm * sm / cnt

    D = np.full((k, n), np.inf)
    arg = np.zeros((k, n), np.int64)
    D[0] = cost(np.zeros(n, np.int64), np.arange(n))
    for m in range(1, k):
        for j in range(m, n):
            i = np.arange(m, j + 1)
            c = D[m - 1][i - 1] + cost(i, np.full(i.size, j))
            t = int(np.argmin(c))
            D[m, j] = c[t]
            arg[m, j] = i[t]
    starts = [0] * k
    j = n - 1
    for m in range(k - 1, 0, -1):
        starts[m] = int(arg[m, j])
        j = starts[m] - 1
    return starts


def kmeans1d_intervals(lam, n_pos_levels, negative_level=True, min_rel_gap=1e-8):
    """Intervals (N_L, 2) float64 from exact 1-D k-means on the positive eigenvalues.

    Levels are ordered by decreasing energy: level 0 holds the largest
    positive eigenvalues; with ``negative_level`` one more level (last) holds
    every eigenvalue <= the positive/negative bound, whether or not any is
    present.  Raises if a bound lies within ``min_rel_gap * max|lam|`` of an
    eigenvalue.
    """
    lam = np.asarray(lam, np.float64)
    scale = max(np.max(np.abs(lam)), 1e-300)
    pos = np.sort(lam[lam > 0])
    nonpos = lam[lam <= 0]
    bounds_hi_to_lo = []
    if pos.size:
        starts = _kmeans1d_sorted(pos, n_pos_levels)
        # clusters ascending: [starts[i], starts[i+1]) ; boundaries between clusters
        inner = [0.5 * (pos[s - 1] + pos[s]) for s in starts[1:]]
        top_down = inner[::-1]
        zero_bound = 0.5 * (pos[0] + (nonpos.max() if nonpos.size else 0.0))
        n_clusters = len(starts)
    else:
        top_down = []
        zero_bound = 0.0
        n_clusters = 0
    his = [np.inf] + top_down
    los = top_down + [zero_bound]
    iv = [[lo, hi] for lo, hi in zip(los, his)][:n_clusters]
    if negative_level:
        # closed intervals: nudge the shared bound so they do not overlap
        iv.append([-np.inf, np.nextafter(zero_bound, -np.inf)])
    iv = np.array(iv, np.float64).reshape(-1, 2)
    for b in np.unique(iv[np.isfinite(iv)]):
        if np.min(np.abs(lam - b)) < min_rel_gap * scale:
            raise ValueError("level bound too close to an eigenvalue")
    return iv


def levels_from_intervals(lam, intervals):
    """Level id per eigenvalue: first closed interval containing it, else -1 (disjoint intervals)."""
    lam = np.asarray(lam, np.float64)
    out = np.full(lam.size, -1, np.int32)
    for i in range(intervals.shape[0] - 1, -1, -1):
        lo, hi = intervals[i]
        out[(lam >= lo) & (lam <= hi)] = i
    return out
