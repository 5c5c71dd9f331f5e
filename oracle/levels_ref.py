"""Energy levels by k-means on the eigenvalues (test infrastructure only).

The paper lets the energy levels be given as intervals or be found by k-means
clustering of the eigenvalues (Section 2.6); its validation clusters the
positive eigenvalues into 1, 2, 4 or 8 levels and gives every negative
eigenvalue one further level of its own (Section 4.2).

Readings (the paper names neither an initialisation nor a stopping rule):
  * the clustering is exact one-dimensional k-means: the partition of the
    positive eigenvalues into k groups with the least total within-group sum of
    squared deviations from the group means.  On a line an optimal partition
    is made of contiguous runs of the sorted values, so the minimum is taken
    over the ways of cutting the sorted list into k runs;
  * ties between equally good partitions go to the one whose highest cut
    comes first, then the next highest, and so on (each group's start is the
    smallest index that attains the minimum);
  * levels are numbered by decreasing energy (level 0 holds the largest
    eigenvalues); the bound between two neighbouring groups is the midpoint of
    the gap between them, the top bound is +inf, and the lowest positive group
    ends at the midpoint between the smallest positive eigenvalue and the
    largest non-positive one (or 0 when there is none);
  * the negative level, when asked for, is [-inf, b) written as the closed
    interval [-inf, nextafter(b, -inf)] with b that lowest positive bound.
"""

import numpy as np

__all__ = ["group_cost", "segment_costs", "kmeans1d", "kmeans_intervals", "level_of", "partition_cost"]


def group_cost(v):
    """Sum of squared deviations of v from its mean (two passes: mean, then deviations)."""
    v = np.asarray(v, np.float64)
    if v.size == 0:
        return 0.0
    m = np.sum(v) / v.size
    return float(np.sum((v - m) ** 2))


def segment_costs(v):
    """C[i, j] = group_cost(v[i..j]) for i <= j (inf below the diagonal); v sorted."""
    v = np.asarray(v, np.float64)
    n = v.size
    C = np.full((n, n), np.inf)
    for i in range(n):
        seg = v[i:]
        cnt = np.arange(1, seg.size + 1, dtype=np.float64)
        mean = np.cumsum(seg) / cnt                     # mean of v[i..j] for every j
        dev = seg[None, :] - mean[:, None]              # row j: deviations of v[i..] from that mean
        inside = np.tri(seg.size, dtype=bool)           # keep v[i..j] only
        C[i, i:] = np.sum(np.where(inside, dev * dev, 0.0), axis=1)
    return C


def kmeans1d(values, k):
    """Exact 1-D k-means of ``values`` into k groups.

    Returns (sorted values, starts, cost): groups are sorted[starts[g]:starts[g+1]]
    in ascending order of value, and cost is the total within-group sum of
    squared deviations.  Dynamic programme over the last cut: best[m][j] is the
    least cost of splitting sorted[0..j] into m + 1 runs.
    """
    v = np.sort(np.asarray(values, np.float64))
    n = v.size
    if k < 1 or k > n:
        raise ValueError("need 1 <= k <= number of values")
    C = segment_costs(v)
    best = np.full((k, n), np.inf)
    cut = np.zeros((k, n), np.int64)
    best[0] = C[0]
    for m in range(1, k):
        for j in range(m, n):
            cand = [best[m - 1][i - 1] + C[i, j] for i in range(m, j + 1)]
            t = int(np.argmin(cand))                    # first minimum: smallest start
            best[m, j] = cand[t]
            cut[m, j] = m + t
    starts = [0] * k
    j = n - 1
    for m in range(k - 1, 0, -1):
        starts[m] = int(cut[m, j])
        j = starts[m] - 1
    return v, starts, float(best[k - 1, n - 1])


def partition_cost(sorted_values, starts):
    """Total within-group cost of the partition given by ascending ``starts``."""
    b = list(starts) + [len(sorted_values)]
    return sum(group_cost(sorted_values[b[g]:b[g + 1]]) for g in range(len(starts)))


def kmeans_intervals(lam, n_pos_levels, negative_level=True):
    """Level intervals (n_levels, 2) [min, max] from exact k-means of the positive eigenvalues.

    n_levels = n_pos_levels + (1 if negative_level else 0).  Raises ValueError
    when there are fewer positive eigenvalues than positive levels.
    """
    lam = np.asarray(lam, np.float64)
    pos = lam[lam > 0]
    nonpos = lam[lam <= 0]
    if pos.size < n_pos_levels:
        raise ValueError("fewer positive eigenvalues than positive levels")
    v, starts, _ = kmeans1d(pos, n_pos_levels)
    low = 0.5 * (v[0] + (np.max(nonpos) if nonpos.size else 0.0))
    # group g (ascending) spans [lower_g, upper_g]; the level id of group g is k - 1 - g
    lowers = [low] + [0.5 * (v[s - 1] + v[s]) for s in starts[1:]]
    uppers = lowers[1:] + [np.inf]
    iv = [[lowers[g], uppers[g]] for g in range(n_pos_levels)][::-1]
    if negative_level:
        iv.append([-np.inf, np.nextafter(low, -np.inf)])
    return np.array(iv, np.float64).reshape(-1, 2)


def level_of(lam, intervals):
    """Level id of each eigenvalue: the first closed interval holding it, else -1."""
    lam = np.asarray(lam, np.float64)
    out = np.full(lam.size, -1, np.int32)
    for k, x in enumerate(lam):
        for lev in range(intervals.shape[0]):
            if intervals[lev, 0] <= x <= intervals[lev, 1]:
                out[k] = lev
                break
    return out
