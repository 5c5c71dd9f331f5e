"""Pins of the k-means level and uniform-weighting oracles (CPU only).

Each test fixes the oracle against something other than itself: brute force
over every partition, closed forms of the sampling density of regular arrays,
exact rounding cases, and invariants that hold for any layout.
"""

import itertools

import numpy as np
import pytest

from oracle import levels_ref as lv
from oracle import weighting_ref as uw


# ---------------------------------------------------------------- k-means ---

def _brute_force(v, k):
    """Least-cost partition of sorted v into k contiguous runs, by enumeration."""
    n = v.size
    best = (np.inf, None)
    for cuts in itertools.combinations(range(1, n), k - 1):
        b = (0,) + cuts + (n,)
        cost = sum(float(np.var(v[b[g]:b[g + 1]]) * (b[g + 1] - b[g])) for g in range(k))
        if best[1] is None or cost < best[0] - 1e-12 * max(best[0], 1.0):
            best = (cost, [0] + list(cuts))
    return best


@pytest.mark.parametrize("seed", range(6))
def test_kmeans_matches_brute_force(seed):
    g = np.random.default_rng(seed)
    n = 9
    vals = np.exp(g.normal(0, 1.5, n))
    for k in range(1, 5):
        v, starts, cost = lv.kmeans1d(vals, k)
        want_cost, want_starts = _brute_force(v, k)
        assert cost == pytest.approx(want_cost, rel=1e-12, abs=1e-14)
        assert starts == want_starts


def test_kmeans_unsorted_input_and_contiguity_claim():
    # exhaustive search over all labelings (not only contiguous ones) on tiny n
    g = np.random.default_rng(11)
    vals = g.normal(0, 1, 7)
    for k in (2, 3):
        _, _, cost = lv.kmeans1d(vals, k)
        best = np.inf
        for lab in itertools.product(range(k), repeat=vals.size):
            lab = np.array(lab)
            if len(set(lab.tolist())) != k:
                continue
            best = min(best, sum(lv.group_cost(vals[lab == c]) for c in range(k)))
        assert cost == pytest.approx(best, rel=1e-12)


def test_group_cost_is_n_times_variance():
    g = np.random.default_rng(3)
    v = g.normal(5, 2, 50)
    assert lv.group_cost(v) == pytest.approx(np.var(v) * v.size, rel=1e-13)
    assert lv.group_cost([4.0]) == 0.0


def test_segment_costs_entries():
    g = np.random.default_rng(4)
    v = np.sort(g.normal(0, 1, 12))
    C = lv.segment_costs(v)
    for i in range(12):
        for j in range(12):
            if j < i:
                assert C[i, j] == np.inf
            else:
                assert C[i, j] == pytest.approx(np.var(v[i:j + 1]) * (j - i + 1), rel=1e-12, abs=1e-15)


def test_kmeans_degenerate_k():
    v = np.array([3.0, 1.0, 2.0, 8.0])
    s, starts, cost = lv.kmeans1d(v, 1)
    assert starts == [0] and cost == pytest.approx(np.var(v) * 4)
    s, starts, cost = lv.kmeans1d(v, 4)
    assert starts == [0, 1, 2, 3] and cost == 0.0
    with pytest.raises(ValueError):
        lv.kmeans1d(v, 5)


def test_kmeans_two_point_masses():
    _, starts, cost = lv.kmeans1d([10.0, 0.0, 10.0, 0.0, 0.0], 2)
    assert starts == [0, 3] and cost == 0.0


def test_kmeans_separated_groups_and_scale_invariance():
    g = np.random.default_rng(5)
    groups = [1 + 0.01 * g.random(5), 10 + 0.1 * g.random(7), 100 + g.random(3)]
    vals = g.permutation(np.concatenate(groups))
    _, starts, _ = lv.kmeans1d(vals, 3)
    assert starts == [0, 5, 12]
    _, starts2, _ = lv.kmeans1d(4.0 * vals, 3)
    assert starts2 == starts


def test_kmeans_intervals_layout():
    lam = np.array([50.0, 49.0, 5.0, 4.5, 4.0, 0.5, 0.4, -0.3, -2.0])
    iv = lv.kmeans_intervals(lam, 3, negative_level=True)
    assert iv.shape == (4, 2)
    # level 0 = largest group, bounds at gap midpoints, top bound +inf
    assert iv[0, 1] == np.inf and iv[0, 0] == 0.5 * (5.0 + 49.0)
    assert iv[1, 1] == iv[0, 0] and iv[1, 0] == 0.5 * (0.5 + 4.0)
    assert iv[2, 1] == iv[1, 0] and iv[2, 0] == 0.5 * (0.4 + (-0.3))
    assert iv[3, 0] == -np.inf and iv[3, 1] == np.nextafter(iv[2, 0], -np.inf)
    lev = lv.level_of(lam, iv)
    assert lev.tolist() == [0, 0, 1, 1, 1, 2, 2, 3, 3]
    # without a negative level the non-positive eigenvalues are in no level
    iv2 = lv.kmeans_intervals(lam, 3, negative_level=False)
    assert iv2.shape == (3, 2)
    assert lv.level_of(lam, iv2).tolist() == [0, 0, 1, 1, 1, 2, 2, -1, -1]
    # all positive: the lowest bound is half the smallest eigenvalue
    iv3 = lv.kmeans_intervals(np.array([8.0, 4.0, 1.0]), 2, negative_level=False)
    assert iv3[1, 0] == 0.5
    with pytest.raises(ValueError):
        lv.kmeans_intervals(np.array([1.0, -1.0]), 2)


def test_level_of_closed_and_first_wins():
    iv = np.array([[2.0, 3.0], [1.0, 2.0]])
    assert lv.level_of(np.array([2.0, 1.0, 3.0, 0.5, 3.5]), iv).tolist() == [0, 1, 0, -1, -1]


def test_kmeans_levels_are_the_groups():
    g = np.random.default_rng(8)
    lam = np.concatenate([np.exp(g.normal(0, 2, 60)), -np.exp(g.normal(-2, 1, 20))])
    iv = lv.kmeans_intervals(lam, 5)
    lev = lv.level_of(lam, iv)
    v, starts, _ = lv.kmeans1d(lam[lam > 0], 5)
    b = starts + [v.size]
    for grp in range(5):
        members = v[b[grp]:b[grp + 1]]
        got = lev[np.isin(lam, members)]
        assert np.all(got == 4 - grp)
    assert np.all(lev[lam <= 0] == 5)


# ------------------------------------------------------- uniform weighting ---

E_U = np.array([1.0, 0.0, 0.0])
E_V = np.array([0.0, 1.0, 0.0])


def test_uniform_linear_array_closed_form():
    # spacing lambda / FoV along e_u: baseline p - q falls in cell p - q,
    # which L - |p - q| ordered pairs share
    L, wl, fov = 9, 2.0, 0.5
    x = np.zeros((L, 3))
    x[:, 0] = 4.0 * np.arange(L)
    w = uw.uniform_weights(x, wl, E_U, E_V, fov)
    p, q = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    np.testing.assert_array_equal(w, 1.0 / (L - np.abs(p - q)))
    # the same array along e_v, with offsets along the third axis (which do not
    # enter the uv cell): same weights
    y = np.zeros((L, 3))
    y[:, 1] = 4.0 * np.arange(L)
    y[:, 2] = np.linspace(-30.0, 70.0, L)
    np.testing.assert_array_equal(uw.uniform_weights(y, wl, E_U, E_V, fov), w)


def test_cells_round_half_away_from_zero():
    wl, fov = 2.0, 0.5                                   # cell coordinate = metres / 4
    x = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [6.0, -10.0, 0.0]])
    iu, iv = uw.uv_cells(x, wl, E_U, E_V, fov)
    assert iu[1, 0] == 1 and iu[0, 1] == -1              # +-0.5
    assert iu[2, 0] == 2 and iu[0, 2] == -2              # +-1.5
    assert iv[0, 2] == 3 and iv[2, 0] == -3              # +-2.5
    w = uw.uniform_weights(x[:2], wl, E_U, E_V, fov)
    np.testing.assert_array_equal(w, [[0.5, 1.0], [1.0, 0.5]])


def test_cell_counts_brute_force():
    g = np.random.default_rng(21)
    x = g.normal(0, 30.0, (12, 3))
    iu, iv = uw.uv_cells(x, 2.0, E_U, E_V, 0.05)
    cnt = uw.cell_counts(iu, iv)
    same = (iu.ravel()[:, None] == iu.ravel()[None, :]) & (iv.ravel()[:, None] == iv.ravel()[None, :])
    np.testing.assert_array_equal(cnt.ravel(), same.sum(axis=1))
    assert cnt.max() > 12                                # the grid is coarse enough to share cells


def test_uniform_weighting_invariants():
    import sims
    g = np.random.default_rng(22)
    enu = sims.spiral_layout(32, "gaussian", 300.0, 96, 3, 300.0, 25_000.0, g)
    x = sims.enu_to_ecef(enu, 52.9)
    e_u, e_v, _ = sims.tangent_basis(50.0)
    fov = np.deg2rad(10.0)
    wl = sims.wavelength_m(150e6)
    iu, iv = uw.uv_cells(x, wl, e_u, e_v, fov)
    np.testing.assert_array_equal(iu, -iu.T)
    np.testing.assert_array_equal(iv, -iv.T)
    w = uw.uniform_weights(x, wl, e_u, e_v, fov)
    np.testing.assert_array_equal(w, w.T)
    assert np.all((w > 0) & (w <= 1))
    n_cells = len(set(zip(iu.ravel().tolist(), iv.ravel().tolist())))
    assert w.sum() == pytest.approx(n_cells, rel=1e-12)     # each cell's weights sum to 1
    assert np.all(np.diag(w) == 1.0 / x.shape[0])            # autocorrelations share cell (0, 0)
    V = g.normal(size=(128, 128)) + 1j * g.normal(size=(128, 128))
    V = V + V.conj().T
    Vw = uw.apply_uniform_weighting(V, x, wl, e_u, e_v, fov)
    np.testing.assert_array_equal(Vw, Vw.conj().T)
    np.testing.assert_allclose(Vw, V * w, rtol=1e-15)
