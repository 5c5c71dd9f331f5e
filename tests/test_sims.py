"""Checks of the seeded workload generators (CPU only)."""

import itertools

import numpy as np

import sims
from sims import configs
from sims.levels import _kmeans1d_sorted


def _sse(v, starts):
    b = list(starts) + [v.size]
    return sum(np.sum((v[b[i]:b[i + 1]] - v[b[i]:b[i + 1]].mean()) ** 2) for i in range(len(starts)))


def test_kmeans1d_is_optimal_by_brute_force():
    g = np.random.default_rng(0)
    for trial in range(20):
        v = np.sort(np.exp(g.normal(0, 2, 9)))
        k = 1 + trial % 4
        best = min(_sse(v, (0,) + c) for c in itertools.combinations(range(1, 9), k - 1))
        assert abs(_sse(v, _kmeans1d_sorted(v, k)) - best) <= 1e-12 * max(best, 1)


def test_intervals_disjoint_and_cover():
    g = np.random.default_rng(1)
    lam = np.concatenate([np.exp(g.normal(0, 2, 40)), -np.abs(g.normal(0, 0.1, 8))])
    iv = sims.kmeans1d_intervals(lam, 4, negative_level=True)
    assert iv.shape == (5, 2)
    lev = sims.levels_from_intervals(lam, iv)
    assert np.all(lev >= 0)
    assert np.all(lev[lam < 0] == 4)
    cnt = ((lam[None, :] >= iv[:, :1]) & (lam[None, :] <= iv[:, 1:])).sum(0)
    assert np.all(cnt == 1)
    # level 0 is the highest-energy cluster
    assert lam[lev == 0].min() > lam[lev == 1].max()


def test_pixel_grid_unit_vectors_and_centre():
    p = sims.pixel_grid(64, 10.0, 50.0)
    assert p.shape == (4096, 3)
    assert np.allclose(np.linalg.norm(p, axis=1), 1.0)
    d = np.deg2rad(50.0)
    c = p.mean(0)
    assert np.allclose(c / np.linalg.norm(c), [np.cos(d), 0, np.sin(d)], atol=1e-6)
    r = sims.pixel_index_direction(64, 10.0, 50.0, 5, 9)
    assert np.allclose(r, p[9 * 64 + 5])


def test_visibility_hermitian_psd_and_snr():
    g = np.random.default_rng(2)
    x = sims.disk_layout(20, 100.0, g)
    dirs, flux, *_ = sims.point_sources(5, 32, 10.0, 90.0, g)
    V = sims.visibility(x, dirs, flux, 2.0)
    assert np.allclose(V, V.conj().T)
    assert np.min(np.linalg.eigvalsh(V)) > -1e-10 * np.abs(V).max()
    assert np.allclose(np.diag(V).real, flux.sum())
    N = sims.hermitian_noise(20, g)
    Vn = sims.add_noise_snr(V, N, 20.0)
    assert abs(np.linalg.norm(V) / np.linalg.norm(Vn - V) - 20.0) < 1e-9


def test_config_shapes_small():
    w = configs.c1()
    inst = w.instance(0)
    assert inst.x.shape == (64, 3) and inst.V.shape == (64, 64)
    assert w.pix.shape == (128 * 128, 3) and w.n_levels == 5
    assert np.max(np.linalg.norm(inst.x[:, :2], axis=1)) <= 1000.0
    w2 = configs.c2(n_steps=3, n_side=64)
    i2 = w2.instance(2)
    assert i2.x.shape == (512, 3)
    span = np.max(np.linalg.norm(i2.x[:, None] - i2.x[None], axis=-1))
    assert 40e3 < span < 60e3
    w3 = configs.c3(n_steps=2, n_side=64)
    i3 = w3.instance(1)
    span3 = np.max(np.linalg.norm(i3.x[:, None] - i3.x[None], axis=-1))
    assert 55e3 < span3 < 70e3
    assert w3.source_pixels().size == 9
    w4 = configs.c4()
    assert w4.n_instances() == 2048
    i4 = w4.instance(77)
    assert 200 <= i4.x.shape[0] <= 512 and 16 <= i4.W.shape[1] <= 128
    w5 = configs.c5()
    assert w5.meta["loss_weights"]().shape == (4, 512 * 512)


def test_seeds_reproducible():
    a = configs.c1().instance(0).V
    b = configs.c1().instance(0).V
    assert np.array_equal(a, b)
