"""Pins of the NUFFT-synthesis oracle (CPU only).

The NUFFT is an approximation: it is pinned to the exact type-3 sum within its
tolerance, to closed forms for single sources, to an independent quadrature of
the kernel transform, and, for images, to standard synthesis (Section 2.4),
which computes the same image exactly.
"""

import numpy as np
import pytest
from scipy import integrate

import oracle as ref
from oracle import levels_ref as lv
from oracle import nufft_ref as nf
from sims import configs


def _problem(seed, n_src=400, n_tgt=200):
    g = np.random.default_rng(seed)
    x = g.uniform(-25.0, 25.0, (n_src, 3)) * np.array([1.0, 1.0, 0.2])
    s = g.normal(0, 1, (n_tgt, 3)) * np.array([0.05, 0.05, 0.003]) + np.array([0.1, -0.2, 0.97])
    c = g.normal(size=n_src) + 1j * g.normal(size=n_src)
    return c, x, s


@pytest.mark.parametrize("eps", [1e-3, 1e-5, 1e-7])
def test_nufft3_within_tolerance_of_exact_sum(eps):
    c, x, s = _problem(1)
    got = nf.nufft3(c, x, s, eps)[:, 0]
    want = nf.nudft3(c, x, s)
    assert np.max(np.abs(got - want)) <= eps * np.sum(np.abs(c))


@pytest.mark.parametrize("eps", [1e-3, 1e-5])
def test_window_end_on_exact_ties_is_immaterial(eps):
    """Targets at the field's edges land exactly half a support from a type-2
    grid point (eta = +-M/4 with an even w): either end of the kernel window
    may be kept there; the two choices differ, and both stay within the
    tolerance of the exact sum (the bound the method states, Section 3.4)."""
    c, x, _ = _problem(8, n_src=300)
    g = np.random.default_rng(9)
    D, S = np.array([0.25, -0.125, 0.875]), np.array([0.125, 0.0625, 0.0078125])
    s = D + S * g.uniform(-1, 1, (60, 3))
    corners = np.array([[a, b, e] for a in (-1, 1) for b in (-1, 1) for e in (-1, 1)], float)
    s = np.concatenate([s, D + S * corners])
    P = nf.plan_params(eps, np.max(np.abs(x), axis=0), s)
    assert P["w"] % 2 == 0
    eta = (s - P["D"]) * (P["h"] * P["M"])
    assert np.any(eta - 0.5 * P["w"] == np.round(eta - 0.5 * P["w"]))   # exact ties are present
    lo = nf.nufft3(c, x, s, eps, tie="low")[:, 0]
    hi = nf.nufft3(c, x, s, eps, tie="high")[:, 0]
    want = nf.nudft3(c, x, s)
    bound = eps * np.sum(np.abs(c))
    assert np.max(np.abs(lo - hi)) > 0.0
    assert np.max(np.abs(lo - want)) <= bound
    assert np.max(np.abs(hi - want)) <= bound


@pytest.mark.parametrize("q", [2, 3, 5])
def test_uvw_cells_within_tolerance_of_exact_sum(q):
    """Splitting the sources into q x q uvw cells (shift by the cell centre,
    transform, multiply by exp(2 pi i <s, C>)) still meets the tolerance
    against the exact sum, with every cell's grid smaller than the whole's."""
    c, x, s = _problem(10)
    X = np.max(np.abs(x), axis=0) * 1.001
    eps = 1e-5
    got = nf.nufft3_uvw_cells(c, x, s, eps, X, q)[:, 0]
    want = nf.nudft3(c, x, s)
    assert np.max(np.abs(got - want)) <= eps * np.sum(np.abs(c))
    whole = nf.plan_params(eps, X, s)["N"]
    Xc = X.copy()
    Xc[:2] = X[:2] / q * (1 + 1e-9)
    part = nf.plan_params(eps, Xc, s)["N"]
    assert part[0] < whole[0] and part[1] < whole[1] and part[2] == whole[2]


def test_uvw_cell_rule():
    X, q = 10.0, 4
    b = np.array([-10.0, -5.0 - 1e-9, -5.0, -0.0, 0.0, 4.999999, 5.0, 9.9, 10.0])
    assert list(nf.uvw_cell(b, X, q)) == [0, 0, 1, 2, 2, 2, 3, 3, 3]
    assert [nf.uvw_cell_centre(i, X, q) for i in range(q)] == [-7.5, -2.5, 2.5, 7.5]


def test_nudft3_is_the_sum():
    c, x, s = _problem(2, 7, 5)
    brute = np.array([sum(c[j] * np.exp(2j * np.pi * np.dot(s[k], x[j])) for j in range(7)) for k in range(5)])
    np.testing.assert_allclose(nf.nudft3(c, x, s), brute, rtol=1e-12)


def test_single_sources():
    g = np.random.default_rng(3)
    s = g.normal(0, 0.02, (50, 3)) + np.array([0.0, 0.3, 0.95])
    # a unit source at the origin: f = 1 everywhere (pins every normalisation)
    f = nf.nufft3(np.array([1.0 + 0j]), np.zeros((1, 3)), s, 1e-8, X=np.array([10.0, 10.0, 2.0]))[:, 0]
    np.testing.assert_allclose(f, 1.0, atol=1e-7)
    # a source at x0: a plane wave exp(+2 pi i <s, x0>) (pins signs and the centring)
    x0 = np.array([[7.3, -4.1, 1.7]])
    f = nf.nufft3(np.array([2.0 - 1.0j]), x0, s, 1e-8, X=np.array([10.0, 10.0, 2.0]))[:, 0]
    np.testing.assert_allclose(f, (2.0 - 1.0j) * np.exp(2j * np.pi * s @ x0[0]), atol=1e-7)


def test_channels_are_independent_and_linear():
    c, x, s = _problem(4)
    c2 = np.stack([c, 3.0 * c, np.conj(c)], axis=1)
    f = nf.nufft3(c2, x, s, 1e-6)
    np.testing.assert_allclose(f[:, 1], 3.0 * f[:, 0], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(f[:, 2], nf.nufft3(np.conj(c), x, s, 1e-6)[:, 0], rtol=1e-12)


def test_kernel_ft_against_adaptive_quadrature():
    # 100 Gauss-Legendre nodes: relative error near 1e-9 at w = 4 (the kernel's end
    # values carry a square-root cusp), far below the tolerances the NUFFT is run at
    for w in (4, 6, 9):
        beta = 2.30 * w
        for a, k in [(1.0, 0.0), (0.5 * w, 1.3), (0.003, 700.0)]:
            want = integrate.quad(lambda z: nf.es_kernel(np.array([z / a]), beta)[0] * np.cos(k * z), -a, a,
                                  epsabs=1e-14, epsrel=1e-12, limit=200)[0]
            assert nf.kernel_ft(np.array([k]), a, beta)[0] == pytest.approx(want, rel=1e-8, abs=1e-14)


def test_es_kernel_values():
    np.testing.assert_allclose(nf.es_kernel(np.array([0.0, 1.0, -1.0, 1.5, 0.6]), 13.8),
                               [1.0, np.exp(-13.8), np.exp(-13.8), 0.0, np.exp(13.8 * (0.8 - 1.0))], rtol=1e-15)


def test_grid_rules():
    assert [nf.smooth_size(n) for n in (1, 7, 11, 13, 17, 31, 49, 121)] == [2, 8, 12, 16, 18, 32, 50, 128]
    assert [nf.kernel_width(e) for e in (1e-2, 1e-3, 1e-5, 1e-6, 3e-6)] == [3, 4, 6, 7, 7]
    P = nf.plan_params(1e-5, np.array([100.0, 50.0, 1.0]), np.array([[0.0, 0.0, 1.0], [0.1, 0.2, 0.99]]))
    np.testing.assert_allclose(P["S"], [0.05, 0.1, 0.005])
    np.testing.assert_allclose(P["h"], 1.0 / (4.0 * P["S"]))
    assert list(P["N"]) == [nf.smooth_size(40 + 6), nf.smooth_size(40 + 6), 12]
    assert list(P["M"]) == [2 * n for n in P["N"]]


def test_rotation_preserves_phases():
    g = np.random.default_rng(5)
    Q, _ = np.linalg.qr(g.normal(size=(3, 3)))
    a, b = g.normal(size=(20, 3)), g.normal(size=(20, 3))
    np.testing.assert_allclose(np.sum(nf.rotate(a, Q) * nf.rotate(b, Q), axis=1), np.sum(a * b, axis=1), rtol=1e-12)


@pytest.mark.parametrize("eps", [1e-4, 1e-6])
def test_nufft_image_equals_standard_synthesis(eps):
    """Section 2.5: NUFFT synthesis computes the same level images as standard synthesis."""
    w = configs.c1(n_ant=48, n_side=40)
    inst = w.instance(0)
    lam, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
    lam, W = ref.select_top(lam, A, 48)
    iv = lv.kmeans_intervals(lam, 3)
    member = ref.level_membership(lam, iv)
    d = ref.lsq_filter(lam)
    want = ref.synthesize_blas(W, d, member, inst.x, w.pix, inst.wl)
    import sims
    frame = np.array(sims.tangent_basis(90.0))
    got = nf.nufft_image(inst.x, inst.wl, W, d, member, w.pix, eps, frame=frame)
    for a, b in zip(got, want):
        assert np.max(np.abs(a - b)) <= 3 * eps * np.max(np.abs(b))


def test_level_visibilities_sum_to_filtered_matrix():
    g = np.random.default_rng(6)
    W = g.normal(size=(6, 4)) + 1j * g.normal(size=(6, 4))
    d = np.array([3.0, 2.0, 1.0, -1.0])
    member = np.array([[1, 1, 0, 0], [0, 0, 1, 0], [0, 0, 0, 1]], bool)
    Vp = nf.level_visibilities(W, d, member)
    np.testing.assert_allclose(Vp.sum(axis=0), W @ np.diag(d) @ W.conj().T, rtol=1e-12, atol=1e-12)
    for V in Vp:
        np.testing.assert_allclose(V, V.conj().T, atol=1e-14)
