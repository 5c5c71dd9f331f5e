"""GPU parity of the k-means levels and of uniform weighting against the oracle.

Integer results (level ids) and the weighted visibilities are compared
exactly: the device takes every decision (a k-means cut, a uv cell) from the
same FP64 quantities as the oracle's definition.  Where two k-means
partitions tie to rounding, the device's must be as good as the oracle's
optimum (several results are then correct).
"""

import sys

import numpy as np
import pytest
import torch

import sims
from oracle import bluebild_ref as ref
from oracle import levels_ref as lv
from oracle import weighting_ref as uw
from sims import configs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2310_09200_amd import Context
    c = Context(0)
    yield c
    c.close()


def _synth(ctx, n_levels, n_ant_max=512, k_max=512):
    from paper_2310_09200_amd import StandardSynthesis
    return StandardSynthesis(ctx, sims.pixel_grid(16, 5.0), n_levels, 1, n_ant_max, k_max, "fp32")


def _eigvals_c1():
    inst = configs.c1().instance(0)
    lam, _ = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
    return lam


def _check_kmeans(s, lam, negative_level):
    k = s.n_levels - int(negative_level)
    iv_d, lev_d = s.levels_kmeans(torch.as_tensor(lam), negative_level=negative_level)
    s.sync()
    iv = iv_d.cpu().numpy()
    lev = lev_d.cpu().numpy()
    want_iv = lv.kmeans_intervals(lam, k, negative_level=negative_level)
    want_lev = lv.level_of(lam, want_iv)
    if np.array_equal(lev, want_lev):
        np.testing.assert_array_equal(iv, want_iv)
        return
    # a different partition is only acceptable when it is equally good
    pos = np.sort(lam[lam > 0])
    _, _, best = lv.kmeans1d(pos, k)
    sizes = [int(np.sum((lev == l) & (lam > 0))) for l in range(k)][::-1]   # ascending groups
    starts = np.cumsum([0] + sizes[:-1]).tolist()
    assert sum(sizes) == pos.size
    assert lv.partition_cost(pos, starts) <= best * (1 + 1e-12) + 1e-300
    np.testing.assert_array_equal(lv.level_of(lam, iv), lev)


@pytest.mark.parametrize("n_pos,neg", [(4, True), (8, True), (8, False), (1, True), (15, True)])
def test_kmeans_c1_eigenvalues(ctx, n_pos, neg):
    say(f"case kmeans C1 eigenvalues n_pos={n_pos} negative={neg}")
    lam = _eigvals_c1()
    s = _synth(ctx, n_pos + int(neg))
    _check_kmeans(s, lam, neg)
    s.close()


def test_kmeans_max_size_and_ragged(ctx):
    g = sims.rng(90, 0)
    for n, n_pos in [(1024, 8), (333, 5), (17, 3), (1, 1)]:
        say(f"case kmeans random n={n} n_pos={n_pos}")
        lam = np.exp(g.normal(0.0, 2.0, n)) * np.where(g.random(n) < 0.8, 1.0, -1.0)
        if n == 1:
            lam = np.abs(lam)
        s = _synth(ctx, n_pos + 1, n_ant_max=1024, k_max=1024)
        _check_kmeans(s, lam, True)
        s.close()


def test_kmeans_all_singletons_and_duplicates(ctx):
    say("case kmeans singletons / duplicates")
    s = _synth(ctx, 4)
    _check_kmeans(s, np.array([3.0, 1.0, 2.0, -1.0, 0.0]), True)            # k = number of positives
    s.close()
    s = _synth(ctx, 3)
    lam = np.array([5.0, 1.0, 5.0, 1.0, 5.0, 1.0])
    iv_d, lev_d = s.levels_kmeans(torch.as_tensor(lam), negative_level=False)
    s.sync()
    want_iv = lv.kmeans_intervals(lam, 3, negative_level=False)
    np.testing.assert_array_equal(iv_d.cpu().numpy(), want_iv)
    np.testing.assert_array_equal(lev_d.cpu().numpy(), lv.level_of(lam, want_iv))
    s.close()


def test_kmeans_too_few_positive_reported_at_sync(ctx):
    from paper_2310_09200_amd import BluebildError
    say("case kmeans too few positive eigenvalues")
    s = _synth(ctx, 5)
    iv_d, lev_d = s.levels_kmeans(torch.as_tensor(np.array([2.0, 1.0, -1.0])), negative_level=True)
    with pytest.raises(BluebildError, match="k-means"):
        s.sync()
    assert np.all(lev_d.cpu().numpy() == -1) and np.all(np.isnan(iv_d.cpu().numpy()))
    # the error word was cleared: a valid call goes through
    _check_kmeans(s, np.array([9.0, 8.0, 4.0, 3.0, 1.0, -2.0]), True)
    s.close()


# ------------------------------------------------------- uniform weighting ---

def _weigh(s, x, wl, V, e_u, e_v, fov):
    out = s.uniform_weighting(torch.as_tensor(x), wl, torch.as_tensor(V), e_u, e_v, fov)
    s.sync()
    return out.cpu().numpy()


def _hermitian(L, g):
    A = g.normal(size=(L, L)) + 1j * g.normal(size=(L, L))
    return A + A.conj().T


@pytest.mark.parametrize("L", [1, 9, 37, 64, 512])
def test_uniform_weighting_c2_layout(ctx, L):
    say(f"case uniform weighting C2 layout L={L}")
    w = configs.c2(n_steps=4)
    x = sims.earth_rotate(w.meta["ecef"], w.meta["angles"][1])[:L]
    e_u, e_v, _ = sims.tangent_basis(50.0)
    fov = np.deg2rad(10.0)
    wl = sims.wavelength_m(150e6)
    V = _hermitian(L, sims.rng(91, L))
    s = _synth(ctx, 2)
    got = _weigh(s, x, wl, V, e_u, e_v, fov)
    s.close()
    np.testing.assert_array_equal(got, uw.apply_uniform_weighting(V, x, wl, e_u, e_v, fov))


def test_uniform_weighting_regular_arrays(ctx):
    say("case uniform weighting regular arrays")
    s = _synth(ctx, 2)
    E_U, E_V = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
    L = 9
    x = np.zeros((L, 3))
    x[:, 0] = 4.0 * np.arange(L)
    V = np.ones((L, L), np.complex128) * (1 + 1j)
    got = _weigh(s, x, 2.0, V, E_U, E_V, 0.5)
    p, q = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    np.testing.assert_array_equal(got.real, 1.0 / (L - np.abs(p - q)))
    np.testing.assert_array_equal(got.imag, 1.0 / (L - np.abs(p - q)))
    # cells on half-way points go away from zero
    x2 = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    got2 = _weigh(s, x2, 2.0, np.ones((2, 2), np.complex128), E_U, E_V, 0.5)
    np.testing.assert_array_equal(got2.real, [[0.5, 1.0], [1.0, 0.5]])
    s.close()


def test_uniform_weighting_max_size(ctx):
    say("case uniform weighting L=1024")
    g = sims.rng(92, 0)
    L = 1024
    x = sims.disk_layout(L, 4000.0, g, z_sigma_m=3.0)
    e_u, e_v, _ = sims.tangent_basis(-30.0)
    V = _hermitian(L, g)
    s = _synth(ctx, 2, n_ant_max=L)
    got = _weigh(s, x, 2.0, V, e_u, e_v, np.deg2rad(8.0))
    s.close()
    np.testing.assert_array_equal(got, uw.apply_uniform_weighting(V, x, 2.0, e_u, e_v, np.deg2rad(8.0)))


def test_uniform_weighting_out_of_range_reported(ctx):
    from paper_2310_09200_amd import BluebildError
    say("case uniform weighting cell out of range")
    s = _synth(ctx, 2)
    x = np.array([[0.0, 0.0, 0.0], [1.0e6, 0.0, 0.0]])
    V = np.ones((2, 2), np.complex128)
    out = s.uniform_weighting(torch.as_tensor(x), 1.0e-4, torch.as_tensor(V), [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], 1.0)
    with pytest.raises(BluebildError, match="uv cell"):
        s.sync()
    # the autocorrelations are in range and weighted; the long baseline is left as it was
    got = out.cpu().numpy()
    assert got[0, 0] == 0.5 and got[0, 1] == 1.0
    s.close()


def test_uniform_weighting_then_collect(ctx):
    """Weighted visibilities through the full step, against the oracle's image of the same."""
    from paper_2310_09200_amd import StandardSynthesis
    say("case uniform weighting then full collect, C1")
    w = configs.c1()
    inst = w.instance(0)
    e_u, e_v, _ = sims.tangent_basis(90.0)
    fov = np.deg2rad(5.0)
    Vw = uw.apply_uniform_weighting(inst.V, inst.x, inst.wl, e_u, e_v, fov)
    lam, _ = ref.geneig(Vw, ref.gram(inst.x, inst.wl))
    intervals = lv.kmeans_intervals(lam, 4)
    s = StandardSynthesis(ctx, w.pix, 5, 1, 64, 64, "fp32")
    Vd = s.uniform_weighting(torch.as_tensor(inst.x), inst.wl, torch.as_tensor(inst.V), e_u, e_v, fov)
    s.collect(0, inst.x, inst.wl, Vd, 64, intervals)
    s.sync()
    got = s.images[0].double().cpu().numpy()
    s.close()
    want = ref.collect(Vw, inst.x, inst.wl, w.pix, 64, intervals)[0]
    for lvl in range(5):
        ref_max = np.max(np.abs(want[lvl]))
        if ref_max > 0:
            assert np.max(np.abs(got[lvl] - want[lvl])) / ref_max <= 1e-5
