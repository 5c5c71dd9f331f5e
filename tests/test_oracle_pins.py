"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test pins part of the oracle to something other than the oracle itself:
closed forms, invariants, special cases that reduce to a textbook routine,
and brute force on tiny inputs.  A plausible mistake anywhere in the oracle
(a dropped term, a wrong sign or index, a transposed operand) fails at least
one of them; the comment on each test names what it pins.
"""

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as ref
import sims
from sims import configs

RNG = np.random.default_rng(12345)


def tiny_case(L=12, n_side=12, fov=30.0, diameter=40.0, snr=20.0, psd=False, seed=7, n_src=4):
    """Small, well-conditioned instance: antennas a few wavelengths apart, wide field."""
    g = np.random.default_rng(seed)
    x = sims.disk_layout(L, diameter, g, z_sigma_m=0.5)
    wl = 2.0
    pix = sims.pixel_grid(n_side, fov, 90.0)
    dirs, flux, ix, iy = sims.point_sources(n_src, n_side, fov, 90.0, g)
    V = sims.visibility(x, dirs, flux, wl)
    N = sims.psd_noise(L, g) if psd else sims.hermitian_noise(L, g)
    V = sims.add_noise_snr(V, N, snr)
    return x, wl, pix, V, (dirs, flux, ix, iy)


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# ---------------------------------------------------------------- P14: Gram
def test_gram_matches_sphere_quadrature():
    """P14a: G_pq = (1/4pi) int exp(+j 2pi <b_pq, r>) dOmega (continuous Psi* Psi, g=1).

    Gauss-Legendre in cos(theta) x uniform phi on the unit sphere, independent
    of the closed form; pins the factor 2 and the normalised sinc.
    """
    g = np.random.default_rng(3)
    x = g.normal(0, 3.0, (6, 3))
    wl = 2.0
    G = ref.gram(x, wl)
    u, wu = np.polynomial.legendre.leggauss(160)
    phi = np.linspace(0, 2 * np.pi, 320, endpoint=False)
    uu, pp = np.meshgrid(u, phi, indexing="ij")
    s = np.sqrt(1 - uu ** 2)
    r = np.stack([s * np.cos(pp), s * np.sin(pp), uu], -1).reshape(-1, 3)
    w = (wu[:, None] * np.full(phi.size, 2 * np.pi / phi.size)[None, :]).ravel() / (4 * np.pi)
    for p_ in range(6):
        for q_ in range(6):
            b = (x[p_] - x[q_]) / wl
            val = np.sum(w * np.exp(2j * np.pi * (r @ b)))
            assert abs(val - G[p_, q_]) < 1e-10
            assert abs(val.imag) < 1e-10


def test_gram_positive_definite_and_singular_when_coincident():
    """P14b: G is PD for distinct antennas; coincident antennas make it singular."""
    x, wl, *_ = tiny_case()
    assert np.min(np.linalg.eigvalsh(ref.gram(x, wl))) > 0
    assert np.allclose(np.diag(ref.gram(x, wl)), 1.0)
    x2 = x.copy()
    x2[1] = x2[0]
    with pytest.raises(np.linalg.LinAlgError):
        ref.geneig(np.eye(x.shape[0], dtype=complex), ref.gram(x2, wl))


# ---------------------------------------------------------------- P10: eigen residual
def test_geneig_residual_and_normalisation():
    """P10: ||V A - G A Lam|| <= 1e-12 ||V|| and A^H G A = I; also equals scipy's hegv eigenvalues."""
    x, wl, pix, V, _ = tiny_case()
    G = ref.gram(x, wl)
    lam, A = ref.geneig(V, G)
    assert np.linalg.norm(V @ A - G @ A * lam[None, :]) <= 1e-11 * np.linalg.norm(V)
    assert np.linalg.norm(A.conj().T @ G @ A - np.eye(A.shape[0])) <= 1e-10
    lam_sp = sla.eigh(V, G, eigvals_only=True)
    assert np.allclose(lam, lam_sp, rtol=0, atol=1e-10 * np.max(np.abs(lam)))
    assert np.all(np.diff(lam) >= 0)


def test_geneig_rejects_non_hermitian():
    x, wl, pix, V, _ = tiny_case()
    V2 = V.copy()
    V2[0, 1] += 1.0
    with pytest.raises(ValueError):
        ref.geneig(V2, ref.gram(x, wl))


# ---------------------------------------------------------------- P1: LSQ identity
@pytest.mark.parametrize("L,n_side,psd", [(8, 16, False), (16, 20, True), (24, 16, False)])
def test_lsq_identity(L, n_side, psd):
    """P1: with all eigenpairs in one level, sum_a lam_a |eps_a|^2 = diag(Psi G^-1 V G^-1 Psi*).

    The right side uses two linear solves and no eigensolve; pins the
    eigensolve, the G-normalisation of the eigenvectors, the LSQ weights and
    the synthesis contraction (a transposed or unconjugated W fails it).
    """
    x, wl, pix, V, _ = tiny_case(L=L, n_side=n_side, psd=psd, seed=L)
    G = ref.gram(x, wl)
    img, lam, W, member = ref.collect(V, x, wl, pix, L, np.array([[-np.inf, np.inf]]))
    rhs = ref.lsq_image(V, G, x, pix, wl)
    assert rel(img[0], rhs) < 1e-10


def test_lsq_identity_is_not_trivially_satisfied():
    """Guard: dropping the conjugate on W breaks P1 (the pin has teeth)."""
    x, wl, pix, V, _ = tiny_case(L=10, seed=2)
    G = ref.gram(x, wl)
    lam, A = ref.geneig(V, G)
    B = ref.phases(x, pix, wl)
    bad = (lam[:, None] * np.abs(A.T @ B) ** 2).sum(0)
    assert rel(bad, ref.lsq_image(V, G, x, pix, wl)) > 1e-3


# ---------------------------------------------------------------- P2: partition invariance
def test_partition_invariance():
    """P2: the summed image is the same for 1, 2, 4 or 8 levels (the paper's Table 2 check)."""
    x, wl, pix, V, _ = tiny_case(L=24, seed=11)
    G = ref.gram(x, wl)
    lam, A = ref.geneig(V, G)
    lam, W = ref.select_top(lam, A, 24)
    d = ref.lsq_filter(lam)
    totals = []
    for npos in (1, 2, 4, 8):
        iv = sims.kmeans1d_intervals(lam, npos, negative_level=True)
        member = ref.level_membership(lam, iv)
        assert np.all(member.sum(0) == 1)  # disjoint intervals cover every eigenvalue
        totals.append(ref.synthesize_blas(W, d, member, x, pix, wl).sum(0))
    for t in totals[1:]:
        assert rel(t, totals[0]) < 1e-12


def test_level_membership_closed_intervals():
    """Closed [min, max] intervals tested independently (Algorithm 1 interval loop)."""
    lam = np.array([5.0, 3.0, 2.0, 2.0, -1.0])
    iv = np.array([[3.0, 5.0], [2.0, 3.0], [-np.inf, 0.0], [10.0, 20.0]])
    m = ref.level_membership(lam, iv)
    expect = np.array([[1, 1, 0, 0, 0], [0, 1, 1, 1, 0], [0, 0, 0, 0, 1], [0, 0, 0, 0, 0]], bool)
    assert np.array_equal(m, expect)


def test_membership_from_level_ids():
    """Membership from one level id per eigenpair (the form the GPU tests pass level ids in).

    A hand-written case (ids -1 and out of range add nothing, repeated ids),
    then agreement with the interval test for disjoint k-means intervals,
    with the ids found by a plain search for the interval holding each value,
    and the images it gives: the levels of a partition add up to the
    single-level image of every kept eigenpair (a swapped axis or an
    off-by-one level index fails one of these).
    """
    m = ref.membership_from_level_of(np.array([0, 2, -1, 1, 2, 5, 0]), 3)
    expect = np.array([[1, 0, 0, 0, 0, 0, 1], [0, 0, 0, 1, 0, 0, 0], [0, 1, 0, 0, 1, 0, 0]], bool)
    assert m.shape == (3, 7) and np.array_equal(m, expect)
    assert not ref.membership_from_level_of(np.array([-1, -1]), 2).any()

    x, wl, pix, V, _ = tiny_case(L=16, seed=5)
    lam, A = ref.geneig(V, ref.gram(x, wl))
    lam, W = ref.select_top(lam, A, 12)
    iv = sims.kmeans1d_intervals(lam, 3, negative_level=True)
    ids = np.full(lam.size, -1)
    for k, v in enumerate(lam):
        for lv in range(iv.shape[0]):
            if iv[lv, 0] <= v <= iv[lv, 1]:
                ids[k] = lv
                break
    assert (ids >= 0).all()
    m = ref.membership_from_level_of(ids, iv.shape[0])
    assert np.array_equal(m, ref.level_membership(lam, iv))
    d = ref.lsq_filter(lam)
    levels = ref.synthesize_blas(W, d, m, x, pix, wl)
    whole = ref.synthesize_blas(W, d, np.ones((1, lam.size), bool), x, pix, wl)[0]
    assert rel(levels.sum(0), whole) < 1e-12
    for lv in range(iv.shape[0]):
        only = ref.synthesize_blas(W[:, ids == lv], d[ids == lv], np.ones((1, int((ids == lv).sum())), bool),
                                   x, pix, wl)[0]
        assert rel(levels[lv], only) < 1e-12


# ---------------------------------------------------------------- P3: non-negativity
def test_nonnegative_levels_for_psd_visibilities():
    """P3: V PSD and G PD => all lam >= 0 (Sylvester inertia) and every level image >= 0."""
    x, wl, pix, V, _ = tiny_case(L=16, psd=True, seed=5)
    assert np.min(np.linalg.eigvalsh(V)) >= -1e-12 * np.max(np.abs(V))
    G = ref.gram(x, wl)
    lam, A = ref.geneig(V, G)
    assert np.min(lam) >= -1e-12 * np.max(lam)
    iv = sims.kmeans1d_intervals(lam, 4, negative_level=False)
    img, lam2, W, member = ref.collect(V, x, wl, pix, 16, iv)
    assert np.min(img) >= -1e-12 * np.max(img)
    # per-level Gram-corrected visibilities are Hermitian PSD
    for lv in range(member.shape[0]):
        Wl = W[:, member[lv]]
        Vl = (Wl * lam2[member[lv]]) @ Wl.conj().T
        assert np.allclose(Vl, Vl.conj().T, atol=1e-12 * max(1, np.abs(Vl).max()))
        assert np.min(np.linalg.eigvalsh(Vl)) >= -1e-10 * max(1, np.abs(Vl).max())


# ---------------------------------------------------------------- P4 / P5: point source, G = I
def test_point_source_psf_with_identity_gram():
    """P4: V = I0 a a^H, G = I => I(p) = I0 |sum_l exp(+j2pi<x_l, r0 - p>/lam)|^2, I(r0) = I0 L^2.

    Pins the phase sign convention (a flipped sign peaks at the mirror pixel)
    and the absolute scale of the eigen-sum.
    """
    L, n_side, fov = 16, 33, 20.0
    g = np.random.default_rng(9)
    x = sims.disk_layout(L, 60.0, g, z_sigma_m=1.0)
    wl = 2.0
    pix = sims.pixel_grid(n_side, fov, 90.0)
    ix, iy = 23, 7
    r0 = sims.pixel_index_direction(n_side, fov, 90.0, ix, iy)
    I0 = 2.5
    V = sims.visibility(x, r0[None, :], np.array([I0]), wl)
    img, lam, W, member = ref.collect(V, x, wl, pix, L, np.array([[-np.inf, np.inf]]), gram_identity=True)
    psf = ref.point_source_image(x, r0, pix, wl, I0)
    assert rel(img[0], psf) < 1e-10
    j0 = iy * n_side + ix
    assert np.argmax(img[0]) == j0
    assert abs(img[0, j0] - I0 * L * L) < 1e-9 * I0 * L * L


def test_point_source_peaks_at_true_pixel_with_gram():
    """P4 (with the sinc Gram, C1-like geometry): the LSQ image peaks at the source pixel."""
    w = configs.c1(n_ant=32, n_side=48, n_src=1, snr=0.0)
    inst = w.instance(0)
    img, *_ = ref.collect(inst.V, inst.x, inst.wl, w.pix, 32, np.array([[-np.inf, np.inf]]))
    assert np.argmax(img[0]) == w.source_pixels()[0]


def test_identity_gram_equals_backprojection():
    """P5: with G = I the Bluebild image equals the back-projected dirty image diag(Psi V Psi*)."""
    x, wl, pix, V, _ = tiny_case(L=14, seed=4)
    img, *_ = ref.collect(V, x, wl, pix, 14, np.array([[-np.inf, np.inf]]), gram_identity=True)
    assert rel(img[0], ref.backprojection_image(V, x, pix, wl)) < 1e-10


# ---------------------------------------------------------------- P6..P9, P11: invariants
def _eig_setup(seed=21, L=16):
    x, wl, pix, V, _ = tiny_case(L=L, seed=seed)
    lam, A = ref.geneig(V, ref.gram(x, wl))
    lam, W = ref.select_top(lam, A, L)
    iv = sims.kmeans1d_intervals(lam, 3, negative_level=True)
    member = ref.level_membership(lam, iv)
    return x, wl, pix, V, lam, W, member


def test_gauge_invariance():
    """P6: per-eigenvector phases and permutations within a level leave every level image unchanged."""
    x, wl, pix, V, lam, W, member = _eig_setup()
    d = ref.lsq_filter(lam)
    base = ref.synthesize_blas(W, d, member, x, pix, wl)
    ph = np.exp(2j * np.pi * RNG.random(W.shape[1]))
    assert rel(ref.synthesize_blas(W * ph[None, :], d, member, x, pix, wl), base) < 1e-12
    perm = np.arange(W.shape[1])
    idx = np.where(member[0])[0]
    perm[idx] = idx[::-1]
    assert rel(ref.synthesize_blas(W[:, perm], d[perm], member[:, perm], x, pix, wl), base) < 1e-12


def test_translation_invariance_geocentric_offset():
    """P7: adding a constant (even 6.4e6 m) to every antenna position leaves the images unchanged."""
    x, wl, pix, V, lam, W, member = _eig_setup(seed=22)
    d = ref.lsq_filter(lam)
    base = ref.synthesize_blas(W, d, member, x, pix, wl)
    for off in (np.array([10.0, -3.0, 2.0]), np.array([6.4e6, -1.1e6, 3.3e5])):
        assert rel(ref.synthesize_blas(W, d, member, x + off, pix, wl), base) < 1e-7
    # the Gram matrix depends on differences only
    assert np.allclose(ref.gram(x + 1e5, wl), ref.gram(x, wl), atol=1e-9)


def test_rotation_invariance():
    """P8: rotating antennas and pixels together leaves the images unchanged."""
    x, wl, pix, V, lam, W, member = _eig_setup(seed=23)
    d = ref.lsq_filter(lam)
    Q, _ = np.linalg.qr(RNG.normal(size=(3, 3)))
    base = ref.synthesize_blas(W, d, member, x, pix, wl)
    assert rel(ref.synthesize_blas(W, d, member, x @ Q.T, pix @ Q.T, wl), base) < 1e-11


def test_linearity_in_visibilities():
    """P9: with all eigenpairs in one level, I(V1 + V2) = I(V1) + I(V2)."""
    x, wl, pix, V1, _ = tiny_case(L=12, seed=31)
    _, _, _, V2, _ = tiny_case(L=12, seed=32)
    one = np.array([[-np.inf, np.inf]])
    a, *_ = ref.collect(V1, x, wl, pix, 12, one)
    b, *_ = ref.collect(V2, x, wl, pix, 12, one)
    c, *_ = ref.collect(V1 + V2, x, wl, pix, 12, one)
    assert rel(c, a + b) < 1e-10


def test_mirror_symmetry():
    """P11: I(V^T; p) = I(V; -p) -- pins the sign of the phase relative to V's convention."""
    x, wl, pix, V, _ = tiny_case(L=12, seed=41)
    one = np.array([[-np.inf, np.inf]])
    a, *_ = ref.collect(V.T.copy(), x, wl, pix, 12, one)
    b, *_ = ref.collect(V, x, wl, -pix, 12, one)
    assert rel(a, b) < 1e-10


# ---------------------------------------------------------------- P12: two evaluators
def test_loops_equal_blas():
    """P12: the literal-loop evaluator (Algorithms 1-2) equals the BLAS evaluator to 1e-13."""
    x, wl, pix, V, lam, W, member = _eig_setup(seed=51, L=8)
    pix = pix[::7]
    d = ref.lsq_filter(lam)
    a = ref.synthesize_loops(W, d, member, x, pix, wl)
    b = ref.synthesize_blas(W, d, member, x, pix, wl)
    assert rel(a, b) < 1e-13


def test_select_top_order_and_ties():
    """Selection by signed value, descending, ties stable by index (reading of Section 2.6)."""
    lam = np.array([1.0, 3.0, -5.0, 3.0, 2.0])
    A = np.eye(5)
    l2, A2 = ref.select_top(lam, A, 3)
    assert np.array_equal(l2, [3.0, 3.0, 2.0])
    assert np.array_equal(np.argmax(A2, axis=0), [1, 3, 4])


def test_std_filter_sums_unit_weights():
    """Standardized filter: d = 1 gives sum_k |E_k|^2, which equals ||B_p||^2_{W W^H}."""
    x, wl, pix, V, lam, W, member = _eig_setup(seed=52, L=8)
    one = np.ones((1, W.shape[1]), bool)
    img = ref.synthesize_blas(W, ref.std_filter(lam), one, x, pix, wl)
    B = ref.phases(x, pix, wl)
    direct = np.real(np.einsum("lp,lm,mp->p", B.conj(), W @ W.conj().T, B))
    assert rel(img[0], direct) < 1e-12


# ---------------------------------------------------------------- P13: gradient
def _grad_case(L, K, n_side, seed):
    g = np.random.default_rng(seed)
    x = sims.disk_layout(L, 200.0, g, z_sigma_m=1.0)
    wl = 2.0
    pix = sims.pixel_grid(n_side, 8.0, 90.0)
    W = sims.random_eigvecs(L, K, g)
    lam = sims.random_eigvals(K, g)
    iv = sims.kmeans1d_intervals(lam, 3, negative_level=True)
    member = ref.level_membership(lam, iv)
    wts = g.standard_normal((member.shape[0], pix.shape[0]))
    return W, lam, x, member, wts, pix, wl


def _check_grad(W, lam, x, member, wts, pix, wl, coords, tol=1e-6):
    dW, dd, dx = ref.grad_ref.grad(W, lam, x, member, wts, pix, wl)
    fd = ref.grad_ref.fd_grad(W, lam, x, member, wts, pix, wl, coords)
    an = []
    for name, idx in coords:
        an.append({"Wr": lambda: dW[idx].real, "Wi": lambda: dW[idx].imag,
                   "d": lambda: dd[idx], "x": lambda: dx[idx]}[name]())
    an = np.array(an)
    scale = {"Wr": np.abs(dW).max(), "Wi": np.abs(dW).max(), "d": np.abs(dd).max(), "x": np.abs(dx).max()}
    for (name, idx), a, f in zip(coords, an, fd):
        assert abs(a - f) <= tol * scale[name], (name, idx, a, f)


def test_gradient_all_coordinates_tiny():
    """P13a: analytic gradient vs FP64 central differences on every coordinate (L=8, K=4, 16^2 px)."""
    W, lam, x, member, wts, pix, wl = _grad_case(8, 4, 16, 61)
    coords = [(n, (l, k)) for n in ("Wr", "Wi") for l in range(8) for k in range(4)]
    coords += [("d", (k,)) for k in range(4)] + [("x", (l, c)) for l in range(8) for c in range(3)]
    _check_grad(W, lam, x, member, wts, pix, wl, coords)


def test_gradient_sampled_coordinates_c5_shape():
    """P13b: 16 random coordinates per leaf at the C5 shape (L=256, K=64), on a 48^2 pixel patch."""
    W, lam, x, member, wts, pix, wl = _grad_case(256, 64, 48, 62)
    g = np.random.default_rng(63)
    coords = []
    for n in ("Wr", "Wi"):
        coords += [(n, (int(g.integers(256)), int(g.integers(64)))) for _ in range(16)]
    coords += [("d", (int(g.integers(64)),)) for _ in range(16)]
    coords += [("x", (int(g.integers(256)), int(g.integers(3)))) for _ in range(16)]
    _check_grad(W, lam, x, member, wts, pix, wl, coords)


def test_energy_truncation_definition():
    """N_eig by energy: brute force over every K on random spectra (with negatives)."""
    g = np.random.default_rng(8)
    for _ in range(50):
        lam = np.concatenate([np.exp(g.normal(0, 2, 30)), -np.abs(g.normal(0, 0.3, 6))])
        frac = g.uniform(0.05, 1.0)
        k = ref.n_eig_for_energy(lam, frac)
        srt = np.sort(lam)[::-1]
        tot = srt[srt > 0].sum()
        ok = [kk for kk in range(1, lam.size + 1) if srt[:kk].sum() >= frac * tot]
        assert k == min(ok)
    assert ref.n_eig_for_energy(np.array([-1.0, -2.0]), 0.5) == 1


def test_beamforming_identity_and_invertible_invariance():
    """Beamforming (Section 2.7): Wbf = I reproduces the plain step; for an invertible square Wbf
    the summed LSQ image is unchanged (G^W and V^W transform congruently), closed form by solves."""
    x, wl, pix, V, _ = tiny_case(L=14, seed=71)
    one = np.array([[-np.inf, np.inf]])
    a, *_ = ref.collect(V, x, wl, pix, 14, one)
    b, *_ = ref.collect_beamformed(V, np.eye(14), x, wl, pix, 14, one)
    assert rel(b, a) < 1e-10
    g = np.random.default_rng(72)
    Wbf = g.standard_normal((14, 14)) + 1j * g.standard_normal((14, 14))
    Vw = Wbf.conj().T @ V @ Wbf
    c, *_ = ref.collect_beamformed(Vw, Wbf, x, wl, pix, 14, one)
    assert rel(c[0], ref.lsq_image(V, ref.gram(x, wl), x, pix, wl)) < 1e-8


def test_beamforming_fewer_beams_is_lsq_of_beamformed_operator():
    """With Kb < L beams the image is diag(Phi (G^W)^-1 V^W (G^W)^-1 Phi*), Phi* = Wbf^H Psi* (no eigensolve)."""
    x, wl, pix, V, _ = tiny_case(L=16, seed=73)
    g = np.random.default_rng(74)
    Wbf = (g.standard_normal((16, 6)) + 1j * g.standard_normal((16, 6))) / 4
    Vw = Wbf.conj().T @ V @ Wbf
    img, *_ = ref.collect_beamformed(Vw, Wbf, x, wl, pix, 6, np.array([[-np.inf, np.inf]]))
    Gw = Wbf.conj().T @ ref.gram(x, wl) @ Wbf
    Vp = np.linalg.solve(Gw, np.linalg.solve(Gw, Vw).conj().T).conj().T
    Phi_star = Wbf.conj().T @ ref.phases(x, pix, wl)          # (Kb, N_pix)
    want = np.real(np.einsum("kp,kq,qp->p", Phi_star.conj(), Vp, Phi_star))
    assert rel(img[0], want) < 1e-9
