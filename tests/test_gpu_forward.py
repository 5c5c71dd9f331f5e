"""GPU parity of the HIP synthesis path against the FP64 oracle (through the C ABI).

Tolerances (per level, error normalised by the level's peak, BASELINE target):
FP32 contraction <= 1e-5, BF16 x3 compensated contraction <= 1e-4.
"""

import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle as ref
import sims
from sims import configs
from tests._helpers import eig_inputs, level_errors, oracle_images

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-4, "bf16x3_3m": 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2310_09200_amd import Context
    c = Context(0)
    yield c


def run_eig(ctx, pix, n_levels, x, wl, W, d, lev, precision="fp32", n_ant_max=None, k_max=None):
    from paper_2310_09200_amd import StandardSynthesis
    L, K = W.shape
    s = StandardSynthesis(ctx, pix, n_levels, 1, n_ant_max or L, k_max or K, precision)
    s.collect_eig(0, x, wl, W, d, lev)
    s.sync()
    out = s.images[0].double().cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("precision", ["fp32", "fp32_3m", "bf16x3", "bf16x3_3m"])
def test_c1_against_oracle(ctx, precision):
    """C1 (L=64, K=64, 128^2 px, 4+1 k-means levels): full image, every level."""
    say(f"case C1 precision={precision}")
    w = configs.c1()
    inst = w.instance(0)
    lam, W, iv, lev = eig_inputs(inst.V, inst.x, inst.wl, 64, 4)
    want = oracle_images(W, lam, lev, inst.x, inst.wl, w.pix, 5)
    got = run_eig(ctx, w.pix, 5, inst.x, inst.wl, W, lam, lev, precision)
    err = level_errors(got, want)
    say("C1", precision, "max err per level", err[:, 0])
    assert np.all(err[:, 0] <= TOL[precision]), err


CASES = [  # (L, K, n_side): ragged antenna / eigenpair / pixel counts covering every tile shape,
    # and the K class edges (16 and 17 rows: one and two 16-row blocks; 64 / 65: classes 1 / 2)
    (7, 5, 23), (40, 16, 19), (33, 17, 21), (50, 37, 37), (64, 64, 40), (100, 65, 27), (129, 100, 41),
    (300, 200, 29), (333, 300, 19), (512, 512, 17),
]


@pytest.mark.parametrize("precision", ["fp32", "fp32_3m", "bf16x3", "bf16x3_3m"])
@pytest.mark.parametrize("L,K,n_side", CASES)
def test_ragged_random_eigpairs(ctx, L, K, n_side, precision):
    """Random W/lambda with unsorted level ids incl. -1; pixel tail not a multiple of the tile."""
    say(f"case ragged L={L} K={K} n_side={n_side} precision={precision}")
    g = np.random.default_rng(1000 + L + K)
    x = sims.disk_layout(L, 3000.0, g, z_sigma_m=2.0)
    wl = sims.wavelength_m(150e6)
    pix = sims.pixel_grid(n_side, 6.0, 60.0)
    W = sims.random_eigvecs(L, K, g)
    d = g.normal(0, 1, K)
    n_levels = 3
    lev = g.integers(-1, n_levels, K).astype(np.int32)
    d32 = d.astype(np.float32).astype(np.float64)
    want = oracle_images(W.astype(np.complex64).astype(np.complex128), d32, lev, x, wl, pix, n_levels)
    got = run_eig(ctx, pix, n_levels, x, wl, W, d, lev, precision)
    err = level_errors(got, want)
    say("max err per level", err[:, 0] if err.size else err)
    assert np.all(err[:, 0] <= TOL[precision]), err


@pytest.mark.parametrize("K,precision", [(20, "fp32"), (50, "fp32_3m"), (100, "fp32_3m"), (100, "bf16x3_3m")])
def test_all_levels_dropped_leaves_images_zero(ctx, K, precision):
    """Every level id -1: no kept eigenpair, so no pass runs and the images stay zero
    (32-row and 16-row tiles)."""
    say(f"case all level ids -1, K={K} precision={precision}")
    g = np.random.default_rng(5)
    x = sims.disk_layout(40, 1000.0, g)
    pix = sims.pixel_grid(16, 5.0, 90.0)
    W = sims.random_eigvecs(40, K, g)
    got = run_eig(ctx, pix, 2, x, 2.0, W, np.ones(K), -np.ones(K, np.int32), precision)
    assert np.all(got == 0)


@pytest.mark.parametrize("precision", ["fp32_3m", "bf16x3_3m"])
def test_sixteen_levels(ctx, precision):
    """The largest level count (16) with K in the K <= 128 class: level ranges of
    16-row and 32-row blocks that span many levels, against the oracle."""
    say(f"case 16 levels precision={precision}")
    g = np.random.default_rng(16)
    L, K = 90, 100
    x = sims.disk_layout(L, 3000.0, g, z_sigma_m=2.0)
    wl = sims.wavelength_m(150e6)
    pix = sims.pixel_grid(30, 6.0, 60.0)
    W = sims.random_eigvecs(L, K, g)
    d = g.normal(0, 1, K)
    lev = g.integers(-1, 16, K).astype(np.int32)
    d32 = d.astype(np.float32).astype(np.float64)
    want = oracle_images(W.astype(np.complex64).astype(np.complex128), d32, lev, x, wl, pix, 16)
    got = run_eig(ctx, pix, 16, x, wl, W, d, lev, precision)
    err = level_errors(got, want)
    say("16 levels", precision, "max err", err[:, 0].max())
    assert np.all(err[:, 0] <= TOL[precision]), err


def test_accumulation_and_determinism(ctx):
    """Two collects accumulate (sum over time steps); identical runs are bitwise equal."""
    from paper_2310_09200_amd import StandardSynthesis
    say("case accumulation/determinism")
    w = configs.c1(n_ant=48, n_side=64)
    inst = w.instance(0)
    lam, W, iv, lev = eig_inputs(inst.V, inst.x, inst.wl, 48, 2)
    outs = []
    for rep in range(2):
        s = StandardSynthesis(ctx, w.pix, 3, 2, 48, 48)
        s.collect_eig(1, inst.x, inst.wl, W, lam, lev)
        s.collect_eig(1, inst.x, inst.wl, W, lam, lev)
        s.sync()
        assert s.count == 2
        outs.append(s.images.cpu().numpy())
        s.close()
    assert np.array_equal(outs[0], outs[1])
    assert np.all(outs[0][0] == 0)
    want = 2 * oracle_images(W, lam, lev, inst.x, inst.wl, w.pix, 3)
    assert np.all(level_errors(outs[0][1], want)[:, 0] <= 1e-5)


@pytest.mark.parametrize("precision", ["fp32", "fp32_3m", "bf16x3", "bf16x3_3m"])
def test_full_collect_prestep_on_gpu(ctx, precision):
    """bb_synth_collect: FP64 Gram + rocSOLVER eigensolve + selection + levels + synthesis on the GPU."""
    from paper_2310_09200_amd import StandardSynthesis
    say(f"case full collect C1 precision={precision}")
    w = configs.c1()
    inst = w.instance(0)
    img_ref, lam, W, member = ref.collect(inst.V, inst.x, inst.wl, w.pix, 64,
                                          sims.kmeans1d_intervals(ref.geneig(inst.V, ref.gram(inst.x, inst.wl))[0],
                                                                  4, negative_level=True))
    iv = sims.kmeans1d_intervals(lam, 4, negative_level=True)
    s = StandardSynthesis(ctx, w.pix, 5, 1, 64, 64, precision)
    s.collect(0, inst.x, inst.wl, inst.V, 64, iv)
    s.sync()
    got = s.images[0].double().cpu().numpy()
    t = s.timings()
    s.close()
    err = level_errors(got, img_ref)
    say("full collect max err per level", err[:, 0], "timings ms", t)
    assert np.all(err[:, 0] <= TOL[precision]), err


def test_prestep_batched_equals_single(ctx):
    """bb_synth_prestep_batched over instances of one antenna count (different
    array rotations and wavelengths) gives each instance's bb_synth_prestep
    eigenvalues, weights and level ids; images from its packed outputs match
    the oracle's full steps.  A non-Hermitian or coincident-antenna instance
    fails the whole call, naming that instance."""
    from paper_2310_09200_amd import Batch, BluebildError, StandardSynthesis, _lib
    say("case batched pre-step vs single pre-step, C1 size")
    w = configs.c1(n_ant=48, n_side=40)
    base = w.instance(0)
    insts = [(sims.earth_rotate(base.x, 0.25 * i), base.wl * (1.0 + 0.07 * i)) for i in range(5)]
    g = np.random.default_rng(7)
    Vs = []
    for x, wl in insts:
        src = w.pix[g.choice(w.n_pix, 4, replace=False)]
        Vs.append(sims.add_noise_snr(sims.visibility(x, src, np.exp(g.normal(size=4)), wl), sims.psd_noise(48, g),
                                     20.0))
    lam0, A0 = ref.geneig(Vs[0], ref.gram(insts[0][0], insts[0][1]))
    lam0, _ = ref.select_top(lam0, A0, 40)
    iv = sims.kmeans1d_intervals(lam0, 3, negative_level=True)
    s = StandardSynthesis(ctx, w.pix, 4, 1, 48, 48, "fp32_3m")
    W, lam, d, lev = s.prestep_batched(np.stack([x for x, _ in insts]), [wl for _, wl in insts], np.stack(Vs), 40, iv)
    want = np.zeros((4, w.n_pix))
    for i, ((x, wl), V) in enumerate(zip(insts, Vs)):
        W1, lam1, d1, lev1 = s.prestep(x, wl, V, 40, iv)
        s.sync()
        np.testing.assert_allclose(lam[i].cpu().numpy(), lam1.cpu().numpy(), rtol=1e-12, atol=1e-12 * float(
            lam1.abs().max()))
        assert torch.equal(lev[i], lev1) and torch.equal(d[i], d1)
        # eigenvectors agree up to a phase per column
        ov = torch.abs(torch.sum(torch.conj(W[i]) * W1, dim=0)) / (torch.linalg.norm(W[i], dim=0) *
                                                                     torch.linalg.norm(W1, dim=0))
        assert float(ov.min()) > 1 - 1e-5
        want += ref.collect(V, x, wl, w.pix, 40, iv)[0]
    s.collect_eig_batched(Batch([(0, insts[i][0], insts[i][1], W[i], d[i], lev[i]) for i in range(5)], ctx.device))
    s.sync()
    got = s.images[0].double().cpu().numpy()
    assert np.all(level_errors(got, want)[:, 0] <= 1e-5)
    before = s.images.clone()
    Vb = [V.copy() for V in Vs]
    Vb[3][0, 5] += 1e-3 * np.abs(Vb[3]).max()
    with pytest.raises(BluebildError, match="instance 3"):
        s.prestep_batched(np.stack([x for x, _ in insts]), [wl for _, wl in insts], np.stack(Vb), 40, iv)
    xs = np.stack([x for x, _ in insts])
    xs[2, 7] = xs[2, 6]
    with pytest.raises(BluebildError, match="instance 2") as e:
        s.prestep_batched(xs, [wl for _, wl in insts], np.stack(Vs), 40, iv)
    assert e.value.status == _lib.BB_ERR_NOT_POSDEF
    with pytest.raises(BluebildError) as e:
        s.prestep_batched(np.stack([x for x, _ in insts]), [wl for _, wl in insts], np.stack(Vs), 49, iv)
    assert e.value.status == _lib.BB_ERR_INVALID_ARG   # n_eig > n_ant
    s.sync()
    assert torch.equal(s.images, before)
    s.close()


def test_full_collect_truncated(ctx):
    """n_eig < L keeps the largest eigenvalues (signed), here with the standardized filter."""
    from paper_2310_09200_amd import StandardSynthesis
    say("case full collect truncated, std filter")
    w = configs.c1(n_ant=40, n_side=48)
    inst = w.instance(0)
    lam_all, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
    lam, W = ref.select_top(lam_all, A, 12)
    iv = sims.kmeans1d_intervals(lam, 2, negative_level=True)
    member = ref.level_membership(lam, iv)
    want = ref.synthesize_blas(W, ref.std_filter(lam), member, inst.x, w.pix, inst.wl)
    s = StandardSynthesis(ctx, w.pix, 3, 1, 40, 40, "fp32", filter="std")
    s.collect(0, inst.x, inst.wl, inst.V, 12, iv)
    s.sync()
    got = s.images[0].double().cpu().numpy()
    s.close()
    assert np.all(level_errors(got, want)[:, 0] <= 1e-5)


@pytest.mark.parametrize("fraction", [0.5, 0.9, 1.0])
def test_energy_truncation(ctx, fraction):
    """N_eig chosen on the GPU from the eigenvalues equals the oracle's choice; images match."""
    from paper_2310_09200_amd import StandardSynthesis
    say(f"case energy truncation {fraction}")
    w = configs.c1(n_ant=48, n_side=40)
    inst = w.instance(0)
    lam_all, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
    k = ref.n_eig_for_energy(lam_all, fraction)
    lam, W = ref.select_top(lam_all, A, k)
    iv = sims.kmeans1d_intervals(lam_all, 2, negative_level=True)
    member = ref.level_membership(lam, iv)
    want = ref.synthesize_blas(W, lam, member, inst.x, w.pix, inst.wl)
    s = StandardSynthesis(ctx, w.pix, 3, 1, 48, 48, "fp32_3m")
    k_gpu = s.collect_energy(0, inst.x, inst.wl, inst.V, fraction, iv)
    s.sync()
    got = s.images[0].double().cpu().numpy()
    s.close()
    assert k_gpu == k
    assert np.all(level_errors(got, want)[:, 0] <= 1e-5)


@pytest.mark.parametrize("n_beam", [20, 48])
def test_beamformed_collect(ctx, n_beam):
    """Beamforming (Section 2.7) on the GPU vs the oracle: G^W = W^H G W, U = W alpha."""
    from paper_2310_09200_amd import StandardSynthesis
    say(f"case beamformed n_beam={n_beam}")
    w = configs.c1(n_ant=48, n_side=40)
    inst = w.instance(0)
    g = np.random.default_rng(n_beam)
    Wbf = (g.standard_normal((48, n_beam)) + 1j * g.standard_normal((48, n_beam))) / np.sqrt(48)
    Vw = Wbf.conj().T @ inst.V @ Wbf
    Vw = 0.5 * (Vw + Vw.conj().T)
    n_eig = n_beam // 2
    lam_all, _ = ref.geneig(Vw, Wbf.conj().T @ ref.gram(inst.x, inst.wl) @ Wbf)
    iv = sims.kmeans1d_intervals(np.sort(lam_all)[::-1][:n_eig], 2, negative_level=True)
    want, lam, U, member = ref.collect_beamformed(Vw, Wbf, inst.x, inst.wl, w.pix, n_eig, iv)
    s = StandardSynthesis(ctx, w.pix, 3, 1, 48, 48, "fp32_3m")
    s.collect_beamformed(0, inst.x, inst.wl, Wbf, Vw, n_eig, iv)
    s.sync()
    got = s.images[0].double().cpu().numpy()
    s.close()
    err = level_errors(got, want)
    say("beamformed max err per level", err[:, 0])
    assert np.all(err[:, 0] <= 1e-5), err


def test_identity_gram_gives_dirty_image(ctx):
    """gram='identity': the pipeline returns the back-projected image diag(Psi V Psi*) (Section 2.8)."""
    from paper_2310_09200_amd import StandardSynthesis
    say("case G = I back-projection")
    w = configs.c1(n_ant=48, n_side=48)
    inst = w.instance(0)
    want = ref.backprojection_image(inst.V, inst.x, w.pix, inst.wl)
    s = StandardSynthesis(ctx, w.pix, 1, 1, 48, 48, "fp32_3m", gram="identity")
    s.collect(0, inst.x, inst.wl, inst.V, 48, np.array([[-np.inf, np.inf]]))
    s.sync()
    got = s.images[0, 0].double().cpu().numpy()
    s.close()
    assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want))


@pytest.mark.parametrize("precision", ["fp32", "fp32_3m", "bf16x3", "bf16x3_3m"])
def test_batched_uneven_instances(ctx, precision):
    """One launch over uneven instances in several slots equals the per-slot oracle sums."""
    from paper_2310_09200_amd import Batch, StandardSynthesis
    say(f"case batched precision={precision}")
    w = configs.c4(n_channels=3, n_steps=4, n_side=40)
    items, want = [], np.zeros((3, 4, w.n_pix))
    for i in range(w.n_instances()):
        inst = w.instance(i)
        items.append((inst.slot, inst.x, inst.wl, inst.W, inst.lam, inst.level_of))
        Wc = inst.W.astype(np.complex64).astype(np.complex128)
        want[inst.slot] += oracle_images(Wc, inst.lam.astype(np.float32), inst.level_of, inst.x, inst.wl, w.pix, 4)
    b = Batch(items, ctx.device)
    s = StandardSynthesis(ctx, w.pix, 4, 3, 512, 128, precision)
    s.collect_eig_batched(b)
    s.sync()
    got = s.images.double().cpu().numpy()
    s.close()
    for sl in range(3):
        err = level_errors(got[sl], want[sl])
        say("slot", sl, "max err", err[:, 0])
        assert np.all(err[:, 0] <= TOL[precision]), (sl, err)


@pytest.fixture(scope="module")
def tile_case():
    """Instances of every K class (K = 20, 50, 100, 200) over two slots, ragged antenna and pixel counts."""
    g = np.random.default_rng(77)
    pix = sims.pixel_grid(45, 6.0, 60.0)
    wl = sims.wavelength_m(150e6)
    items, want = [], np.zeros((2, 3, pix.shape[0]))
    for i, (L, K) in enumerate([(70, 20), (90, 50), (60, 100), (130, 200), (45, 33)]):
        x = sims.disk_layout(L, 3000.0, g, z_sigma_m=2.0)
        W = sims.random_eigvecs(L, K, g).astype(np.complex64)
        d = g.normal(0, 1, K).astype(np.float32)
        lev = g.integers(-1, 3, K).astype(np.int32)
        items.append((i % 2, x, wl, W, d, lev))
        want[i % 2] += oracle_images(W.astype(np.complex128), d.astype(np.float64), lev, x, wl, pix, 3)
    return pix, items, want


@pytest.mark.parametrize("precision", ["fp32", "fp32_3m", "bf16x3", "bf16x3_3m"])
def test_every_tile_shape(ctx, tile_case, precision):
    """Every tile shape each K class may use images a mixed batch within the oracle tolerance."""
    from paper_2310_09200_amd import Batch, StandardSynthesis, tile_shapes
    pix, items, want = tile_case
    shapes = tile_shapes(precision)
    allowed = [[t for t, *_, cl in shapes if c in cl] for c in range(4)]
    for j in range(max(len(a) for a in allowed)):
        tiles = [a[j % len(a)] for a in allowed]
        say(f"case tiles precision={precision} tiles={tiles}")
        s = StandardSynthesis(ctx, pix, 3, 2, 130, 200, precision)
        s.tiles = tiles
        assert s.tiles == tiles
        s.collect_eig_batched(Batch(items, ctx.device))
        s.sync()
        got = s.images.double().cpu().numpy()
        s.close()
        for sl in range(2):
            err = level_errors(got[sl], want[sl])
            assert np.all(err[:, 0] <= TOL[precision]), (tiles, sl, err)


def test_autotune_keeps_images_and_picks_candidates(ctx, tile_case):
    """Autotuning times the candidates on the batch without touching the handle's images; the chosen
    tiles are candidates of their class, and the handle then images the batch correctly."""
    from paper_2310_09200_amd import Batch, BluebildError, StandardSynthesis, tile_shapes
    say("case autotune")
    pix, items, want = tile_case
    s = StandardSynthesis(ctx, pix, 3, 2, 130, 200, "fp32_3m")
    b = Batch(items, ctx.device)
    reps = 2
    ms, scratch = s.autotune_batched(b, reps=reps, return_scratch=True)
    s.sync()
    assert torch.count_nonzero(s.images).item() == 0
    shapes = tile_shapes("fp32_3m")
    assert sorted(ms) == [0, 1, 2, 3]
    for c, row in ms.items():
        assert set(row) == {t for t, *_, cl in shapes if c in cl} and min(row.values()) > 0
        assert s.tiles[c] == min(row, key=row.get)
    # every timed launch (one warm-up + reps per candidate) imaged its class's instances into the scratch
    kclass = [min(3, (int(np.ceil(W.shape[1] / 32)) * 32 > 32) + (int(np.ceil(W.shape[1] / 32)) * 32 > 64)
                  + (int(np.ceil(W.shape[1] / 32)) * 32 > 128)) for _, _, _, W, _, _ in items]
    want_scr = np.zeros_like(want)
    for (slot, x, wl, W, d, lev), c in zip(items, kclass):
        want_scr[slot] += (reps + 1) * len(ms[c]) * oracle_images(W.astype(np.complex128), d.astype(np.float64),
                                                                   lev, x, wl, pix, 3)
    got_scr = scratch.double().cpu().numpy()
    for sl in range(2):
        assert np.all(level_errors(got_scr[sl], want_scr[sl])[:, 0] <= 1e-5)
    s.collect_eig_batched(b)
    s.sync()
    got = s.images.double().cpu().numpy()
    for sl in range(2):
        assert np.all(level_errors(got[sl], want[sl])[:, 0] <= 1e-5)
    with pytest.raises(BluebildError):
        s.tiles = [0, 0, 0, 0]        # a 256-eigenpair tile is not a candidate for K <= 32
    s.tiles = [-1, -1, -1, -1]        # defaults
    assert s.tiles == [3, 9, 11, 0]
    s.close()


@pytest.fixture(scope="module")
def c2_case():
    """Twelve C2 epochs spread over the 6 h track, FP64 oracle eigenpairs, sampled pixels.

    Pixels: every 8th row and column of the 1024^2 grid, the 9 x 9
    neighbourhood of every point source, and the last pixel.
    """
    w = configs.c2(n_steps=100)
    steps = np.linspace(0, 99, 12).round().astype(int)
    sel = sims.sample_pixels(w.n_side, w.source_pixels(), stride=8)
    want = np.zeros((9, sel.size))
    iv = None
    items = []
    for st in steps:
        inst = w.instance(int(st))
        lam, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
        lam, W = ref.select_top(lam, A, 512)
        if iv is None:
            iv = sims.kmeans1d_intervals(lam, 8, negative_level=True)
        lev = sims.levels_from_intervals(lam, iv)
        W64 = W.astype(np.complex64)
        want += oracle_images(W64.astype(np.complex128), lam.astype(np.float32), lev, inst.x, inst.wl, w.pix[sel], 9)
        items.append((0, inst.x, inst.wl, W64, lam.astype(np.float32), lev))
    return w, steps, sel, items, want


@pytest.mark.parametrize("precision", ["fp32", "fp32_3m", "bf16x3", "bf16x3_3m"])
def test_c2_full_size_sampled(ctx, c2_case, precision):
    """C2 at full size (L=512, K=512, 1024^2, 8+1 levels) in the benchmarked launch (batched), sampled pixels."""
    from paper_2310_09200_amd import Batch, StandardSynthesis
    w, steps, sel, items, want = c2_case
    say(f"case C2 full size precision={precision} epochs={len(steps)} sampled pixels={sel.size}")
    s = StandardSynthesis(ctx, w.pix, 9, 1, 512, 512, precision)
    s.collect_eig_batched(Batch(items, ctx.device))
    s.sync()
    got = s.images[0][:, torch.as_tensor(sel, device=ctx.device)].double().cpu().numpy()
    s.close()
    err = level_errors(got, want)
    say("C2 max err per level", err[:, 0])
    say("C2 rms err per level", err[:, 1])
    assert np.all(err[:, 0] <= TOL[precision]), err


def test_single_and_batched_launch_agree(ctx):
    """collect_eig per instance and one batched launch give the same images (to FP32 summation order)."""
    from paper_2310_09200_amd import Batch, StandardSynthesis
    say("case single vs batched")
    g = np.random.default_rng(77)
    pix = sims.pixel_grid(48, 5.0, 90.0)
    items = []
    for i in range(5):
        L, K = int(g.integers(30, 200)), int(g.integers(5, 150))
        x = sims.disk_layout(L, 2000.0, g)
        items.append((i % 2, x, 2.0, sims.random_eigvecs(L, K, g), g.normal(0, 1, K), g.integers(-1, 3, K)))
    a = StandardSynthesis(ctx, pix, 3, 2, 256, 256, "fp32_3m")
    for it in items:
        a.collect_eig(*it)
    b = StandardSynthesis(ctx, pix, 3, 2, 256, 256, "fp32_3m")
    b.collect_eig_batched(Batch(items, ctx.device))
    a.sync()
    b.sync()
    ia, ib = a.images.double().cpu().numpy(), b.images.double().cpu().numpy()
    a.close()
    b.close()
    assert np.max(np.abs(ia - ib)) <= 1e-6 * np.max(np.abs(ia))


# ---------------------------------------------------------------- error paths (forced from the host)
def _status(fn):
    from paper_2310_09200_amd import BluebildError
    with pytest.raises(BluebildError) as e:
        fn()
    return e.value.status


def test_error_codes_from_host(ctx):
    from paper_2310_09200_amd import StandardSynthesis, _lib
    say("case error codes")
    g = np.random.default_rng(0)
    pix = sims.pixel_grid(8, 5.0, 90.0)
    s = StandardSynthesis(ctx, pix, 2, 1, 16, 16)
    x = sims.disk_layout(16, 100.0, g)
    V = sims.add_noise_snr(sims.visibility(x, pix[:3], np.ones(3), 2.0), sims.psd_noise(16, g), 10.0)
    iv = np.array([[1.0, np.inf], [-np.inf, 0.5]])
    before = s.images.clone()
    # shape beyond the handle's maxima
    assert _status(lambda: s.collect(0, np.zeros((17, 3)), 2.0, np.eye(17), 4, iv)) == _lib.BB_ERR_SHAPE
    # bad slot, bad wavelength, n_eig > n_ant
    assert _status(lambda: s.collect(1, x, 2.0, V, 4, iv)) == _lib.BB_ERR_INVALID_ARG
    assert _status(lambda: s.collect(0, x, -2.0, V, 4, iv)) == _lib.BB_ERR_INVALID_ARG
    assert _status(lambda: s.collect(0, x, float("nan"), V, 4, iv)) == _lib.BB_ERR_INVALID_ARG
    # interval with min > max, overlapping intervals, NaN bound
    assert _status(lambda: s.collect(0, x, 2.0, V, 4, np.array([[2.0, 1.0], [-1.0, 0.0]]))) == _lib.BB_ERR_INVALID_ARG
    assert _status(lambda: s.collect(0, x, 2.0, V, 4, np.array([[0.0, 2.0], [1.0, 3.0]]))) == _lib.BB_ERR_INVALID_ARG
    assert _status(lambda: s.collect(0, x, 2.0, V, 4, np.array([[np.nan, 2.0], [-1.0, 0.0]]))) == _lib.BB_ERR_INVALID_ARG
    # non-Hermitian or NaN visibilities (V is a correlation matrix, Section 2.1)
    Vb = V.copy()
    Vb[0, 5] += 1e-3 * np.abs(V).max()
    assert _status(lambda: s.collect(0, x, 2.0, Vb, 4, iv)) == _lib.BB_ERR_INVALID_ARG
    Vn = V.copy()
    Vn[2, 2] = np.nan
    assert _status(lambda: s.collect(0, x, 2.0, Vn, 4, iv)) == _lib.BB_ERR_INVALID_ARG
    # coincident antennas: G is singular, the Cholesky factorisation fails
    x2 = x.copy()
    x2[3] = x2[2]
    assert _status(lambda: s.collect(0, x2, 2.0, V, 4, iv)) == _lib.BB_ERR_NOT_POSDEF
    s.sync()
    assert torch.equal(s.images, before)  # failed calls leave the images untouched
    # level id out of range is reported by sync and ignored
    W = sims.random_eigvecs(16, 4, g)
    s.collect_eig(0, x, 2.0, W, np.ones(4), np.array([0, 5, 1, -1], np.int32))
    assert _status(lambda: s.sync()) == _lib.BB_ERR_INVALID_ARG
    s.sync()  # flag cleared
    # too small a workspace
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.bb_synth_create(ctx.handle, ctypes.byref(s.opt), s.n_pix, ctypes.c_void_p(s.pix_cm.data_ptr()),
                             ctypes.c_void_p(s.images.data_ptr()), ctypes.c_void_p(s.workspace.data_ptr()), 1024,
                             ctypes.byref(h))
    assert st == _lib.BB_ERR_WORKSPACE
    # destroying a context with a live handle
    assert lib.bb_context_destroy(ctx.handle) == _lib.BB_ERR_STATE
    s.close()


def test_reset_and_count(ctx):
    from paper_2310_09200_amd import StandardSynthesis
    say("case reset/count")
    g = np.random.default_rng(1)
    pix = sims.pixel_grid(8, 5.0, 90.0)
    s = StandardSynthesis(ctx, pix, 1, 1, 8, 8)
    x = sims.disk_layout(8, 100.0, g)
    s.collect_eig(0, x, 2.0, sims.random_eigvecs(8, 8, g), np.ones(8), np.zeros(8, np.int32))
    s.sync()
    assert s.count == 1 and float(s.images.abs().sum()) > 0
    s.reset()
    s.sync()
    assert s.count == 0 and float(s.images.abs().sum()) == 0
    s.count = 7
    assert s.count == 7
    s.close()


@pytest.mark.gpu
def test_phase_probe_against_fp64(ctx):
    """The phase-generation probe sums cos + sin of every (antenna, pixel) phase with the kernel's arithmetic."""
    from paper_2310_09200_amd import phase_probe
    g = np.random.default_rng(11)
    n_ant, n_pix, reps, wl = 37, 1000, 3, 1.9986
    x = g.uniform(-2.5e4, 2.5e4, (n_ant, 3))
    p = g.normal(size=(n_pix, 3))
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    say(f"case phase probe n_ant={n_ant} n_pix={n_pix} reps={reps}")
    got = phase_probe(ctx, x, wl, p, reps).cpu().numpy().astype(np.float64)
    t = p @ x.T / wl  # turns, FP64
    want = reps * (np.cos(2 * np.pi * t) + np.sin(2 * np.pi * t)).sum(axis=1)
    # per term: ~1.3e-7 (hardware sin/cos) + 3e-8 (FP32 argument); the FP32 running sum of 111 terms adds
    # at most ~1e-4 at the magnitudes reached here
    assert np.max(np.abs(got - want)) < 2e-4


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["fp32", "fp32_3m", "bf16x3_3m"])
def test_maximum_sizes_against_oracle(ctx, precision):
    """The largest instance the library accepts: 1024 antennas (the workgroup's LDS position table full) and
    1024 eigenpairs (four K passes of the K > 128 tile), ragged pixel count."""
    L, K, n_side = 1024, 1024, 13
    say(f"case maximum sizes L={L} K={K} n_side={n_side} precision={precision}")
    g = np.random.default_rng(77)
    x = sims.disk_layout(L, 20000.0, g, z_sigma_m=5.0)
    wl = sims.wavelength_m(150e6)
    pix = sims.pixel_grid(n_side, 4.0, 50.0)
    W = sims.random_eigvecs(L, K, g)
    d = g.normal(0, 1, K)
    n_levels = 4
    lev = g.integers(-1, n_levels, K).astype(np.int32)
    d32 = d.astype(np.float32).astype(np.float64)
    want = oracle_images(W.astype(np.complex64).astype(np.complex128), d32, lev, x, wl, pix, n_levels)
    got = run_eig(ctx, pix, n_levels, x, wl, W, d, lev, precision)
    err = level_errors(got, want)
    say("max err per level", err[:, 0])
    assert np.all(err[:, 0] <= TOL[precision]), err


@pytest.mark.gpu
@pytest.mark.parametrize("L,K,n_pix", [(1, 1, 1), (1, 1, 97), (33, 1, 1), (2, 2, 2), (40, 40, 1)])
def test_degenerate_sizes(ctx, L, K, n_pix):
    """One antenna, one eigenpair, one pixel: tiles that are almost entirely padding."""
    say(f"case degenerate L={L} K={K} n_pix={n_pix}")
    g = np.random.default_rng(300 + L + K + n_pix)
    x = g.uniform(-500.0, 500.0, (L, 3))
    wl = 2.0
    pix = g.normal(size=(n_pix, 3)) + np.array([0.0, 0.0, 4.0])
    pix /= np.linalg.norm(pix, axis=1, keepdims=True)
    W = (g.normal(size=(L, K)) + 1j * g.normal(size=(L, K))) / np.sqrt(2 * L)
    d = np.abs(g.normal(0, 1, K)) + 0.5
    lev = np.zeros(K, np.int32)
    d32 = d.astype(np.float32).astype(np.float64)
    want = oracle_images(W.astype(np.complex64).astype(np.complex128), d32, lev, x, wl, pix, 1)
    for precision in ("fp32", "fp32_3m", "bf16x3", "bf16x3_3m"):
        got = run_eig(ctx, pix, 1, x, wl, W, d, lev, precision)
        err = level_errors(got, want)
        assert np.all(err[:, 0] <= TOL[precision]), (precision, err)


@pytest.mark.gpu
def test_empty_batch_is_rejected(ctx):
    """A batch of zero instances is an argument error and leaves the images untouched."""
    from paper_2310_09200_amd import StandardSynthesis, _lib
    say("case empty batch")
    s = StandardSynthesis(ctx, sims.pixel_grid(8, 5.0, 90.0), 2, 1, 16, 16)
    sz = ctypes.c_size_t()
    assert s.lib.bb_batched_workspace_size(s.handle, 0, None, ctypes.byref(sz)) == _lib.BB_ERR_INVALID_ARG
    # valid (dummy) device buffers, so that the empty instance table is what gets rejected
    dev = ctx.device
    ant = torch.zeros(3, dtype=torch.float64, device=dev)
    W = torch.zeros(2, dtype=torch.float32, device=dev)
    d = torch.zeros(1, dtype=torch.float32, device=dev)
    lev = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.zeros(4096, dtype=torch.uint8, device=dev)
    ws_ptr = (ws.data_ptr() + 255) // 256 * 256
    st = s.lib.bb_synth_collect_eig_batched(s.handle, 0, None, 1, 1, 1, ctypes.c_void_p(ant.data_ptr()),
                                            ctypes.c_void_p(W.data_ptr()), ctypes.c_void_p(d.data_ptr()),
                                            ctypes.c_void_p(lev.data_ptr()), ctypes.c_void_p(ws_ptr), 2048)
    assert st == _lib.BB_ERR_INVALID_ARG
    assert b"empty" in s.lib.bb_last_error(ctx.handle)
    s.sync()
    assert torch.count_nonzero(s.images).item() == 0
    s.close()


@pytest.mark.gpu
def test_batched_instance_table_out_of_range_is_rejected(ctx):
    """An instance whose W block or eigenpairs run past the packed arrays is an argument error.

    The lengths of the packed arrays go into the call, so a wrong table is
    caught on the host: nothing is enqueued and the images stay as they were.
    """
    from paper_2310_09200_amd import Batch, StandardSynthesis, _lib
    say("case batched table out of range")
    g = np.random.default_rng(4)
    L, K = 40, 24
    x = sims.disk_layout(L, 100.0, g)
    W = (g.normal(size=(L, K)) + 1j * g.normal(size=(L, K))) / np.sqrt(2 * L)
    d = np.ones(K)
    lev = np.zeros(K, np.int32)
    s = StandardSynthesis(ctx, sims.pixel_grid(16, 5.0, 90.0), 1, 1, 64, 32)
    b = Batch([(0, x, 2.0, W, d, lev), (0, x, 2.0, W, d, lev)], ctx.device)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    ws = torch.zeros(1 << 22, dtype=torch.uint8, device=ctx.device)
    ws_ptr = ctypes.c_void_p((ws.data_ptr() + 255) // 256 * 256)
    for field, delta in (("w_off", 1), ("eig_off", 1), ("w_off", L * K), ("eig_off", K)):
        inst = [_lib.bb_instance(n_ant=i.n_ant, n_eig=i.n_eig, slot=i.slot, wavelength_m=i.wavelength_m,
                                 ant_off=i.ant_off, w_off=i.w_off, eig_off=i.eig_off) for i in b.inst]
        setattr(inst[1], field, getattr(inst[1], field) + delta)
        arr = (_lib.bb_instance * 2)(*inst)
        st = s.lib.bb_synth_collect_eig_batched(s.handle, 2, arr, b.n_ant_rows, b.n_w, b.n_eig_rows, vp(b.ant),
                                                vp(b.W), vp(b.d), vp(b.lev), ws_ptr, (1 << 22) - 256)
        assert st == _lib.BB_ERR_INVALID_ARG, (field, delta, st)
        assert b"beyond the" in s.lib.bb_last_error(ctx.handle)
    s.sync()
    assert torch.count_nonzero(s.images).item() == 0
    s.collect_eig_batched(b)  # the table itself is valid
    s.sync()
    assert torch.count_nonzero(s.images).item() > 0
    s.close()


@pytest.mark.gpu
def test_phase_probe_rejects_bad_arguments(ctx):
    """Sizes out of range and null pointers are argument errors, found before anything is enqueued."""
    from paper_2310_09200_amd import _lib
    say("case phase probe errors")
    dev = ctx.device
    x = torch.zeros(3 * 1025, dtype=torch.float64, device=dev)
    p = torch.zeros(3 * 4, dtype=torch.float64, device=dev)
    out = torch.full((4,), 7.0, dtype=torch.float32, device=dev)
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    lib, h = ctx.lib, ctx.handle
    assert lib.bb_phase_probe(h, 0, 2.0, vp(x), 4, vp(p), 1, vp(out)) == _lib.BB_ERR_INVALID_ARG
    assert lib.bb_phase_probe(h, 1025, 2.0, vp(x), 4, vp(p), 1, vp(out)) == _lib.BB_ERR_INVALID_ARG
    assert lib.bb_phase_probe(h, 3, 2.0, vp(x), 0, vp(p), 1, vp(out)) == _lib.BB_ERR_INVALID_ARG
    assert lib.bb_phase_probe(h, 3, 2.0, vp(x), 4, vp(p), 0, vp(out)) == _lib.BB_ERR_INVALID_ARG
    assert lib.bb_phase_probe(h, 3, -1.0, vp(x), 4, vp(p), 1, vp(out)) == _lib.BB_ERR_INVALID_ARG
    assert lib.bb_phase_probe(h, 3, 2.0, None, 4, vp(p), 1, vp(out)) == _lib.BB_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert torch.all(out == 7.0)  # nothing was written
