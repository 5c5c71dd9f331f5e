"""Full-size workloads on the GPU, checked on sampled pixels against the FP64 oracle.

C3: SKA-Low-like precision study (L=512, K=512, 2048^2 pixels, 65 km baselines),
    FP32 and BF16x3 contraction, several epochs in one batched launch.
C4: 2048 uneven instances (L 200..512, K 16..128, 64 channel slots, 512^2 pixels)
    in one batched call, all four contraction modes.
C2 pre-step: one LOFAR-like epoch (L=512) through the full step on the GPU
    (FP64 Gram, rocSOLVER generalized eigensolve, selection, synthesis).
Translation: a geocentric offset of every antenna leaves the images unchanged
    (the FP64 phase argument and its exact reduction).
"""

import sys

import numpy as np
import pytest
import torch

import oracle as ref
import sims
from sims import configs
from tests._helpers import level_errors

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-4, "bf16x3_3m": 1e-4}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2310_09200_amd import Context
    return Context(0)


@pytest.fixture(scope="module")
def c3_case():
    w = configs.c3()
    epochs = [0, 17, 33, 49]
    sel = sims.sample_pixels(w.n_side, w.source_pixels(), 64)
    items, want, iv = [], np.zeros((9, sel.size)), None
    for e in epochs:
        inst = w.instance(e)
        lam, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
        lam, W = ref.select_top(lam, A, 512)
        if iv is None:
            iv = sims.kmeans1d_intervals(lam, 8, negative_level=True)
        lev = sims.levels_from_intervals(lam, iv)
        W64 = W.astype(np.complex64)
        items.append((0, inst.x, inst.wl, W64, lam.astype(np.float32), lev))
        member = ref.membership_from_level_of(lev, 9)
        want += ref.synthesize_blas(W64.astype(np.complex128), lam.astype(np.float32).astype(np.float64),
                                    member, inst.x, w.pix[sel], inst.wl)
    return w, sel, items, want


@pytest.mark.parametrize("precision", ["fp32", "fp32_3m", "bf16x3", "bf16x3_3m"])
def test_c3_precision_study(ctx, c3_case, precision):
    from paper_2310_09200_amd import Batch, StandardSynthesis
    w, sel, items, want = c3_case
    say(f"case C3 full size precision={precision} epochs={len(items)} sampled pixels={sel.size}")
    s = StandardSynthesis(ctx, w.pix, 9, 1, 512, 512, precision)
    s.collect_eig_batched(Batch(items, ctx.device))
    s.sync()
    got = s.images[0][:, torch.as_tensor(sel, device=ctx.device)].double().cpu().numpy()
    s.close()
    err = level_errors(got, want)
    say(f"C3 {precision} per-level max err {np.array2string(err[:, 0], formatter={'float_kind': lambda v: f'{v:.2e}'})}")
    say(f"C3 {precision} per-level rms err {np.array2string(err[:, 1], formatter={'float_kind': lambda v: f'{v:.2e}'})}")
    assert np.all(err[:, 0] <= TOL[precision]), err


@pytest.fixture(scope="module")
def c4_case():
    """All 2048 C4 instances and the FP64 oracle's per-slot sums on 98 sampled pixels."""
    w = configs.c4()
    n_inst = w.n_instances()
    g = np.random.default_rng(44)
    sel = np.unique(np.concatenate([g.choice(w.n_pix, 96, replace=False), [0, w.n_pix - 1]]))
    items = []
    want = np.zeros((64, 4, sel.size))
    for i in range(n_inst):
        inst = w.instance(i)
        W64 = inst.W.astype(np.complex64)
        items.append((inst.slot, inst.x, inst.wl, W64, inst.lam.astype(np.float32), inst.level_of))
        member = ref.membership_from_level_of(inst.level_of, 4)
        want[inst.slot] += ref.synthesize_blas(W64.astype(np.complex128),
                                               inst.lam.astype(np.float32).astype(np.float64), member, inst.x,
                                               w.pix[sel], inst.wl)
    return w, sel, items, want


@pytest.mark.parametrize("precision", ["fp32_3m", "fp32", "bf16x3", "bf16x3_3m"])
def test_c4_batched_full_size(ctx, c4_case, precision):
    """C4 in one batched call (every K class, the default tile of each), all four contraction modes."""
    from paper_2310_09200_amd import Batch, StandardSynthesis
    w, sel, items, want = c4_case
    say(f"case C4 full size precision={precision}: {len(items)} instances, {w.meta['n_channels']} slots, "
        f"{w.n_pix} pixels")
    batch = Batch(items, ctx.device)
    s = StandardSynthesis(ctx, w.pix, 4, 64, 512, 128, precision)
    say(f"C4 products {batch.products * w.n_pix:.3e}, tiles {s.tiles}")
    s.collect_eig_batched(batch)
    s.sync()
    t = s.timings()
    got = s.images[:, :, torch.as_tensor(sel, device=ctx.device)].double().cpu().numpy()
    s.close()
    say(f"C4 {precision} synthesis kernels {t[2]:.1f} ms -> {batch.products * w.n_pix / (t[2] / 1e3):.3e} products/s")
    worst = 0.0
    for sl in range(64):
        err = level_errors(got[sl], want[sl])
        worst = max(worst, float(np.max(err[:, 0])))
    say(f"C4 {precision} worst per-level max err over 64 slots: {worst:.2e}")
    assert worst <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp32_3m", "bf16x3_3m"])
def test_c2_full_step_prestep_on_gpu(ctx, precision):
    """Full Algorithm 1 step at the C2 size: GPU Gram + FP64 eigensolve (L = 512) + selection + synthesis.

    Compared with the oracle's own full step (Gram, Cholesky reduction and
    eigh in FP64, selection, closed-interval levels) on sampled pixels of the
    1024^2 grid.  The eigenvectors of the two eigensolvers differ by a phase
    per eigenpair (the images do not); the level bounds sit at eigenvalue-gap
    midpoints, so membership does not depend on the last bits of either solver.
    """
    from paper_2310_09200_amd import StandardSynthesis
    w = configs.c2(n_steps=100)
    inst = w.instance(37)
    say(f"case C2 full step (GPU pre-step) precision={precision}, epoch 37")
    sel = sims.sample_pixels(w.n_side, w.source_pixels(), 16)
    lam, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
    lam, W = ref.select_top(lam, A, 512)
    iv = sims.kmeans1d_intervals(lam, 8, negative_level=True)
    want, lam_o, _, _ = ref.collect(inst.V, inst.x, inst.wl, w.pix[sel], 512, iv)
    s = StandardSynthesis(ctx, w.pix, 9, 1, 512, 512, precision)
    s.collect(0, inst.x, inst.wl, inst.V, 512, iv)
    s.sync()
    got = s.images[0][:, torch.as_tensor(sel, device=ctx.device)].double().cpu().numpy()
    Wg, lam_g, _, lev_g = s.prestep(inst.x, inst.wl, inst.V, 512, iv)
    s.sync()
    s.close()
    lam_g = lam_g.cpu().numpy()
    say(f"eigenvalues: max |GPU - oracle| / max |lam| = {np.max(np.abs(lam_g - lam_o)) / np.max(np.abs(lam_o)):.2e}")
    assert np.max(np.abs(lam_g - lam_o)) <= 1e-10 * np.max(np.abs(lam_o))
    assert np.array_equal(lev_g.cpu().numpy(), sims.levels_from_intervals(lam_o, iv))
    err = level_errors(got, want)
    say(f"C2 full step {precision} per-level max err {err[:, 0]}")
    assert np.all(err[:, 0] <= TOL[precision]), err


@pytest.mark.parametrize("precision", ["fp32_3m", "bf16x3_3m"])
def test_geocentric_translation_leaves_images_unchanged(ctx, precision):
    """Translation invariance on the GPU: every antenna moved by (6.4e6, -1.1e6, 3.3e5) m.

    The phase of every antenna at a pixel shifts by the same <c, p> / lambda
    (about 3.3e6 turns here), which |E|^2 does not see.  With an FP32 phase
    argument the shift alone would leave errors of order one; with the FP64
    argument and its exact reduction the images stay within the contraction's
    own rounding.  SKA-Low-like epoch (512 stations, 65 km baselines), full
    2048^2 grid; both images also checked against the oracle on sampled pixels.
    """
    from paper_2310_09200_amd import StandardSynthesis
    w = configs.c3()
    inst = w.instance(11)
    say(f"case geocentric translation precision={precision}")
    lam, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
    lam, W = ref.select_top(lam, A, 512)
    iv = sims.kmeans1d_intervals(lam, 8, negative_level=True)
    lev = sims.levels_from_intervals(lam, iv)
    W64 = W.astype(np.complex64)
    shift = np.array([6.4e6, -1.1e6, 3.3e5])
    imgs = []
    for x in (inst.x, inst.x + shift[None, :]):
        s = StandardSynthesis(ctx, w.pix, 9, 1, 512, 512, precision)
        s.collect_eig(0, x, inst.wl, W64, lam.astype(np.float32), lev)
        s.sync()
        imgs.append(s.images[0].double().cpu().numpy())
        s.close()
    err = level_errors(imgs[1], imgs[0])
    say(f"translated vs original, per-level max {err[:, 0]}")
    assert np.all(err[:, 0] <= 1e-5), err
    sel = sims.sample_pixels(w.n_side, w.source_pixels(), 128)
    member = ref.membership_from_level_of(lev, 9)
    want = ref.synthesize_blas(W64.astype(np.complex128), lam.astype(np.float32).astype(np.float64), member,
                               inst.x, w.pix[sel], inst.wl)
    for img in imgs:
        e = level_errors(img[:, sel], want)
        assert np.all(e[:, 0] <= TOL[precision]), e


def test_c2_batched_prestep_then_batched_synthesis(ctx):
    """Algorithm 1 over several epochs with the pre-step batched: one
    strided-batched FP64 eigensolve for all epochs (L = 512), then one batched
    synthesis launch over its packed outputs.  Eigenvalues and level ids
    against the oracle's per epoch; images against the oracle's full steps
    summed over the epochs, on sampled pixels of the 1024^2 grid."""
    from paper_2310_09200_amd import Batch, StandardSynthesis
    w = configs.c2(n_steps=100)
    epochs = [3, 41, 77, 98]
    say(f"case C2 batched pre-step, epochs {epochs}")
    sel = sims.sample_pixels(w.n_side, w.source_pixels(), 32)
    insts = [w.instance(e) for e in epochs]
    lam0, A0 = ref.geneig(insts[0].V, ref.gram(insts[0].x, insts[0].wl))
    lam0, _ = ref.select_top(lam0, A0, 512)
    iv = sims.kmeans1d_intervals(lam0, 8, negative_level=True)
    want = np.zeros((9, sel.size))
    lam_o = []
    for inst in insts:
        img, lam, _, _ = ref.collect(inst.V, inst.x, inst.wl, w.pix[sel], 512, iv)
        want += img
        lam_o.append(lam)
    s = StandardSynthesis(ctx, w.pix, 9, 1, 512, 512, "fp32_3m")
    W, lam_g, d, lev = s.prestep_batched(np.stack([i.x for i in insts]), [i.wl for i in insts],
                                         np.stack([i.V for i in insts]), 512, iv)
    s.sync()
    t = s.timings()
    say(f"batched pre-step of {len(epochs)} epochs: {t[0] + t[1]:.1f} ms")
    lam_g = lam_g.cpu().numpy()
    for e, lo in enumerate(lam_o):
        assert np.max(np.abs(lam_g[e] - lo)) <= 1e-10 * np.max(np.abs(lo)), e
        assert np.array_equal(lev[e].cpu().numpy(), sims.levels_from_intervals(lo, iv)), e
    items = [(0, insts[e].x, insts[e].wl, W[e], d[e], lev[e]) for e in range(len(epochs))]
    s.collect_eig_batched(Batch(items, ctx.device))
    s.sync()
    got = s.images[0][:, torch.as_tensor(sel, device=ctx.device)].double().cpu().numpy()
    s.close()
    err = level_errors(got, want)
    say(f"C2 batched pre-step + synthesis per-level max err {err[:, 0]}")
    assert np.all(err[:, 0] <= 1e-5), err
