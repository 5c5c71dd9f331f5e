"""Full-size workloads on the GPU, checked on sampled pixels against the FP64 oracle.

C3: SKA-Low-like precision study (L=512, K=512, 2048^2 pixels, 65 km baselines),
    FP32 and BF16x3 contraction, several epochs in one batched launch.
C4: 2048 uneven instances (L 200..512, K 16..128, 64 channel slots, 512^2 pixels)
    in one batched launch.
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


def sample_pixels(n_side, src, stride):
    iy, ix = np.meshgrid(np.arange(0, n_side, stride), np.arange(0, n_side, stride), indexing="ij")
    sel = set((iy * n_side + ix).ravel().tolist())
    for p in src:
        cy, cx = divmod(int(p), n_side)
        for dy in range(-4, 5):
            for dx in range(-4, 5):
                if 0 <= cy + dy < n_side and 0 <= cx + dx < n_side:
                    sel.add((cy + dy) * n_side + cx + dx)
    sel.add(n_side * n_side - 1)   # last pixel (ragged tail of the last tile)
    return np.array(sorted(sel))


@pytest.fixture(scope="module")
def c3_case():
    w = configs.c3()
    epochs = [0, 17, 33, 49]
    sel = sample_pixels(w.n_side, w.source_pixels(), 64)
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


def test_c4_batched_full_size(ctx):
    from paper_2310_09200_amd import Batch, StandardSynthesis
    w = configs.c4()
    n_inst = w.n_instances()
    say(f"case C4 full size: {n_inst} instances, {w.meta['n_channels']} slots, {w.n_pix} pixels")
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
    batch = Batch(items, ctx.device)
    say(f"C4 products {batch.products * w.n_pix:.3e}")
    s = StandardSynthesis(ctx, w.pix, 4, 64, 512, 128, "fp32_3m")
    s.collect_eig_batched(batch)
    s.sync()
    t = s.timings()
    got = s.images[:, :, torch.as_tensor(sel, device=ctx.device)].double().cpu().numpy()
    s.close()
    say(f"C4 synthesis kernel {t[2]:.1f} ms -> {batch.products * w.n_pix / (t[2] / 1e3):.3e} products/s")
    worst = 0.0
    for sl in range(64):
        err = level_errors(got[sl], want[sl])
        worst = max(worst, float(np.max(err[:, 0])))
    say(f"C4 worst per-level max err over 64 slots: {worst:.2e}")
    assert worst <= 1e-5
