"""Why the phase argument is FP64 (CPU emulation at the C3 SKA-Low-like geometry)."""

import numpy as np

import oracle as ref
import sims
from sims import configs
from tests._helpers import level_errors


def test_fp32_phase_argument_fails_at_long_baselines():
    """With 65 km baselines |<x,p>/lambda| reaches ~1e4 turns; an FP32 argument then misses 1e-5."""
    w = configs.c3(n_steps=50, n_side=2048)
    inst = w.instance(0)
    g = np.random.default_rng(3)
    sel = np.unique(np.concatenate([g.choice(w.n_pix, 512, replace=False), w.source_pixels()]))
    p = w.pix[sel]
    lam, A = ref.geneig(inst.V, ref.gram(inst.x, inst.wl))
    lam, W = ref.select_top(lam, A, 512)
    iv = sims.kmeans1d_intervals(lam, 8, negative_level=True)
    member = ref.level_membership(lam, iv)
    exact = ref.synthesize_blas(W, lam, member, inst.x, p, inst.wl)
    t32 = ((inst.x.astype(np.float32) / np.float32(inst.wl)) @ p.astype(np.float32).T).astype(np.float64)
    E = W.conj().T @ np.exp(2j * np.pi * t32)
    img32 = (member * lam[None, :]) @ (np.abs(E) ** 2)
    err = level_errors(img32, exact)
    tmax = np.max(np.abs(inst.x @ p.T / inst.wl))
    print(f"max |t| = {tmax:.0f} turns; FP32-argument per-level max error {np.max(err[:, 0]):.2e}")
    assert tmax > 5e3
    assert np.max(err[:, 0]) > 1e-5
