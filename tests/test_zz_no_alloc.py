"""The entry point that allocates nothing (bb_synth_collect_eig_noalloc), through the C ABI.

Its images must equal those of bb_synth_collect_eig on a handle of the same
precision and level count (the same staging and synthesis kernels, staging
in the library's fixed scratch instead of the handle's workspace), and stay
within the oracle tolerance of the FP64 images.  Two calls in a row, the
second with a smaller instance over fewer pixels, so that the second reads a
scratch area the first left behind.
"""

import ctypes
import sys

import numpy as np
import pytest
import torch

import sims
from paper_2310_09200_amd import _lib
from tests._helpers import level_errors, oracle_images

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp32_3m": 1e-5, "bf16x3": 1e-4, "bf16x3_3m": 1e-4}
PREC = {"fp32": 0, "bf16x3": 1, "fp32_3m": 2, "bf16x3_3m": 3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu):
    from paper_2310_09200_amd import Context
    c = Context(0)
    yield c


def _inputs(L, K, n_side, n_levels, seed):
    g = np.random.default_rng(seed)
    x = sims.disk_layout(L, 3000.0, g, z_sigma_m=2.0)
    wl = sims.wavelength_m(150e6)
    pix = sims.pixel_grid(n_side, 6.0, 60.0)
    W = sims.random_eigvecs(L, K, g)
    d = g.normal(0, 1, K)
    lev = g.integers(-1, n_levels, K).astype(np.int32)
    return x, wl, pix, W, d, lev


def _cm(a, dtype, dev):
    return torch.as_tensor(a).to(device=dev, dtype=dtype).transpose(0, 1).contiguous()


def _noalloc(ctx, precision, n_levels, x, wl, pix, W, d, lev):
    dev = ctx.device
    L, K = W.shape
    pix_cm = _cm(pix, torch.float64, dev)
    x_cm = _cm(x, torch.float64, dev)
    W_cm = _cm(W, torch.complex64, dev)
    d_t = torch.as_tensor(d).to(device=dev, dtype=torch.float32)
    lev_t = torch.as_tensor(lev).to(device=dev, dtype=torch.int32)
    images = torch.zeros((n_levels, pix.shape[0]), dtype=torch.float32, device=dev)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    ctx.bind_current_stream()
    _lib.check(ctx.lib.bb_synth_collect_eig_noalloc(ctx.handle, PREC[precision], n_levels, pix.shape[0], p(pix_cm),
                                                    p(images), L, K, float(wl), p(x_cm), p(W_cm), p(d_t), p(lev_t)),
               ctx.handle)
    torch.cuda.synchronize()
    return images.double().cpu().numpy()


def _handle(ctx, precision, n_levels, x, wl, pix, W, d, lev):
    from paper_2310_09200_amd import StandardSynthesis
    L, K = W.shape
    s = StandardSynthesis(ctx, pix, n_levels, 1, L, K, precision)
    s.collect_eig(0, x, wl, W, d, lev)
    s.sync()
    out = s.images[0].double().cpu().numpy()
    s.close()
    return out


@pytest.mark.parametrize("precision", ["fp32_3m", "fp32", "bf16x3", "bf16x3_3m"])
def test_noalloc_equals_collect_eig_twice(ctx, precision):
    n_levels = 3
    for L, K, n_side, seed in [(300, 200, 71, 1), (40, 24, 37, 2)]:   # the second call is smaller
        say(f"case noalloc precision={precision} L={L} K={K} n_pix={n_side * n_side}")
        x, wl, pix, W, d, lev = _inputs(L, K, n_side, n_levels, seed)
        got = _noalloc(ctx, precision, n_levels, x, wl, pix, W, d, lev)
        want = _handle(ctx, precision, n_levels, x, wl, pix, W, d, lev)
        assert np.array_equal(got, want), np.max(np.abs(got - want))
        d32 = d.astype(np.float32).astype(np.float64)
        ref = oracle_images(W.astype(np.complex64).astype(np.complex128), d32, lev, x, wl, pix, n_levels)
        err = level_errors(got, ref)
        say("  max level error vs oracle", err[:, 0].max())
        assert np.all(err[:, 0] <= TOL[precision]), err


def test_noalloc_rejects_instances_beyond_the_scratch(ctx):
    say("case noalloc size limit")
    dev = ctx.device
    L = K = 1024
    pix = torch.zeros((3, 16), dtype=torch.float64, device=dev)
    images = torch.full((2, 16), 7.0, dtype=torch.float32, device=dev)
    x = torch.zeros((3, L), dtype=torch.float64, device=dev)
    W = torch.zeros((K, L), dtype=torch.complex64, device=dev)
    d = torch.zeros(K, dtype=torch.float32, device=dev)
    lev = torch.zeros(K, dtype=torch.int32, device=dev)
    p = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    st = ctx.lib.bb_synth_collect_eig_noalloc(ctx.handle, 2, 2, 16, p(pix), p(images), L, K, 2.0, p(x), p(W), p(d),
                                              p(lev))
    assert st == _lib.BB_ERR_WORKSPACE
    assert b"scratch" in ctx.lib.bb_last_error(ctx.handle)
    torch.cuda.synchronize()
    assert torch.all(images == 7.0)
