"""Host-side marshalling of the Python binding (CPU only; no library calls)."""

import numpy as np
import torch

from paper_2310_09200_amd import _lib
from paper_2310_09200_amd.synthesis import Batch, _colmajor


def test_colmajor_layout():
    a = torch.arange(12, dtype=torch.float64).reshape(4, 3)      # (rows=4, cols=3)
    cm = _colmajor(a, torch.float64, "cpu")
    flat = cm.reshape(-1).numpy()
    # element (r, c) at r + c * rows
    for r in range(4):
        for c in range(3):
            assert flat[r + c * 4] == a[r, c]


def test_batch_packing_offsets_and_layout():
    g = np.random.default_rng(0)
    items = []
    for slot, (L, K) in enumerate([(5, 3), (7, 2), (4, 4)]):
        W = (g.standard_normal((L, K)) + 1j * g.standard_normal((L, K))).astype(np.complex64)
        items.append((slot % 2, g.standard_normal((L, 3)), 1.5 + slot, W, g.standard_normal(K),
                      g.integers(-1, 2, K)))
    b = Batch(items, "cpu")
    assert b.n_ant_rows == 16
    assert [i.ant_off for i in b.inst] == [0, 5, 12]
    assert [i.w_off for i in b.inst] == [0, 15, 29]
    assert [i.eig_off for i in b.inst] == [0, 3, 5]
    # products count antennas x kept eigenpairs (level id >= 0), the work the synthesis does per pixel
    assert b.products == sum(x.shape[0] * int((np.asarray(lev) >= 0).sum()) for _, x, _, _, _, lev in items)
    assert b.products < 5 * 3 + 7 * 2 + 4 * 4       # this draw drops some eigenpairs
    assert b.n_w == 5 * 3 + 7 * 2 + 4 * 4 and b.n_eig_rows == 3 + 2 + 4
    ant = b.ant.numpy()                       # column-major n_rows x 3
    Wp = b.W.numpy()
    for (slot, x, wl, W, d, lev), inst in zip(items, b.inst):
        L, K = W.shape
        for c in range(3):
            assert np.allclose(ant[c, inst.ant_off:inst.ant_off + L], x[:, c])
        blk = Wp[inst.w_off:inst.w_off + L * K]
        assert np.array_equal(blk, W.ravel(order="F"))
        assert inst.slot == slot and inst.wavelength_m == wl


def test_struct_sizes_match_header():
    # bb_options: 8 int32; bb_instance: 4 int32 + double + 3 int64
    import ctypes
    assert ctypes.sizeof(_lib.bb_options) == 32
    assert ctypes.sizeof(_lib.bb_instance) == 48
