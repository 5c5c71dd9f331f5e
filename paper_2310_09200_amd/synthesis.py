"""Python front end: Context and StandardSynthesis over the C ABI (torch tensors for memory and streams).

Every step of the computation runs in libbluebild.so; this module only turns
tensors into column-major device pointers, allocates the caller-owned
buffers (images, workspaces) with torch, and passes torch's current stream.
"""

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import bb_instance, bb_options, check, load

_PREC = {"fp32": _lib.BB_PREC_FP32, "bf16x3": _lib.BB_PREC_BF16X3, "fp32_3m": _lib.BB_PREC_FP32_3M,
         "bf16x3_3m": _lib.BB_PREC_BF16X3_3M}
_FILT = {"lsq": _lib.BB_FILTER_LSQ, "std": _lib.BB_FILTER_STD}
_GRAM = {"sinc": _lib.BB_GRAM_SINC, "identity": _lib.BB_GRAM_IDENTITY}


def _colmajor(t, dtype, device):
    """(rows, cols) tensor -> contiguous (cols, rows) tensor: its storage is the column-major matrix."""
    return t.to(device=device, dtype=dtype).transpose(0, 1).contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """Device + stream + eigensolver handle (the paper's Context, Section 3.1)."""

    def __init__(self, device=0):
        if not torch.cuda.is_available():
            raise RuntimeError("Bluebild needs a HIP device; none is visible")
        self.lib = load()
        self.device = torch.device("cuda", device)
        h = ctypes.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        check(self.lib.bb_context_create(device, ctypes.c_void_p(stream), ctypes.byref(h)))
        self.handle = h

    def bind_current_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(self.lib.bb_context_set_stream(self.handle, ctypes.c_void_p(s)), self.handle)

    def close(self):
        if self.handle:
            check(self.lib.bb_context_destroy(self.handle), self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tile_shapes(precision):
    """Tile shapes of a contraction mode: [(id, eigenpairs per pass, pixels per tile, waves, K classes)]."""
    lib = load()
    out = []
    for t in range(_lib.BB_MAX_TILES):
        kc, nt, wv, mask = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        if lib.bb_tile_info(_PREC[precision], t, ctypes.byref(kc), ctypes.byref(nt), ctypes.byref(wv),
                            ctypes.byref(mask)) != _lib.BB_OK:
            break
        out.append((t, kc.value, nt.value, wv.value, [c for c in range(_lib.BB_K_CLASSES) if mask.value >> c & 1]))
    return out


def phase_probe(ctx, ant_xyz, wavelength_m, pix, reps=1, out=None):
    """Phase-generation throughput probe (measurement only; ``bb_phase_probe``).

    ``ant_xyz`` (n_ant, 3) metres and ``pix`` (n_pix, 3) unit vectors; returns
    ``out`` (n_pix,) float32 with reps * sum over antennas of (cos + sin) of the
    phase 2 pi <x, p> / wavelength.  Enqueued on torch's current stream (time
    it with events there).
    """
    dev = ctx.device
    x = _colmajor(torch.as_tensor(ant_xyz), torch.float64, dev)
    p = _colmajor(torch.as_tensor(pix), torch.float64, dev)
    n_ant, n_pix = x.shape[1], p.shape[1]
    if out is None:
        out = torch.empty(n_pix, dtype=torch.float32, device=dev)
    ctx.bind_current_stream()
    check(ctx.lib.bb_phase_probe(ctx.handle, n_ant, float(wavelength_m), _ptr(x), n_pix, _ptr(p), int(reps),
                                 _ptr(out)), ctx.handle)
    return out


class StandardSynthesis:
    """Imaging handle: accumulates per-level images over collected instances.

    ``pix`` is (n_pix, 3) float64 unit vectors.  Images are a float32 tensor
    ``[n_slots, n_levels, n_pix]`` owned by this object (``.images``).
    """

    def __init__(self, ctx, pix, n_levels, n_slots=1, n_ant_max=512, k_max=512, precision="fp32", filter="lsq",
                 images=None, gram="sinc"):
        self.ctx = ctx
        self.lib = ctx.lib
        dev = ctx.device
        self.n_pix = int(pix.shape[0])
        self.n_levels = int(n_levels)
        self.n_slots = int(n_slots)
        self.opt = bb_options(n_levels=n_levels, n_slots=n_slots, n_ant_max=n_ant_max, k_max=k_max,
                              precision=_PREC[precision], filter=_FILT[filter], gram=_GRAM[gram])
        self.pix_cm = _colmajor(torch.as_tensor(pix), torch.float64, dev)
        if images is None:
            images = torch.zeros((n_slots, n_levels, self.n_pix), dtype=torch.float32, device=dev)
        assert images.shape == (n_slots, n_levels, self.n_pix) and images.dtype == torch.float32
        assert images.is_contiguous()
        self.images = images
        sz = ctypes.c_size_t()
        check(self.lib.bb_workspace_size(ctx.handle, ctypes.byref(self.opt), self.n_pix, ctypes.byref(sz)),
              ctx.handle)
        self.workspace = torch.empty(int(sz.value) + 256, dtype=torch.uint8, device=dev)
        ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        h = ctypes.c_void_p()
        ctx.bind_current_stream()
        check(self.lib.bb_synth_create(ctx.handle, ctypes.byref(self.opt), self.n_pix, _ptr(self.pix_cm),
                                       _ptr(self.images), ctypes.c_void_p(ws_ptr), sz.value, ctypes.byref(h)),
              ctx.handle)
        self.handle = h
        self._keep = []

    # -- calls ---------------------------------------------------------------
    def collect(self, slot, x, wavelength, V, n_eig, intervals):
        """Full step (Algorithm 1): x (L,3) f64, V (L,L) complex128 Hermitian, intervals (n_levels,2)."""
        dev = self.ctx.device
        L = int(x.shape[0])
        xc = _colmajor(torch.as_tensor(x), torch.float64, dev)
        Vc = _colmajor(torch.as_tensor(V), torch.complex128, dev)
        iv = np.ascontiguousarray(np.asarray(intervals, np.float64).reshape(self.n_levels, 2).T).ravel()
        ivp = iv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_collect(self.handle, slot, L, float(wavelength), _ptr(xc), _ptr(Vc), int(n_eig),
                                        ivp), self.ctx.handle)
        self._keep = [xc, Vc]

    def collect_beamformed(self, slot, x, wavelength, W_bf, V_bf, n_eig, intervals):
        """Full step with beamforming: W_bf (L, Kb) complex, V_bf (Kb, Kb) beamformed visibilities."""
        dev = self.ctx.device
        L, Kb = int(W_bf.shape[0]), int(W_bf.shape[1])
        xc = _colmajor(torch.as_tensor(x), torch.float64, dev)
        Wc = _colmajor(torch.as_tensor(W_bf), torch.complex128, dev)
        Vc = _colmajor(torch.as_tensor(V_bf), torch.complex128, dev)
        iv = np.ascontiguousarray(np.asarray(intervals, np.float64).reshape(self.n_levels, 2).T).ravel()
        ivp = iv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_collect_beamformed(self.handle, slot, L, Kb, float(wavelength), _ptr(xc), _ptr(Wc),
                                                   _ptr(Vc), int(n_eig), ivp), self.ctx.handle)
        self._keep = [xc, Wc, Vc]

    def collect_energy(self, slot, x, wavelength, V, energy_fraction, intervals):
        """Full step keeping the fewest eigenpairs that reach ``energy_fraction`` of the energy; returns K."""
        dev = self.ctx.device
        L = int(x.shape[0])
        xc = _colmajor(torch.as_tensor(x), torch.float64, dev)
        Vc = _colmajor(torch.as_tensor(V), torch.complex128, dev)
        iv = np.ascontiguousarray(np.asarray(intervals, np.float64).reshape(self.n_levels, 2).T).ravel()
        ivp = iv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        k = ctypes.c_int32()
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_collect_energy(self.handle, slot, L, float(wavelength), _ptr(xc), _ptr(Vc),
                                               float(energy_fraction), ivp, ctypes.byref(k)), self.ctx.handle)
        self._keep = [xc, Vc]
        return k.value

    def prestep(self, x, wavelength, V, n_eig, intervals):
        """FP64 pre-step alone: returns (W (L,K) complex64, lam (K,) f64, d (K,) f32, level_of (K,) i32) on device."""
        dev = self.ctx.device
        L = int(x.shape[0])
        K = int(n_eig)
        xc = _colmajor(torch.as_tensor(x), torch.float64, dev)
        Vc = _colmajor(torch.as_tensor(V), torch.complex128, dev)
        iv = np.ascontiguousarray(np.asarray(intervals, np.float64).reshape(self.n_levels, 2).T).ravel()
        ivp = iv.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        Wt = torch.empty((K, L), dtype=torch.complex64, device=dev)   # column-major (L, K)
        lam = torch.empty(K, dtype=torch.float64, device=dev)
        d = torch.empty(K, dtype=torch.float32, device=dev)
        lev = torch.empty(K, dtype=torch.int32, device=dev)
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_prestep(self.handle, L, float(wavelength), _ptr(xc), _ptr(Vc), K, ivp, _ptr(Wt),
                                        _ptr(lam), _ptr(d), _ptr(lev)), self.ctx.handle)
        self._keep = [xc, Vc]
        return Wt.transpose(0, 1), lam, d, lev

    def prestep_batched(self, xs, wavelengths, Vs, n_eig, intervals):
        """FP64 pre-step of many instances with one antenna count (one batched eigensolve, one wait).

        ``xs`` (n_inst, L, 3) f64, ``wavelengths`` (n_inst,), ``Vs`` (n_inst, L, L) complex128.
        Returns device tensors (W (n_inst, L, K) complex64, lam (n_inst, K) f64, d (n_inst, K) f32,
        level_of (n_inst, K) i32); their storage is the packed layout ``collect_eig_batched`` takes
        (instance i's W column-major at element i L K).
        """
        dev = self.ctx.device
        xs = torch.as_tensor(xs)
        n_inst, L = int(xs.shape[0]), int(xs.shape[1])
        K = int(n_eig)
        x_cm = xs.to(device=dev, dtype=torch.float64).reshape(n_inst * L, 3).transpose(0, 1).contiguous()
        V_cm = torch.as_tensor(Vs).to(device=dev, dtype=torch.complex128).transpose(1, 2).contiguous()
        wl = np.ascontiguousarray(np.asarray(wavelengths, np.float64).reshape(n_inst))
        iv = np.ascontiguousarray(np.asarray(intervals, np.float64).reshape(self.n_levels, 2).T).ravel()
        dp = ctypes.POINTER(ctypes.c_double)
        Wt = torch.empty((n_inst, K, L), dtype=torch.complex64, device=dev)   # instance i: column-major (L, K)
        lam = torch.empty((n_inst, K), dtype=torch.float64, device=dev)
        d = torch.empty((n_inst, K), dtype=torch.float32, device=dev)
        lev = torch.empty((n_inst, K), dtype=torch.int32, device=dev)
        sz = ctypes.c_size_t()
        check(self.lib.bb_prestep_batched_workspace_size(self.handle, n_inst, L, K, ctypes.byref(sz)),
              self.ctx.handle)
        ws = torch.empty(int(sz.value) + 256, dtype=torch.uint8, device=dev)
        ws_ptr = (ws.data_ptr() + 255) // 256 * 256
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_prestep_batched(self.handle, n_inst, L, K, wl.ctypes.data_as(dp), _ptr(x_cm),
                                                _ptr(V_cm), iv.ctypes.data_as(dp), _ptr(Wt), _ptr(lam), _ptr(d),
                                                _ptr(lev), ctypes.c_void_p(ws_ptr), sz.value), self.ctx.handle)
        self._keep = [x_cm, V_cm, ws]
        return Wt.transpose(1, 2), lam, d, lev

    def levels_kmeans(self, lam, negative_level=True):
        """Level intervals by exact k-means of the eigenvalues ``lam`` (n,), on the device.

        n_levels - negative_level positive levels (level 0 the largest), plus one
        level for the non-positive eigenvalues when ``negative_level``.  Returns
        (intervals (n_levels, 2) float64, level_of (n,) int32), both on the device;
        too few positive eigenvalues raises at the next ``sync``.
        """
        dev = self.ctx.device
        lam_d = torch.as_tensor(lam).to(device=dev, dtype=torch.float64).contiguous().reshape(-1)
        n = int(lam_d.numel())
        iv = torch.empty((2, self.n_levels), dtype=torch.float64, device=dev)   # column-major (n_levels, 2)
        lev = torch.empty(n, dtype=torch.int32, device=dev)
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_levels_kmeans(self.handle, n, _ptr(lam_d), int(bool(negative_level)), _ptr(iv),
                                              _ptr(lev)), self.ctx.handle)
        self._keep = [lam_d]
        return iv.transpose(0, 1), lev

    def uniform_weighting(self, x, wavelength, V, e_u, e_v, fov_rad):
        """Uniformly weighted copy of V (L, L) on the device (complex128); V itself is not written."""
        dev = self.ctx.device
        L = int(x.shape[0])
        xc = _colmajor(torch.as_tensor(x), torch.float64, dev)
        Vc = _colmajor(torch.as_tensor(V), torch.complex128, dev).clone()   # the library overwrites this copy
        eu = np.ascontiguousarray(np.asarray(e_u, np.float64).reshape(3))
        ev = np.ascontiguousarray(np.asarray(e_v, np.float64).reshape(3))
        dp = ctypes.POINTER(ctypes.c_double)
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_uniform_weighting(self.handle, L, float(wavelength), _ptr(xc), eu.ctypes.data_as(dp),
                                                  ev.ctypes.data_as(dp), float(fov_rad), _ptr(Vc)), self.ctx.handle)
        self._keep = [xc]
        return Vc.transpose(0, 1)

    def collect_eig(self, slot, x, wavelength, W, d, level_of):
        """Hot path: x (L,3) f64, W (L,K) complex, d (K,) weights, level_of (K,) int (-1 = unused)."""
        dev = self.ctx.device
        L, K = int(W.shape[0]), int(W.shape[1])
        xc = _colmajor(torch.as_tensor(x), torch.float64, dev)
        Wc = _colmajor(torch.as_tensor(W), torch.complex64, dev)
        dc = torch.as_tensor(d).to(device=dev, dtype=torch.float32).contiguous()
        lc = torch.as_tensor(level_of).to(device=dev, dtype=torch.int32).contiguous()
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_collect_eig(self.handle, slot, L, K, float(wavelength), _ptr(xc), _ptr(Wc),
                                            _ptr(dc), _ptr(lc)), self.ctx.handle)
        self._keep = [xc, Wc, dc, lc]

    def collect_eig_batched(self, batch):
        """Many instances in one launch; ``batch`` is a :class:`Batch` (packed device arrays)."""
        arr = (bb_instance * len(batch.inst))(*batch.inst)
        sz = ctypes.c_size_t()
        check(self.lib.bb_batched_workspace_size(self.handle, len(batch.inst), arr, ctypes.byref(sz)),
              self.ctx.handle)
        ws = torch.empty(int(sz.value) + 256, dtype=torch.uint8, device=self.ctx.device)
        ws_ptr = (ws.data_ptr() + 255) // 256 * 256
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_collect_eig_batched(
            self.handle, len(batch.inst), arr, batch.n_ant_rows, batch.n_w, batch.n_eig_rows, _ptr(batch.ant),
            _ptr(batch.W), _ptr(batch.d), _ptr(batch.lev), ctypes.c_void_p(ws_ptr), sz.value), self.ctx.handle)
        self._keep = [ws]

    @property
    def tiles(self):
        """Tile id per K class (K rounded up to 32: <= 32, <= 64, <= 128, more) used by the synthesis launches."""
        t = (ctypes.c_int32 * _lib.BB_K_CLASSES)()
        check(self.lib.bb_synth_get_tiles(self.handle, t), self.ctx.handle)
        return list(t)

    @tiles.setter
    def tiles(self, ids):
        t = (ctypes.c_int32 * _lib.BB_K_CLASSES)(*[int(i) for i in ids])
        check(self.lib.bb_synth_set_tiles(self.handle, t), self.ctx.handle)

    def autotune_batched(self, batch, reps=2, return_scratch=False):
        """Time every tile each K class of ``batch`` may use and keep the fastest (images untouched).

        Returns {k_class: {tile_id: ms per launch}} (and, with ``return_scratch``, the scratch
        images every timed launch accumulated into).
        """
        arr = (bb_instance * len(batch.inst))(*batch.inst)
        sz = ctypes.c_size_t()
        check(self.lib.bb_batched_workspace_size(self.handle, len(batch.inst), arr, ctypes.byref(sz)),
              self.ctx.handle)
        ws = torch.empty(int(sz.value) + 256, dtype=torch.uint8, device=self.ctx.device)
        ws_ptr = (ws.data_ptr() + 255) // 256 * 256
        scratch = torch.empty_like(self.images)
        ms = (ctypes.c_double * (_lib.BB_K_CLASSES * _lib.BB_MAX_TILES))()
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_autotune_batched(
            self.handle, len(batch.inst), arr, batch.n_ant_rows, batch.n_w, batch.n_eig_rows, _ptr(batch.ant),
            _ptr(batch.W), _ptr(batch.d), _ptr(batch.lev), ctypes.c_void_p(ws_ptr), sz.value, _ptr(scratch),
            int(reps), ms), self.ctx.handle)
        out = {}
        for c in range(_lib.BB_K_CLASSES):
            row = {t: ms[c * _lib.BB_MAX_TILES + t] for t in range(_lib.BB_MAX_TILES)
                   if ms[c * _lib.BB_MAX_TILES + t] >= 0}
            if row:
                out[c] = row
        return (out, scratch) if return_scratch else out

    def eig_backward(self, x, wavelength, W, d, level_of, grad_images):
        """Gradient of sum(grad_images * I) for one instance's images I (before accumulation).

        Returns (dW (L,K) complex64 = dLoss/dRe W + j dLoss/dIm W, dd (K,) float32, dx (L,3) float64).
        """
        dev = self.ctx.device
        L, K = int(W.shape[0]), int(W.shape[1])
        xc = _colmajor(torch.as_tensor(x), torch.float64, dev)
        Wc = _colmajor(torch.as_tensor(W), torch.complex64, dev)
        dc = torch.as_tensor(d).to(device=dev, dtype=torch.float32).contiguous()
        lc = torch.as_tensor(level_of).to(device=dev, dtype=torch.int32).contiguous()
        g = torch.as_tensor(grad_images).to(device=dev, dtype=torch.float32).reshape(self.n_levels,
                                                                                     self.n_pix).contiguous()
        dWt = torch.empty((K, L), dtype=torch.complex64, device=dev)
        dd = torch.empty(K, dtype=torch.float32, device=dev)
        dxt = torch.empty((3, L), dtype=torch.float64, device=dev)
        sz = ctypes.c_size_t()
        check(self.lib.bb_backward_workspace_size(self.handle, L, K, ctypes.byref(sz)), self.ctx.handle)
        ws = torch.empty(int(sz.value) + 256, dtype=torch.uint8, device=dev)
        ws_ptr = (ws.data_ptr() + 255) // 256 * 256
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_eig_backward(self.handle, L, K, float(wavelength), _ptr(xc), _ptr(Wc), _ptr(dc),
                                             _ptr(lc), _ptr(g), _ptr(dWt), _ptr(dd), _ptr(dxt),
                                             ctypes.c_void_p(ws_ptr), sz.value), self.ctx.handle)
        self._keep = [xc, Wc, dc, lc, g, ws]
        return dWt.transpose(0, 1), dd, dxt.transpose(0, 1)

    def sync(self):
        check(self.lib.bb_synth_sync(self.handle), self.ctx.handle)

    def reset(self):
        self.ctx.bind_current_stream()
        check(self.lib.bb_synth_reset(self.handle), self.ctx.handle)

    @property
    def count(self):
        c = ctypes.c_int64()
        check(self.lib.bb_synth_get_count(self.handle, ctypes.byref(c)), self.ctx.handle)
        return c.value

    @count.setter
    def count(self, v):
        check(self.lib.bb_synth_set_count(self.handle, int(v)), self.ctx.handle)

    def timings(self):
        """(pre-step, staging, synthesis) device milliseconds of the last call."""
        out = (ctypes.c_double * 3)()
        check(self.lib.bb_synth_timings(self.handle, out, 3), self.ctx.handle)
        return tuple(out)

    def close(self):
        if getattr(self, "handle", None):
            check(self.lib.bb_synth_destroy(self.handle), self.ctx.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class NufftSynthesis:
    """NUFFT synthesis plan (Section 2.5; Section 3.4, Algorithm 3) over the C ABI.

    ``pix`` (n_pix, 3) float64 unit vectors; ``frame`` rows e_u, e_v, p0 (orthonormal,
    same frame as the antenna positions); ``uvw_max`` (3,) bound on |baseline| / wavelength
    along the frame rows over every instance to be collected; ``eps`` the requested accuracy.
    Instances go in with :meth:`collect_eig_batched` (a :class:`Batch` with slot 0
    everywhere); :meth:`emit` transforms what was collected into ``images`` (n_levels, n_pix).
    ``transform``: ``"auto"`` (the library's own line FFTs where every axis fits, else
    rocFFT) or ``"rocfft"``.  ``partitions``: image-domain tiles per axis;
    ``uvw_partitions``: uvw-domain cells per axis (one NUFFT per (tile, cell) pair,
    one after another on one shared grid; each collect then transforms right away).
    """

    def __init__(self, ctx, pix, n_levels, n_ant_max, k_max, eps, frame, uvw_max, transform="auto", partitions=1,
                 uvw_partitions=1):
        self.ctx = ctx
        self.lib = ctx.lib
        dev = ctx.device
        pix_np = np.ascontiguousarray(np.asarray(pix, np.float64).T)        # host, column-major (n_pix, 3)
        self.n_pix = int(pix_np.shape[1])
        self.n_levels = int(n_levels)
        self.pix_cm = torch.as_tensor(pix_np).to(dev)
        self.opt = _lib.bb_nufft_options(n_levels=int(n_levels), n_ant_max=int(n_ant_max), k_max=int(k_max),
                                         transform={"auto": 0, "rocfft": 1}[transform], epsilon=float(eps),
                                         partitions=int(partitions), uvw_partitions=int(uvw_partitions))
        fr = np.asarray(frame, np.float64).reshape(9)
        um = np.asarray(uvw_max, np.float64).reshape(3)
        for i in range(9):
            self.opt.frame[i] = float(fr[i])
        for i in range(3):
            self.opt.uvw_max[i] = float(um[i])
        hp = ctypes.c_void_p(pix_np.ctypes.data)
        sz = ctypes.c_size_t()
        check(self.lib.bb_nufft_workspace_size(ctx.handle, ctypes.byref(self.opt), self.n_pix, hp, ctypes.byref(sz)),
              ctx.handle)
        self.workspace = torch.empty(sz.value + 256, dtype=torch.uint8, device=dev)
        ws_ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.images = torch.zeros((self.n_levels, self.n_pix), dtype=torch.float32, device=dev)
        h = ctypes.c_void_p()
        ctx.bind_current_stream()
        check(self.lib.bb_nufft_create(ctx.handle, ctypes.byref(self.opt), self.n_pix, hp, _ptr(self.pix_cm),
                                       _ptr(self.images), ctypes.c_void_p(ws_ptr), sz.value, ctypes.byref(h)),
              ctx.handle)
        self.handle = h
        self._keep = []

    @property
    def shape(self):
        """(spread grid N (3,), FFT grid M (3,), kernel width w)."""
        n = (ctypes.c_int32 * 3)()
        m = (ctypes.c_int32 * 3)()
        w = ctypes.c_int32()
        check(self.lib.bb_nufft_shape(self.handle, n, m, ctypes.byref(w)), self.ctx.handle)
        return tuple(n), tuple(m), w.value

    def collect_eig_batched(self, batch):
        arr = (_lib.bb_instance * len(batch.inst))(*batch.inst)
        sz = ctypes.c_size_t()
        check(self.lib.bb_nufft_batched_workspace_size(self.handle, len(batch.inst), arr, ctypes.byref(sz)),
              self.ctx.handle)
        ws = torch.empty(sz.value + 256, dtype=torch.uint8, device=self.ctx.device)
        ws_ptr = (ws.data_ptr() + 255) // 256 * 256
        self.ctx.bind_current_stream()
        check(self.lib.bb_nufft_collect_eig_batched(
            self.handle, len(batch.inst), arr, batch.n_ant_rows, batch.n_w, batch.n_eig_rows, _ptr(batch.ant),
            _ptr(batch.W), _ptr(batch.d), _ptr(batch.lev), ctypes.c_void_p(ws_ptr), sz.value), self.ctx.handle)
        self._keep = [batch, ws]

    def emit(self):
        self.ctx.bind_current_stream()
        check(self.lib.bb_nufft_emit(self.handle), self.ctx.handle)

    def sync(self):
        check(self.lib.bb_nufft_sync(self.handle), self.ctx.handle)

    def timings(self):
        """(spread, emit) device milliseconds of the last calls."""
        out = (ctypes.c_double * 2)()
        check(self.lib.bb_nufft_timings(self.handle, out, 2), self.ctx.handle)
        return tuple(out)

    def close(self):
        if getattr(self, "handle", None):
            check(self.lib.bb_nufft_destroy(self.handle), self.ctx.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Packed device arrays + instance table for :meth:`StandardSynthesis.collect_eig_batched`.

    ``items`` is a list of (slot, x (L,3), wavelength, W (L,K), d (K,), level_of (K,)); arrays may be
    numpy arrays or tensors on any device.  ``products`` counts antennas x kept eigenpairs (level id
    >= 0) over the instances: the complex products per pixel that the synthesis performs.
    """

    def __init__(self, items, device):
        xs, Ws, ds, ls, inst = [], [], [], [], []
        ant_off = w_off = eig_off = 0
        for slot, x, wl, W, d, lev in items:
            x = torch.as_tensor(x).to(device=device, dtype=torch.float64)
            W = torch.as_tensor(W).to(device=device, dtype=torch.complex64)
            L, K = int(W.shape[0]), int(W.shape[1])
            inst.append(bb_instance(n_ant=L, n_eig=K, slot=int(slot), wavelength_m=float(wl), ant_off=ant_off,
                                    w_off=w_off, eig_off=eig_off))
            xs.append(x)
            Ws.append(W.transpose(0, 1).contiguous().reshape(-1))      # column-major L x K
            ds.append(torch.as_tensor(d).to(device=device, dtype=torch.float32).reshape(-1))
            ls.append(torch.as_tensor(lev).to(device=device, dtype=torch.int32).reshape(-1))
            ant_off += L
            w_off += L * K
            eig_off += K
        X = torch.cat(xs, dim=0)
        self.n_ant_rows = int(X.shape[0])
        self.ant = X.transpose(0, 1).contiguous()                      # column-major n_rows x 3
        self.W = torch.cat(Ws)
        self.d = torch.cat(ds)
        self.lev = torch.cat(ls)
        self.inst = inst
        self.n_w = int(self.W.numel())
        self.n_eig_rows = int(self.d.numel())
        # pixel-independent work: antennas x kept eigenpairs (level id >= 0) summed over instances
        kept = (self.lev.cpu().numpy() >= 0).astype(np.int64)
        csum = np.concatenate([[0], np.cumsum(kept)])
        self.products = sum(int(i.n_ant) * int(csum[i.eig_off + i.n_eig] - csum[i.eig_off]) for i in inst)
