"""torch.autograd.Function over the library's forward and backward kernels.

``bluebild_image(W, d, x, pix, level_of, wavelength, n_levels)`` returns the
(n_levels, n_pix) float32 level images of one instance; its backward gives
the gradients with respect to W (complex, torch's d/dRe + j d/dIm), the filter
weights d and the antenna positions x.  Level ids and pixels are not
differentiated.
"""

from collections import OrderedDict

import torch

from .synthesis import Context, StandardSynthesis

_CTX = {}
# Handles keep their own column-major copy of the pixels, so a cache entry
# holds the pixel tensor it was made from (its storage cannot be reused while
# the entry lives) and is keyed on that tensor's identity and version counter
# (an in-place edit bumps the version and misses the entry).  At most
# _MAX_HANDLES handles are kept; the least recently used one is dropped (and
# freed once no saved autograd context refers to it any more).
_SYNTH = OrderedDict()
_MAX_HANDLES = 4


def _handle(pix, n_levels, n_ant, n_eig, precision):
    dev = pix.device if pix.is_cuda else torch.device("cuda", torch.cuda.current_device())
    ctx = _CTX.get(dev.index)
    if ctx is None:
        ctx = _CTX[dev.index] = Context(dev.index or 0)
    key = (dev.index, id(pix), pix._version, int(pix.shape[0]), n_levels, precision)
    ent = _SYNTH.get(key)
    if ent is not None and ent[0] is pix and ent[1].opt.n_ant_max >= n_ant and ent[1].opt.k_max >= n_eig:
        _SYNTH.move_to_end(key)
        return ent[1]
    if ent is not None:
        del _SYNTH[key]
    s = StandardSynthesis(ctx, pix, n_levels, 1, max(n_ant, 32), max(n_eig, 32), precision)
    _SYNTH[key] = (pix, s)
    while len(_SYNTH) > _MAX_HANDLES:
        _SYNTH.popitem(last=False)
    return s


class _BluebildImage(torch.autograd.Function):
    @staticmethod
    def forward(fctx, W, d, x, pix, level_of, wavelength, n_levels, precision):
        s = _handle(pix, n_levels, int(W.shape[0]), int(W.shape[1]), precision)
        s.reset()
        s.collect_eig(0, x.detach(), wavelength, W.detach(), d.detach(), level_of)
        img = s.images[0].clone()
        fctx.save_for_backward(W, d, x)
        fctx.s = s
        fctx.level_of = level_of
        fctx.wavelength = wavelength
        return img

    @staticmethod
    def backward(fctx, grad):
        W, d, x = fctx.saved_tensors
        dW, dd, dx = fctx.s.eig_backward(x.detach(), fctx.wavelength, W.detach(), d.detach(), fctx.level_of,
                                         grad.contiguous())
        gW = dW.to(W.dtype) if fctx.needs_input_grad[0] else None
        gd = dd.to(d.dtype) if fctx.needs_input_grad[1] else None
        gx = dx.to(x.dtype) if fctx.needs_input_grad[2] else None
        return gW, gd, gx, None, None, None, None, None


def bluebild_image(W, d, x, pix, level_of, wavelength, n_levels, precision="fp32"):
    """Differentiable level images (n_levels, n_pix) of one instance (Sections 2.4 and 2.6)."""
    return _BluebildImage.apply(W, d, x, pix, level_of, float(wavelength), int(n_levels), precision)
