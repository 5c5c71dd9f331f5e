"""FP64 gradient of a weighted image loss (test infrastructure only).

Loss: ``loss = sum_l sum_p w_lp I_lp`` with ``I_lp = sum_{k in l} d_k |E_kp|^2``,
``E = W^H B``, ``B_lp = exp(+j 2 pi <x_l, p> / lambda_w)``.  The leaves are W
(complex, L x K), d (real, K) and x (real, L x 3); the eigen-decomposition is
not differentiated.  The image is the standard-synthesis image of Sections
2.4 and 2.6; the derivatives below follow from it by the chain rule:

    c_kp  = sum_l member_lk w_lp
    dd_k  = sum_p c_kp |E_kp|^2
    M_kp  = d_k c_kp conj(E_kp)
    dW    = 2 B M^T                       (complex gradient d/dRe + j d/dIm)
    H     = conj(W) M
    dx_l  = -(4 pi / lambda_w) sum_p Im(H_lp B_lp) p
"""

import numpy as np

from .bluebild_ref import phases, synthesize_blas


def loss(W, d, x, member, wts, p, wl):
    """Scalar loss sum_{l,p} wts[l,p] * I[l,p]."""
    return float(np.sum(wts * synthesize_blas(W, d, member, x, p, wl)))


def grad(W, d, x, member, wts, p, wl, chunk=8192):
    """Analytic gradient (dW complex128 (L,K), dd float64 (K,), dx float64 (L,3))."""
    W = np.asarray(W, np.complex128)
    d = np.asarray(d, np.float64)
    x = np.asarray(x, np.float64)
    memf = np.asarray(member, np.float64)
    L, K = W.shape
    dW = np.zeros((L, K), np.complex128)
    dd = np.zeros(K)
    dx = np.zeros((L, 3))
    for s in range(0, p.shape[0], chunk):
        ps = p[s:s + chunk]
        B = phases(x, ps, wl)                   # (L, n)
        E = W.conj().T @ B                      # (K, n)
        c = memf.T @ wts[:, s:s + chunk]        # (K, n)
        dd += np.sum(c * (E.real ** 2 + E.imag ** 2), axis=1)
        M = d[:, None] * c * E.conj()           # (K, n)
        dW += 2.0 * (B @ M.T)
        H = W.conj() @ M                        # (L, n)
        dx += -(4.0 * np.pi / wl) * (np.imag(H * B) @ ps)
    return dW, dd, dx


def fd_grad(W, d, x, member, wts, p, wl, coords, h=1e-6):
    """Central finite differences of :func:`loss` at the listed coordinates.

    ``coords`` is a list of (name, index) with name in {"Wr", "Wi", "d", "x"}
    and index a tuple into that leaf; the step is ``h * max(1, |theta|)``.
    Returns a float64 array, one derivative per coordinate (for "Wr"/"Wi"
    the real and imaginary parts of the torch-convention complex gradient).
    """
    out = []
    for name, idx in coords:
        W1, d1, x1 = W.astype(np.complex128).copy(), d.astype(np.float64).copy(), x.astype(np.float64).copy()
        W2, d2, x2 = W1.copy(), d1.copy(), x1.copy()
        if name == "Wr":
            th = W1[idx].real
            st = h * max(1.0, abs(th))
            W1[idx] += st
            W2[idx] -= st
        elif name == "Wi":
            th = W1[idx].imag
            st = h * max(1.0, abs(th))
            W1[idx] += 1j * st
            W2[idx] -= 1j * st
        elif name == "d":
            st = h * max(1.0, abs(d1[idx]))
            d1[idx] += st
            d2[idx] -= st
        elif name == "x":
            st = h * max(1.0, abs(x1[idx]))
            x1[idx] += st
            x2[idx] -= st
        else:
            raise ValueError(name)
        out.append((loss(W1, d1, x1, member, wts, p, wl) - loss(W2, d2, x2, member, wts, p, wl)) / (2 * st))
    return np.array(out)
