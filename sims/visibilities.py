"""Visibility simulation: the measurement model of Section 2.1 (the instrument, not the imager).

Convention (the reading adopted for the paper's two opposite phase signs):
the sampling operator is ``Psi*_{l s} = exp(+j 2 pi <x_l, r_s> / lambda_w)``
and ``V = Psi* diag(I) Psi + noise``, i.e.

    V_pq = sum_s I_s exp(+j 2 pi <x_p - x_q, r_s> / lambda_w) + N_pq.

Data in the usual radio convention must be conjugated to match.
"""

import numpy as np


def steering(x, dirs, wl):
    """(L, S) complex128 matrix ``exp(+j 2 pi <x_l, r_s> / wl)`` (direct FP64 evaluation)."""
    arg = (2.0 * np.pi / wl) * (np.asarray(x, np.float64) @ np.asarray(dirs, np.float64).T)
    return np.exp(1j * arg)


def visibility(x, dirs, flux, wl, chunk=4096):
    """Noise-free visibility matrix ``a diag(flux) a^H`` (L, L) complex128, Hermitian PSD."""
    L = x.shape[0]
    V = np.zeros((L, L), np.complex128)
    for s0 in range(0, dirs.shape[0], chunk):
        a = steering(x, dirs[s0:s0 + chunk], wl)
        V += (a * flux[s0:s0 + chunk]) @ a.conj().T
    return 0.5 * (V + V.conj().T)


def hermitian_noise(L, g):
    """Hermitian Gaussian ``(X + X^H)/2`` with ``X_ij ~ CN(0, 1)``: indefinite."""
    X = (g.standard_normal((L, L)) + 1j * g.standard_normal((L, L))) / np.sqrt(2.0)
    return 0.5 * (X + X.conj().T)


def psd_noise(L, g, factor=4):
    """Positive semidefinite noise ``Y Y^H / M`` with ``Y`` (L, M=factor*L) complex normal."""
    M = factor * L
    Y = (g.standard_normal((L, M)) + 1j * g.standard_normal((L, M))) / np.sqrt(2.0)
    N = (Y @ Y.conj().T) / M
    return 0.5 * (N + N.conj().T)


def add_noise_snr(V_sig, N, snr):
    """``V_sig + c N`` with ``c`` chosen so that ||V_sig||_F / ||c N||_F = snr (linear ratio)."""
    if snr is None or snr <= 0:
        return V_sig.copy()
    c = np.linalg.norm(V_sig) / (snr * np.linalg.norm(N))
    V = V_sig + c * N
    return 0.5 * (V + V.conj().T)
