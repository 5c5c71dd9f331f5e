"""Plain FP64 definition of Bluebild standard synthesis (test infrastructure only).

Notation (paper -> here): antennas N_A -> L, kept eigenpairs N_eig -> K,
pixels N_sky -> N_pix, eigenvectors alpha_a -> columns of W, the sampling
operator Psi* (Section 2.1, with g = 1) -> the phase matrix B (L x N_pix),
eps_a = Psi alpha_a -> the rows of E = W^H B up to conjugation (|E_kp| = |eps_k(p)|).

Everything is float64 / complex128, evaluated directly from the paper's
equations with numpy/scipy primitives and no blocking beyond pixel chunking.
"""

import numpy as np
import scipy.linalg as sla

C_LIGHT = 299_792_458.0

__all__ = [
    "C_LIGHT", "wavelength", "gram", "check_hermitian", "geneig", "select_top", "n_eig_for_energy",
    "level_membership", "membership_from_level_of", "lsq_filter", "std_filter", "phases",
    "synthesize_blas", "synthesize_loops", "collect", "collect_beamformed", "lsq_image",
    "backprojection_image", "point_source_image",
]


def wavelength(freq_hz):
    """lambda_w = c / f in metres (Section 2.2 defines baselines in units of f/c)."""
    return C_LIGHT / float(freq_hz)


def gram(x, wl):
    """Gram matrix of the instrument, closed form for g = 1 (Section 2.2, Eq. gram).

    G_pq = sinc(2 ||b_pq||), b_pq = (x_p - x_q) / lambda_w, with the normalised
    sinc(u) = sin(pi u) / (pi u), sinc(0) = 1 (the paper's appendix states this sinc).
    """
    x = np.asarray(x, np.float64)
    d = x[:, None, :] - x[None, :, :]
    dist = np.sqrt(np.sum(d * d, axis=-1))
    return np.sinc(2.0 * dist / wl)


def check_hermitian(V, rtol=1e-12):
    """Return (V + V^H)/2 after checking ||V - V^H||_F <= rtol ||V||_F.

    V is a correlation matrix E[v v^*] (Section 2.1), hence Hermitian.
    """
    V = np.asarray(V, np.complex128)
    if np.linalg.norm(V - V.conj().T) > rtol * max(np.linalg.norm(V), 1e-300):
        raise ValueError("visibility matrix is not Hermitian")
    return 0.5 * (V + V.conj().T)


def geneig(V, G):
    """Generalized eigenpairs of V alpha = lambda G alpha (Section 2.3, Eq. eigenvaleq).

    Reduction to a standard Hermitian problem with the Cholesky factor of G:
    G = C C^H, M = C^{-1} V C^{-H}, M Y = Y diag(mu), alpha = C^{-H} Y.  The
    eigenvectors come out G-orthonormal (alpha^H G alpha = I).  Returns
    (lam ascending float64 (L,), alpha complex128 (L, L)).  Raises
    numpy.linalg.LinAlgError if G is not positive definite.
    """
    V = check_hermitian(V)
    G = np.asarray(G, np.complex128)
    C = np.linalg.cholesky(G)  # lower
    X = sla.solve_triangular(C, V, lower=True)            # C^{-1} V
    M = sla.solve_triangular(C, X.conj().T, lower=True)   # C^{-1} (C^{-1} V)^H = C^{-1} V C^{-H}
    M = 0.5 * (M + M.conj().T)
    mu, Y = np.linalg.eigh(M)
    alpha = sla.solve_triangular(C.conj().T, Y, lower=False)
    return mu, alpha


def select_top(lam, alpha, n_eig):
    """Keep the n_eig largest eigenvalues by signed value, descending; ties stable by index.

    Truncation to the leading eigenpairs (Section 2.6; Algorithm 1, selection step).
    """
    lam = np.asarray(lam, np.float64)
    order = np.argsort(-lam, kind="stable")[:n_eig]
    return lam[order], alpha[:, order]


def n_eig_for_energy(lam, fraction):
    """Fewest leading eigenpairs whose eigenvalues reach ``fraction`` of the total energy (Section 2.6).

    Reading: the energy is the sum of the positive eigenvalues; leading means
    largest by signed value.  Returns K >= 1 (all positive eigenpairs at most,
    or 1 when there is no positive eigenvalue).
    """
    lam = np.sort(np.asarray(lam, np.float64))[::-1]
    total = float(np.sum(lam[lam > 0]))
    if total <= 0:
        return 1
    acc = 0.0
    for k, v in enumerate(lam):
        acc += v
        if acc >= fraction * total:
            return k + 1
    return int(np.sum(lam > 0))


def level_membership(lam, intervals):
    """(N_L, K) boolean: eigenpair k belongs to level l iff lo_l <= lam_k <= hi_l.

    Each interval is tested on its own, as in the interval loop of Algorithm 1
    (closed [min, max] intervals, Table 1); an eigenpair in no interval adds nothing.
    """
    lam = np.asarray(lam, np.float64)
    iv = np.asarray(intervals, np.float64).reshape(-1, 2)
    return (lam[None, :] >= iv[:, 0:1]) & (lam[None, :] <= iv[:, 1:2])


def membership_from_level_of(level_of, n_levels):
    """(N_L, K) boolean from one level id per eigenpair (-1 = in no level).

    The same membership as :func:`level_membership` when the ids come from
    intervals that share at most their endpoints (Algorithm 1's interval loop
    with each eigenpair in at most one level): eigenpair k is in level l iff
    level_of[k] == l.  An id outside [0, n_levels) puts the eigenpair in no level.
    """
    level_of = np.asarray(level_of)
    return level_of[None, :] == np.arange(n_levels)[:, None]


def lsq_filter(lam):
    """Least-squares filter: weights d_k = lambda_k (Section 2.6; Eq. eigenvaluedeco1)."""
    return np.asarray(lam, np.float64).copy()


def std_filter(lam):
    """Standardized filter: uniform sum over eigen-images, d_k = 1 (Section 2.6)."""
    return np.ones_like(np.asarray(lam, np.float64))


def phases(x, p, wl):
    """Phase matrix B_lp = exp(+j 2 pi <x_l, p> / lambda_w), (L, N_pix) complex128.

    This is the sampling operator Psi* of Section 2.1 with g = 1.
    """
    t = (np.asarray(x, np.float64) @ np.asarray(p, np.float64).T) / wl
    return np.exp(2j * np.pi * t)


def synthesize_blas(W, d, member, x, p, wl, chunk=8192):
    """Level images I_l(p) = sum_{k in l} d_k |E_kp|^2 with E = W^H B  (N_L, N_pix) float64.

    Standard synthesis (Section 2.4, Eq. standard_synthesis) followed by the
    level partition (Section 2.6, the level equation) and the filter weights
    of Algorithm 1.  ``member`` is the (N_L, K) membership matrix.
    """
    W = np.asarray(W, np.complex128)
    d = np.asarray(d, np.float64)
    member = np.asarray(member, bool)
    p = np.asarray(p, np.float64)
    out = np.zeros((member.shape[0], p.shape[0]))
    Dw = member.astype(np.float64) * d[None, :]          # (N_L, K)
    for s in range(0, p.shape[0], chunk):
        B = phases(x, p[s:s + chunk], wl)                 # (L, n)
        E = W.conj().T @ B                                # (K, n)
        out[:, s:s + chunk] = Dw @ (E.real ** 2 + E.imag ** 2)
    return out


def synthesize_loops(W, d, member, x, p, wl):
    """Same images as :func:`synthesize_blas` by literal loops (tiny inputs only).

    Pixel loop, antenna loop with one complex exponential per (pixel, antenna)
    and an eigenvector loop accumulating R_k += conj(W_lk) B_lp, then
    |R_k|^2 into every level containing k (Algorithms 1 and 2).
    """
    W = np.asarray(W, np.complex128)
    L, K = W.shape
    n_lev = member.shape[0]
    out = np.zeros((n_lev, p.shape[0]))
    for j in range(p.shape[0]):
        R = [0j] * K
        for l in range(L):
            t = (x[l, 0] * p[j, 0] + x[l, 1] * p[j, 1] + x[l, 2] * p[j, 2]) / wl
            b = complex(np.cos(2 * np.pi * t), np.sin(2 * np.pi * t))
            for k in range(K):
                R[k] += W[l, k].conjugate() * b
        for k in range(K):
            e2 = R[k].real ** 2 + R[k].imag ** 2
            for lv in range(n_lev):
                if member[lv, k]:
                    out[lv, j] += d[k] * e2
    return out


def collect(V, x, wl, p, n_eig, intervals, filt="lsq", gram_identity=False, evaluator="blas"):
    """One full step of Algorithm 1: Gram, generalized eigensolve, selection, synthesis.

    Returns (images (N_L, N_pix), lam (K,), W (L, K), member (N_L, K)).
    ``gram_identity`` replaces G by I, which turns the image into the
    back-projected (dirty) image (Section 2.8).
    """
    G = np.eye(x.shape[0]) if gram_identity else gram(x, wl)
    lam, alpha = geneig(V, G)
    lam, W = select_top(lam, alpha, n_eig)
    member = level_membership(lam, intervals)
    d = lsq_filter(lam) if filt == "lsq" else std_filter(lam)
    f = synthesize_blas if evaluator == "blas" else synthesize_loops
    return f(W, d, member, x, p, wl), lam, W, member


def collect_beamformed(Vw, Wbf, x, wl, p, n_eig, intervals, filt="lsq"):
    """Full step with beamforming (Section 2.7): antennas combined into beams by Wbf (L x Kb).

    The sampling operator becomes Phi* = Wbf^H Psi*, so the Gram matrix is
    G^W = Wbf^H G Wbf and the eigenpairs solve Vw a = lambda G^W a (Kb x Kb).
    The eigen-images are eps = Phi a = Psi (Wbf a): the synthesis runs over the
    L antennas with U = Wbf a.  Returns (images, lam, U, member).
    """
    Wbf = np.asarray(Wbf, np.complex128)
    Gw = Wbf.conj().T @ gram(x, wl) @ Wbf
    Gw = 0.5 * (Gw + Gw.conj().T)
    lam, alpha = geneig(Vw, Gw)
    lam, alpha = select_top(lam, alpha, n_eig)
    U = Wbf @ alpha
    member = level_membership(lam, intervals)
    d = lsq_filter(lam) if filt == "lsq" else std_filter(lam)
    return synthesize_blas(U, d, member, x, p, wl), lam, U, member


def lsq_image(V, G, x, p, wl):
    """Least-squares image diag(Psi G^{-1} V G^{-1} Psi*) (Section 2.2, Eq. skyreco) by two solves.

    Uses no eigendecomposition: V' = G^{-1} V G^{-1}, I(p) = Re(b_p^H V' b_p).
    """
    Vp = np.linalg.solve(G, np.linalg.solve(G, V).conj().T).conj().T
    B = phases(x, p, wl)
    return np.real(np.einsum("lp,lm,mp->p", B.conj(), Vp, B))


def backprojection_image(V, x, p, wl):
    """Back-projected (dirty) image diag(Psi V Psi*) (Section 2.8, Eq. cleanlike)."""
    B = phases(x, p, wl)
    return np.real(np.einsum("lp,lm,mp->p", B.conj(), V, B))


def point_source_image(x, r0, p, wl, flux=1.0):
    """|sum_l exp(+j 2 pi <x_l, r0 - p> / lambda_w)|^2 * flux: a point source seen through G = I.

    This is the PSF of Section 2.8 (sum over all N_A^2 antenna pairs) centred on r0.
    """
    t = (x @ (np.asarray(r0)[None, :] - p).T) / wl
    s = np.exp(2j * np.pi * t).sum(axis=0)
    return flux * (s.real ** 2 + s.imag ** 2)
