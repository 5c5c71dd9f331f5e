"""NUFFT synthesis (test infrastructure only).

The least-squares image of a level is also a Fourier sum over baselines
(Section 2.5): with the Gram-corrected visibilities V'_l = A_l Lambda_l A_l^H
(the eigenpairs of the level, the others set to zero),

    I_l(p) = sum_{l,m} V'_l[m, l] exp(+2 pi i <b_lm, p>),   b_lm = (x_l - x_m) / lambda_w,

in the sign convention of the phase matrix B = exp(+2 pi i <x, p> / lambda_w)
used everywhere here (Section 2.4 then gives exactly the same image).  The
paper evaluates this type-3 (nonuniform to nonuniform) sum with a NUFFT
(Section 3.4, Algorithm 3): rescale the coordinates, spread the sources onto
a fine regular grid with the "exponential of semicircle" kernel, evaluate
that grid's Fourier series at the rescaled targets with a type-2 NUFFT, and
divide by the kernel's Fourier transform.  This module writes those steps out
in FP64 (``nufft3``), next to the exact sum they approximate (``nudft3``).

Readings (the paper gives the steps, not the constants):
  * Hermitian symmetry: V'_l is Hermitian and b_ml = -b_lm, so
    I_l = sum_l V'_l[l, l] + 2 Re sum_{l < m} V'_l[m, l] e^{+2 pi i <b_lm, p>};
    only the pairs l < m are transformed;
  * kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1, with
    w grid points of support (one more than the digits asked for), beta = 2.30 w and
    upsampling sigma = 2 (the published choices of Barnett, Magland and
    af Klinteberg, 2019, for this kernel);
  * the transform runs in an image frame (e_u, e_v, p0): the pixels of a
    field of view then span a small range along p0, and the grid stays thin
    along that axis.  Rotated coordinates are ((a0 e0 + a1 e1) + a2 e2),
    evaluated in that order;
  * per axis d, with sources centred at 0 (half-width X_d, a given bound on
    |b_d|) and targets centred at D_d (half-width S_d, floored at 1e-12):
    spacing h_d = 1 / (2 sigma S_d) turns (the targets use half of the grid's
    band) and N_d = smooth(max(2 w, ceil(2 sigma (2 pi X_d) S_d / pi) + w))
    = smooth(max(2 w, ceil(8 X_d S_d) + w)) spread-grid points, so the spread
    sources do not wrap around; the type-2 grid has M_d = sigma N_d points;
  * w is evaluated as ceil(log10(1 / eps) - 1e-9) + 1, so that a tolerance
    that is a power of ten does not gain a point from rounding;
  * grid coordinates are formed as x * (1 / h) for sources and
    (s - D) * (h * M) for targets, and the w points used are the half-open
    window [xi - w/2, xi + w/2): ceil(xi - w/2) .. ceil(xi - w/2) + w - 1.
    The kernel is e^{-beta}, not 0, at the ends of its support, so when a
    coordinate lands exactly on a grid point (the extreme pixels do: they sit
    at +-S, i.e. at +-M/4) the window could keep either end, and the two
    choices differ by about e^{-beta} of a grid value.  Section 3.4 fixes
    neither the window nor the arithmetic of the coordinates; both are a
    convention here (``tie="low"`` keeps the lower end, ``tie="high"`` the
    upper one), and either meets the same accuracy bound against the exact
    sum (pinned on the CPU), which is what the method promises;
  * "smooth" is the least even integer >= n with no prime factor above 5;
  * kernel Fourier transforms are evaluated by 100-node Gauss-Legendre
    quadrature of the (even) kernel.

Coordinates are in turns: the phase of source x at target s is 2 pi <x, s>.
"""

import math

import numpy as np

__all__ = ["level_visibilities", "nudft3", "kernel_width", "plan_params", "rotate", "es_kernel", "kernel_ft",
           "nufft3", "nufft3_uvw_cells", "nufft_image", "nufft_images", "smooth_size", "uvw_cell", "uvw_cell_centre"]

SIGMA = 2
QUAD_NODES = 100


def level_visibilities(W, d, member):
    """V'_l = W_l diag(d_l) W_l^H for each level l: (N_L, L, L) complex128 (Section 2.5)."""
    W = np.asarray(W, np.complex128)
    out = []
    for row in np.asarray(member, bool):
        Wl = W[:, row]
        out.append((Wl * np.asarray(d, np.float64)[row]) @ Wl.conj().T)
    return np.array(out)


def nudft3(c, x, s):
    """Exact type-3 sum f_k = sum_j c_j exp(+2 pi i <s_k, x_j>) (the definition)."""
    c = np.asarray(c, np.complex128)
    ph = np.asarray(s, np.float64) @ np.asarray(x, np.float64).T       # (n_targets, n_sources), turns
    ph = ph - np.rint(ph)
    return np.exp(2j * np.pi * ph) @ c


def smooth_size(n):
    """Least even integer >= n whose prime factors are all 2, 3 or 5."""
    n = max(int(n), 2)
    while True:
        if n % 2 == 0:
            m = n
            for p in (2, 3, 5):
                while m % p == 0:
                    m //= p
            if m == 1:
                return n
        n += 1


def kernel_width(eps):
    """Grid points of kernel support for tolerance eps."""
    return int(math.ceil(math.log10(1.0 / eps) - 1e-9)) + 1


def plan_params(eps, X, s):
    """Kernel and grid parameters from the tolerance, the source half-widths X (3,) and the targets s."""
    w = kernel_width(eps)
    beta = 2.30 * w
    s = np.asarray(s, np.float64)
    lo, hi = s.min(axis=0), s.max(axis=0)
    D = 0.5 * (lo + hi)
    S = np.maximum(0.5 * (hi - lo), 1e-12)
    X = np.asarray(X, np.float64)
    h = 1.0 / (2.0 * SIGMA * S)                     # turns: 2 pi h S = pi / sigma
    N = np.array([smooth_size(max(2 * w, math.ceil(8.0 * X[i] * S[i]) + w)) for i in range(3)])
    M = SIGMA * N
    return dict(w=w, beta=beta, D=D, S=S, X=X, h=h, N=N, M=M)


def rotate(a, frame):
    """Coordinates of the rows of a (n, 3) along the rows of frame (3, 3), as ((a0 e0 + a1 e1) + a2 e2)."""
    a = np.asarray(a, np.float64)
    R = np.asarray(frame, np.float64)
    return np.stack([(a[:, 0] * R[d, 0] + a[:, 1] * R[d, 1]) + a[:, 2] * R[d, 2] for d in range(3)], axis=1)


def es_kernel(z, beta):
    """phi(z) = exp(beta (sqrt(1 - z^2) - 1)) for |z| <= 1, else 0."""
    z = np.asarray(z, np.float64)
    out = np.zeros_like(z)
    inside = np.abs(z) <= 1.0
    out[inside] = np.exp(beta * (np.sqrt(1.0 - z[inside] ** 2) - 1.0))
    return out


def kernel_ft(k, half_width, beta):
    """integral of phi(z / a) exp(i k z) dz over |z| <= a (a = half_width): a * int_{-1}^{1} phi(t) cos(k a t) dt."""
    t, wq = np.polynomial.legendre.leggauss(QUAD_NODES)
    k = np.asarray(k, np.float64)
    vals = es_kernel(t, beta)
    return half_width * np.cos(np.multiply.outer(k * half_width, t)) @ (wq * vals)


def _neighbours(xi, w, tie="low"):
    """The w integer grid points of the window around xi, and the kernel arguments (g - xi) / (w/2).

    tie="low": the half-open window [xi - w/2, xi + w/2); tie="high": (xi - w/2, xi + w/2].
    They differ only when xi - w/2 is an integer.
    """
    if tie == "low":
        first = np.ceil(xi - 0.5 * w).astype(np.int64)
    elif tie == "high":
        first = np.floor(xi - 0.5 * w).astype(np.int64) + 1
    else:
        raise ValueError("tie must be 'low' or 'high'")
    g = first[..., None] + np.arange(w)
    return g, (g - xi[..., None]) / (0.5 * w)


def nufft3(c, x, s, eps, X=None, tie="low"):
    """Type-3 NUFFT approximation of nudft3(c, x, s) in the steps of Section 3.4.

    c: (n_src, n_ch) strengths (several channels share the coordinates);
    x: (n_src, 3) sources, centred at 0, |x_d| <= X_d; s: (n_tgt, 3) targets;
    tie: which end of the kernel window is kept when a grid coordinate sits
    exactly half a support from a grid point (see the module notes).
    Returns (n_tgt, n_ch) complex128.
    """
    c = np.asarray(c, np.complex128)
    if c.ndim == 1:
        c = c[:, None]
    x = np.asarray(x, np.float64)
    s = np.asarray(s, np.float64)
    if X is None:
        X = np.max(np.abs(x), axis=0)
    P = plan_params(eps, X, s)
    w, beta, D, h, N, M = P["w"], P["beta"], P["D"], P["h"], P["N"], P["M"]
    if np.any(np.abs(x) > P["X"][None, :] * (1 + 1e-12)):
        raise ValueError("a source lies outside the planned extent")

    # 1. rescale: sources in spread-grid units; pre-phase so the targets are centred at D
    xi = x * (1.0 / h)[None, :]
    pre = np.exp(2j * np.pi * (x @ D - np.rint(x @ D)))
    cs = c * pre[:, None]

    # 2. spread onto the periodic N grid with the tensor-product kernel
    grid = np.zeros((c.shape[1],) + tuple(N), np.complex128)
    gi, ki = [], []
    for d in range(3):
        g, z = _neighbours(xi[:, d], w, tie)
        gi.append(np.mod(g, N[d]))
        ki.append(es_kernel(z, beta))
    n_src = x.shape[0]
    idx = (gi[0][:, :, None, None] * N[1] + gi[1][:, None, :, None]) * N[2] + gi[2][:, None, None, :]
    ker = ki[0][:, :, None, None] * ki[1][:, None, :, None] * ki[2][:, None, None, :]
    flat_idx = idx.reshape(n_src, -1)
    flat_ker = ker.reshape(n_src, -1)
    for ch in range(c.shape[1]):
        acc = np.zeros(int(np.prod(N)), np.complex128)
        np.add.at(acc, flat_idx.ravel(), (flat_ker * cs[:, ch:ch + 1]).ravel())
        grid[ch] = acc.reshape(tuple(N))

    # 3. type-2 NUFFT of the grid's Fourier series: deconvolve, zero-pad to M, FFT (e^{+i}), interpolate
    # With the type-2 kernel psi(z) = phi(z / (w pi / M)) on the M-grid z_m = 2 pi m / M,
    # sum_m u_m psi(t - z_m) = (M / 2 pi) sum_g (b_g / psi_hat(g)) psi_hat(g) e^{i g t} up to aliasing;
    # deconvolving by psi_hat(g) M / (2 pi) = (w/2) int phi(t) cos(g (2 pi / M)(w/2) t) dt
    # makes the interpolated value the Fourier series sum_g b_g e^{i g t} itself.
    freqs = [np.fft.fftfreq(N[d], 1.0 / N[d]).astype(np.int64) for d in range(3)]   # g for each stored index
    psi_hat = [kernel_ft(freqs[d] * (2 * np.pi / M[d]), 0.5 * w, beta) for d in range(3)]
    corr = psi_hat[0][:, None, None] * psi_hat[1][None, :, None] * psi_hat[2][None, None, :]
    big = np.zeros((c.shape[1],) + tuple(M), np.complex128)
    ix = np.ix_(np.mod(freqs[0], M[0]), np.mod(freqs[1], M[1]), np.mod(freqs[2], M[2]))
    for ch in range(c.shape[1]):
        big[ch][ix] = grid[ch] / corr
    u = np.fft.ifftn(big, axes=(1, 2, 3)) * float(np.prod(M))

    st = s - D[None, :]
    eta = st * (h * M)[None, :]                   # targets in type-2 grid units (2 pi s h M / (2 pi))
    gi, ki = [], []
    for d in range(3):
        g, z = _neighbours(eta[:, d], w, tie)
        gi.append(np.mod(g, M[d]))
        ki.append(es_kernel(z, beta))
    n_tgt = s.shape[0]
    idx = (gi[0][:, :, None, None] * M[1] + gi[1][:, None, :, None]) * M[2] + gi[2][:, None, None, :]
    ker = ki[0][:, :, None, None] * ki[1][:, None, :, None] * ki[2][:, None, None, :]
    F = np.einsum("tq,ctq->tc", ker.reshape(n_tgt, -1), u.reshape(c.shape[1], -1)[:, idx.reshape(n_tgt, -1)])

    # 4. diagonal correction: divide by the spreading kernel's transform at each target
    phi_hat = np.ones(n_tgt)
    for d in range(3):
        phi_hat = phi_hat * kernel_ft(2 * np.pi * st[:, d], 0.5 * w * h[d], beta) / h[d]
    return F / phi_hat[:, None]


def uvw_cell(b, X, q):
    """uvw cell of baseline coordinates b along one axis: floor((b + X) q / (2 X)), clamped to [0, q - 1]."""
    c = np.floor((np.asarray(b, np.float64) + X) * (q / (2.0 * X))).astype(np.int64)
    return np.clip(c, 0, q - 1)


def uvw_cell_centre(i, X, q):
    """Centre of cell i of q along an axis of half-width X: (i + 1/2) (2 X / q) - X."""
    return (i + 0.5) * (2.0 * X / q) - X


def nufft3_uvw_cells(c, x, s, eps, X, q, tie="low"):
    """nufft3 with the sources split into q x q cells along axes 0 and 1 (Section 3.4.1).

    The sum over all sources is the sum over the cells; a cell's sources are
    shifted by its centre C (the sum then gains the factor exp(2 pi i <s, C>))
    and transformed with the cell's half-width (X / q)(1 + 1e-9) on axes 0, 1.
    """
    c = np.asarray(c, np.complex128)
    if c.ndim == 1:
        c = c[:, None]
    x = np.asarray(x, np.float64)
    s = np.asarray(s, np.float64)
    X = np.asarray(X, np.float64)
    iu, iv = uvw_cell(x[:, 0], X[0], q), uvw_cell(x[:, 1], X[1], q)
    Xc = X.copy()
    Xc[:2] = (X[:2] / q) * (1.0 + 1e-9)
    out = np.zeros((s.shape[0], c.shape[1]), np.complex128)
    for a in range(q):
        for b in range(q):
            sel = (iu == a) & (iv == b)
            if not np.any(sel):
                continue
            C = np.array([uvw_cell_centre(a, X[0], q), uvw_cell_centre(b, X[1], q), 0.0])
            t = s @ C
            out += nufft3(c[sel], x[sel] - C, s, eps, X=Xc, tie=tie) * np.exp(2j * np.pi * (t - np.rint(t)))[:, None]
    return out


def nufft_images(instances, pix, eps, X=None, frame=None, tie="low", uvw_cells=1):
    """Level images summed over instances by NUFFT synthesis.

    instances: iterable of (x (L, 3) metres, wavelength, W (L, K), d (K,), member (N_L, K) bool).
    frame: rows e_u, e_v, p0 (default: the identity); X: per-axis bound on |b| in
    wavelengths in that frame (default: the largest over the instances); tie: as in nufft3;
    uvw_cells: q > 1 splits the baselines into q x q cells of [-X, X] along e_u, e_v
    (nufft3_uvw_cells).
    Returns (N_L, N_pix) float64.
    """
    R = np.eye(3) if frame is None else np.asarray(frame, np.float64)
    pos, val, diag = [], [], 0.0
    for x, wl, W, d, member in instances:
        Vp = level_visibilities(W, d, member)                   # (N_L, L, L)
        li, mi = np.triu_indices(x.shape[0], k=1)              # l < m
        pos.append(rotate(x[li] - x[mi], R) / wl)
        val.append(Vp[:, mi, li].T)                            # V'[m, l]
        diag = diag + np.real(np.einsum("nll->n", Vp))
    pos = np.concatenate(pos)
    val = np.concatenate(val)
    if uvw_cells > 1:
        if X is None:
            X = np.max(np.abs(pos), axis=0)
        f = nufft3_uvw_cells(val, pos, rotate(pix, R), eps, X, uvw_cells, tie=tie)
    else:
        f = nufft3(val, pos, rotate(pix, R), eps, X=X, tie=tie)    # (N_pix, N_L)
    return (2.0 * np.real(f)).T + np.asarray(diag)[:, None]


def nufft_image(x, wl, W, d, member, pix, eps, X=None, frame=None):
    """NUFFT synthesis of one instance: (N_L, N_pix) float64."""
    return nufft_images([(x, wl, W, d, member)], pix, eps, X=X, frame=frame)
