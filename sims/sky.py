"""Synthetic skies: point sources and Gaussian blobs sampled as point components.

Each function returns ``(directions (S, 3) float64 unit vectors, fluxes (S,) float64)``
and, for sources placed on pixel centres, their (ix, iy) pixel indices.
"""

import numpy as np

from .geometry import tangent_basis, direction_cosines, pixel_index_direction

ARCMIN = np.pi / (180.0 * 60.0)


def _lm_to_dir(l_, m_, dec0_deg):
    e1, e2, p0 = tangent_basis(dec0_deg)
    n_ = np.sqrt(1.0 - l_ * l_ - m_ * m_)
    return l_[:, None] * e1 + m_[:, None] * e2 + n_[:, None] * p0


def point_sources(n_src, n_pix_side, fov_deg, dec0_deg, g, snap=True, log_sigma=1.0):
    """``n_src`` sources uniform in the field with log-normal flux ``exp(N(0, log_sigma))``.

    With ``snap`` the positions are moved to pixel centres (the paper places
    its validation sources on pixel centres, Section 4.1).  Returns
    ``(dirs, flux, ix, iy)``; ``ix``/``iy`` are None when not snapped.
    """
    flux = np.exp(g.normal(0.0, log_sigma, n_src))
    if snap:
        ix = g.integers(0, n_pix_side, n_src)
        iy = g.integers(0, n_pix_side, n_src)
        return pixel_index_direction(n_pix_side, fov_deg, dec0_deg, ix, iy), flux, ix, iy
    h = np.sin(np.deg2rad(fov_deg) / 2.0)
    l_ = g.uniform(-h, h, n_src)
    m_ = g.uniform(-h, h, n_src)
    return _lm_to_dir(l_, m_, dec0_deg), flux, None, None


def gaussian_blobs(n_blobs, n_comp, fov_deg, dec0_deg, g, fwhm_arcmin=(3.0, 15.0),
                   flux_mu=np.log(5.0), flux_sigma=0.5):
    """Diffuse blobs, each sampled as ``n_comp`` equal-flux point components.

    Blob centres are uniform in the field, FWHM ~ U(fwhm_arcmin), total flux
    log-normal(flux_mu, flux_sigma).  Returns ``(dirs, flux)``.
    """
    h = np.sin(np.deg2rad(fov_deg) / 2.0)
    dirs, flux = [], []
    for _ in range(n_blobs):
        lc, mc = g.uniform(-0.8 * h, 0.8 * h, 2)
        fwhm = g.uniform(*fwhm_arcmin) * ARCMIN
        sig = fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))
        tot = np.exp(g.normal(flux_mu, flux_sigma))
        l_ = lc + sig * g.standard_normal(n_comp)
        m_ = mc + sig * g.standard_normal(n_comp)
        dirs.append(_lm_to_dir(l_, m_, dec0_deg))
        flux.append(np.full(n_comp, tot / n_comp))
    return np.concatenate(dirs), np.concatenate(flux)


def grid_sources(n_pix_side, fov_deg, dec0_deg, fractions=(1, 4, 7), denom=8, flux=1.0):
    """Sources on the pixel centres at ``fractions/denom`` of the width on both axes.

    With the defaults these are the paper's nine 1 Jy validation sources
    (Section 4.1, footnote on source placement).  Returns ``(dirs, flux, ix, iy)``.
    """
    idx = np.array([(f * n_pix_side) // denom for f in fractions])
    ix, iy = np.meshgrid(idx, idx, indexing="xy")
    ix = ix.ravel()
    iy = iy.ravel()
    dirs = pixel_index_direction(n_pix_side, fov_deg, dec0_deg, ix, iy)
    return dirs, np.full(ix.size, float(flux)), ix, iy


__all__ = ["point_sources", "gaussian_blobs", "grid_sources", "direction_cosines"]
