"""Antenna layouts, Earth rotation and pixel grids (all FP64, metres / unit vectors).

Frame: an Earth-fixed Cartesian frame whose z axis is the rotation axis, and
whose x axis points to longitude 0 at the start of the observation.  Celestial
directions are unit vectors in the same axes at hour angle 0; Earth rotation
is applied to the antennas (the sky stays fixed), which is what makes the
sampling operator time dependent (Section 2.4).
"""

import numpy as np

C_LIGHT = 299_792_458.0  # m/s
SIDEREAL_DAY_S = 86_164.0905


def wavelength_m(freq_hz):
    """Wavelength c/f in metres (the paper's garbled "lambda = f/c" read as c/f)."""
    return C_LIGHT / float(freq_hz)


def disk_layout(n, diameter_m, g, z_sigma_m=0.0):
    """``n`` antennas uniform in a disk of the given diameter (ENU metres)."""
    r = 0.5 * diameter_m * np.sqrt(g.random(n))
    th = 2.0 * np.pi * g.random(n)
    z = g.normal(0.0, z_sigma_m, n) if z_sigma_m > 0 else np.zeros(n)
    return np.stack([r * np.cos(th), r * np.sin(th), z], axis=1)


def _core_gaussian(n, sigma_m, g):
    xy = g.normal(0.0, sigma_m, (n, 2))
    return np.concatenate([xy, np.zeros((n, 1))], axis=1)


def _core_disk(n, radius_m, g):
    return disk_layout(n, 2.0 * radius_m, g)[:, :]


def spiral_layout(n_core, core, core_scale_m, n_arm_total, n_arms, r_min_m, r_max_m, g,
                  radial_jitter=0.02, height_sigma_m=5.0, turns=1.25):
    """Core plus ``n_arms`` logarithmic spiral arms ``r = r0 * exp(b * theta)``.

    ``core`` is ``"gaussian"`` (``core_scale_m`` = sigma) or ``"disk"``
    (``core_scale_m`` = radius).  Arm stations are evenly spaced in
    ``theta`` (hence in log r) from ``r_min_m`` to ``r_max_m`` over ``turns``
    revolutions, with a multiplicative radial jitter and Gaussian heights.
    """
    if core == "gaussian":
        c = _core_gaussian(n_core, core_scale_m, g)
    elif core == "disk":
        c = _core_disk(n_core, core_scale_m, g)
    else:
        raise ValueError(core)
    per_arm = [n_arm_total // n_arms + (1 if a < n_arm_total % n_arms else 0) for a in range(n_arms)]
    th_max = 2.0 * np.pi * turns
    b = np.log(r_max_m / r_min_m) / th_max
    arms = []
    for a, m in enumerate(per_arm):
        th = np.linspace(0.0, th_max, m)
        r = r_min_m * np.exp(b * th) * (1.0 + radial_jitter * g.standard_normal(m))
        phi = th + 2.0 * np.pi * a / n_arms
        arms.append(np.stack([r * np.cos(phi), r * np.sin(phi), np.zeros(m)], axis=1))
    enu = np.concatenate([c] + arms, axis=0)
    enu[:, 2] = g.normal(0.0, height_sigma_m, enu.shape[0]) if height_sigma_m > 0 else 0.0
    return enu


def enu_to_ecef(enu, lat_deg):
    """Rotate local East/North/Up offsets at (lat, lon=0) into the Earth-fixed frame."""
    phi = np.deg2rad(lat_deg)
    east = np.array([0.0, 1.0, 0.0])
    north = np.array([-np.sin(phi), 0.0, np.cos(phi)])
    up = np.array([np.cos(phi), 0.0, np.sin(phi)])
    return enu[:, 0:1] * east + enu[:, 1:2] * north + enu[:, 2:3] * up


def earth_rotate(xyz, angle_rad):
    """Rotate Earth-fixed positions about the z (polar) axis by ``angle_rad``."""
    c, s = np.cos(angle_rad), np.sin(angle_rad)
    out = np.empty_like(xyz)
    out[:, 0] = c * xyz[:, 0] - s * xyz[:, 1]
    out[:, 1] = s * xyz[:, 0] + c * xyz[:, 1]
    out[:, 2] = xyz[:, 2]
    return out


def hour_angles(n_steps, span_hours=6.0):
    """Earth-rotation angles (rad) of ``n_steps`` epochs evenly spread over ``span_hours``."""
    if n_steps == 1:
        return np.zeros(1)
    span = 2.0 * np.pi * span_hours * 3600.0 / SIDEREAL_DAY_S
    return np.linspace(-0.5 * span, 0.5 * span, n_steps)


def tangent_basis(dec0_deg):
    """Orthonormal (e1, e2, p0) at the phase centre of declination dec0 (p0 the centre)."""
    d = np.deg2rad(dec0_deg)
    p0 = np.array([np.cos(d), 0.0, np.sin(d)])
    e1 = np.array([0.0, 1.0, 0.0])
    e2 = np.array([-np.sin(d), 0.0, np.cos(d)])
    return e1, e2, p0


def direction_cosines(n, fov_deg):
    """Pixel-centre direction cosines of an ``n``-point axis spanning the field of view."""
    h = np.sin(np.deg2rad(fov_deg) / 2.0)
    return -h + (np.arange(n) + 0.5) * (2.0 * h / n)


def pixel_grid(n, fov_deg, dec0_deg=90.0):
    """``n*n`` unit vectors, row-major (index ``iy*n + ix``), around the phase centre.

    ``p = l e1 + m e2 + sqrt(1 - l^2 - m^2) p0`` with (l, m) on a regular
    direction-cosine grid; ``dec0_deg = 90`` puts the phase centre on +z.
    Returned as an (n*n, 3) float64 array.
    """
    e1, e2, p0 = tangent_basis(dec0_deg)
    lc = direction_cosines(n, fov_deg)
    ll, mm = np.meshgrid(lc, lc, indexing="xy")
    ll = ll.ravel()
    mm = mm.ravel()
    nn = np.sqrt(1.0 - ll * ll - mm * mm)
    return ll[:, None] * e1 + mm[:, None] * e2 + nn[:, None] * p0


def pixel_index_direction(n, fov_deg, dec0_deg, ix, iy):
    """Unit vector of pixel centre (ix, iy) of :func:`pixel_grid`."""
    e1, e2, p0 = tangent_basis(dec0_deg)
    lc = direction_cosines(n, fov_deg)
    ix = np.asarray(ix)
    iy = np.asarray(iy)
    l_ = lc[ix]
    m_ = lc[iy]
    n_ = np.sqrt(1.0 - l_ * l_ - m_ * m_)
    return l_[..., None] * e1 + m_[..., None] * e2 + n_[..., None] * p0
