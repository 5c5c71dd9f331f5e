"""The five synthetic workloads (C1..C5) shaped like the paper's SKA-Low / LOFAR runs.

None of the paper's datasets (OSKAR SKA-Low simulations, LOFAR Toothbrush,
MWA solar data) nor real station layouts are available; these seeded
stand-ins reproduce their shapes: station counts, baseline lengths, Earth
rotation over 6 h, image sizes and fields of view, and sky structure.

Every builder is lazy where generation is expensive: ``instance(i)``
returns one (time step, channel) instance on demand.
"""

from dataclasses import dataclass, field

import numpy as np

from . import geometry as geo
from . import sky as skymod
from . import visibilities as vis
from .levels import kmeans1d_intervals, levels_from_intervals
from .random_fields import random_eigvecs, random_eigvals
from .seeds import rng, STREAM_LAYOUT, STREAM_SKY, STREAM_NOISE, STREAM_FLAG, STREAM_WEIGHTS, STREAM_EIG


@dataclass
class Instance:
    """One (time step, channel) imaging instance."""
    x: np.ndarray            # (L, 3) float64 antenna positions, metres, this epoch
    wl: float                # wavelength, metres
    V: np.ndarray = None     # (L, L) complex128 visibility matrix (None: not simulated)
    slot: int = 0            # output image slot (channel)
    n_eig: int = 0           # eigenpairs to keep
    step: int = 0
    channel: int = 0


@dataclass
class Workload:
    name: str
    n_side: int
    fov_deg: float
    dec0_deg: float
    n_steps: int
    n_eig: int
    n_pos_levels: int
    negative_level: bool
    n_slots: int = 1
    src_ix: np.ndarray = None
    src_iy: np.ndarray = None
    meta: dict = field(default_factory=dict)
    _builder: object = None
    _pix: np.ndarray = None

    @property
    def n_pix(self):
        return self.n_side * self.n_side

    @property
    def n_levels(self):
        return self.n_pos_levels + (1 if self.negative_level else 0)

    @property
    def pix(self):
        if self._pix is None:
            self._pix = geo.pixel_grid(self.n_side, self.fov_deg, self.dec0_deg)
        return self._pix

    def instance(self, i):
        return self._builder(i)

    def n_instances(self):
        return self.meta.get("n_instances", self.n_steps)

    def source_pixels(self):
        if self.src_ix is None:
            return np.zeros(0, np.int64)
        return (np.asarray(self.src_iy) * self.n_side + np.asarray(self.src_ix)).astype(np.int64)


C1, C2, C3, C4, C5 = 1, 2, 3, 4, 5


def _sky_vis(x, dirs, flux, wl, snr, gnoise, psd):
    V = vis.visibility(x, dirs, flux, wl)
    N = vis.psd_noise(x.shape[0], gnoise) if psd else vis.hermitian_noise(x.shape[0], gnoise)
    return vis.add_noise_snr(V, N, snr)


def c1(n_ant=64, n_side=128, fov_deg=5.0, freq_hz=150e6, n_src=10, snr=20.0, psd=False,
       n_pos_levels=4, variant=0):
    """C1 small: L=64 uniform in a 2 km disk (z=0), 128^2 over 5 deg, 10 sources, SNR 20."""
    cid = C1 * 100 + variant
    x = geo.disk_layout(n_ant, 2000.0, rng(cid, STREAM_LAYOUT))
    wl = geo.wavelength_m(freq_hz)
    dirs, flux, ix, iy = skymod.point_sources(n_src, n_side, fov_deg, 90.0, rng(cid, STREAM_SKY))
    w = Workload("C1", n_side, fov_deg, 90.0, 1, n_ant, n_pos_levels, True, 1, ix, iy,
                 meta=dict(freq_hz=freq_hz, snr=snr, psd=psd, dirs=dirs, flux=flux))

    def build(i):
        assert i == 0
        V = _sky_vis(x, dirs, flux, wl, snr, rng(cid, STREAM_NOISE), psd)
        return Instance(x=x.copy(), wl=wl, V=V, slot=0, n_eig=n_ant, step=0)

    w._builder = build
    return w


def lofar_like_enu(g, n_core=128, n_arm=384):
    return geo.spiral_layout(n_core, "gaussian", 300.0, n_arm, 3, 300.0, 25_000.0, g,
                             radial_jitter=0.02, height_sigma_m=5.0)


def ska_low_like_enu(g, n_core=224, n_arm=288):
    return geo.spiral_layout(n_core, "disk", 500.0, n_arm, 3, 600.0, 32_500.0, g,
                             radial_jitter=0.02, height_sigma_m=5.0)


def c2(n_steps=100, n_side=1024, fov_deg=10.0, freq_hz=150e6, n_src=200, n_blobs=5, n_comp=256,
       snr=20.0, n_pos_levels=8, n_ant=512):
    """C2 LOFAR-like: 512 stations over 50 km, 100 epochs over 6 h, 1024^2 over 10 deg at dec +50."""
    lat, dec0 = 52.9, 50.0
    g = rng(C2, STREAM_LAYOUT)
    enu = lofar_like_enu(g, n_core=n_ant // 4, n_arm=n_ant - n_ant // 4)
    ecef = geo.enu_to_ecef(enu, lat)
    angles = geo.hour_angles(n_steps)
    wl = geo.wavelength_m(freq_hz)
    gs = rng(C2, STREAM_SKY)
    d1, f1, ix, iy = skymod.point_sources(n_src, n_side, fov_deg, dec0, gs)
    d2, f2 = skymod.gaussian_blobs(n_blobs, n_comp, fov_deg, dec0, gs)
    dirs = np.concatenate([d1, d2])
    flux = np.concatenate([f1, f2])
    w = Workload("C2", n_side, fov_deg, dec0, n_steps, n_ant, n_pos_levels, True, 1, ix, iy,
                 meta=dict(freq_hz=freq_hz, snr=snr, lat=lat, angles=angles, dirs=dirs, flux=flux,
                           ecef=ecef))

    def build(i):
        x = geo.earth_rotate(ecef, angles[i])
        V = _sky_vis(x, dirs, flux, wl, snr, rng(C2, STREAM_NOISE, i), False)
        return Instance(x=x, wl=wl, V=V, slot=0, n_eig=n_ant, step=i)

    w._builder = build
    return w


def c3(n_steps=50, n_side=2048, fov_deg=8.0, freq_hz=150e6, snr=20.0, n_pos_levels=8, n_ant=512):
    """C3 SKA-Low-like: 512 stations, 65 km max baseline, 50 epochs over 6 h, 2048^2 over 8 deg."""
    lat, dec0 = -26.7, -30.0
    g = rng(C3, STREAM_LAYOUT)
    n_core = (n_ant * 224) // 512
    enu = ska_low_like_enu(g, n_core=n_core, n_arm=n_ant - n_core)
    ecef = geo.enu_to_ecef(enu, lat)
    angles = geo.hour_angles(n_steps)
    wl = geo.wavelength_m(freq_hz)
    dirs, flux, ix, iy = skymod.grid_sources(n_side, fov_deg, dec0)
    w = Workload("C3", n_side, fov_deg, dec0, n_steps, n_ant, n_pos_levels, True, 1, ix, iy,
                 meta=dict(freq_hz=freq_hz, snr=snr, lat=lat, angles=angles, dirs=dirs, flux=flux,
                           ecef=ecef))

    def build(i):
        x = geo.earth_rotate(ecef, angles[i])
        V = _sky_vis(x, dirs, flux, wl, snr, rng(C3, STREAM_NOISE, i), False)
        return Instance(x=x, wl=wl, V=V, slot=0, n_eig=n_ant, step=i)

    w._builder = build
    return w


def c4(n_channels=64, n_steps=32, n_side=512, fov_deg=10.0, f_lo=100e6, f_hi=200e6,
       l_range=(200, 512), k_range=(16, 128), n_pos_levels=4, simulate_vis=False, snr=20.0):
    """C4 batched uneven instances: 64 channels x 32 epochs of a flagged C2 array.

    Per instance ``L_i ~ U{200..512}`` stations (drawn without replacement)
    and ``K_i ~ U{16..128}`` kept eigenpairs in 4 levels.  By default the
    eigenpairs are random stand-ins (``simulate_vis=False``), because 2048
    dense eigensolves would dominate any test; with ``simulate_vis`` the
    instance carries its visibility matrix instead.
    """
    base = c2(n_steps=n_steps, n_side=n_side, fov_deg=fov_deg, n_pos_levels=n_pos_levels)
    ecef = base.meta["ecef"]
    angles = base.meta["angles"]
    freqs = np.linspace(f_lo, f_hi, n_channels)
    n_inst = n_channels * n_steps
    gf = rng(C4, STREAM_FLAG)
    Ls = gf.integers(l_range[0], l_range[1] + 1, n_inst)
    Ks = gf.integers(k_range[0], k_range[1] + 1, n_inst)
    w = Workload("C4", n_side, fov_deg, base.dec0_deg, n_steps, int(k_range[1]), n_pos_levels, False,
                 n_channels, base.src_ix, base.src_iy,
                 meta=dict(freqs=freqs, Ls=Ls, Ks=Ks, n_instances=n_inst, n_channels=n_channels,
                           dirs=base.meta["dirs"], flux=base.meta["flux"], snr=snr))

    def build(i):
        ch, st = divmod(int(i), n_steps)
        gi = rng(C4, STREAM_FLAG, i)
        keep = np.sort(gi.choice(ecef.shape[0], size=int(Ls[i]), replace=False))
        x = geo.earth_rotate(ecef[keep], angles[st])
        wl = geo.wavelength_m(freqs[ch])
        inst = Instance(x=x, wl=wl, slot=ch, n_eig=int(Ks[i]), step=st, channel=ch)
        if simulate_vis:
            inst.V = _sky_vis(x, w.meta["dirs"], w.meta["flux"], wl, snr, rng(C4, STREAM_NOISE, i), False)
        else:
            ge = rng(C4, STREAM_EIG, i)
            K = int(Ks[i])
            inst.W = random_eigvecs(x.shape[0], K, ge)
            lam = random_eigvals(K, ge, frac_neg=0.0)
            inst.lam = lam
            inst.intervals = kmeans1d_intervals(lam, n_pos_levels, negative_level=False)
            inst.level_of = levels_from_intervals(lam, inst.intervals)
        return inst

    w._builder = build
    return w


def c5(n_ant=256, n_side=512, fov_deg=5.0, freq_hz=150e6, n_src=10, snr=20.0, n_eig=64,
       n_pos_levels=4):
    """C5 differentiation: L=256 in a 2 km disk with N(0, 1 m) heights, 512^2 over 5 deg, K=64."""
    x = geo.disk_layout(n_ant, 2000.0, rng(C5, STREAM_LAYOUT), z_sigma_m=1.0)
    wl = geo.wavelength_m(freq_hz)
    dirs, flux, ix, iy = skymod.point_sources(n_src, n_side, fov_deg, 90.0, rng(C5, STREAM_SKY))
    w = Workload("C5", n_side, fov_deg, 90.0, 1, n_eig, n_pos_levels, False, 1, ix, iy,
                 meta=dict(freq_hz=freq_hz, snr=snr, dirs=dirs, flux=flux))

    def build(i):
        assert i == 0
        V = _sky_vis(x, dirs, flux, wl, snr, rng(C5, STREAM_NOISE), False)
        return Instance(x=x.copy(), wl=wl, V=V, slot=0, n_eig=n_eig, step=0)

    w._builder = build
    w.meta["loss_weights"] = lambda: rng(C5, STREAM_WEIGHTS).standard_normal((n_pos_levels, n_side * n_side))
    return w
