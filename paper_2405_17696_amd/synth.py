"""Seeded synthetic inputs: velocity media, absorbing layer, frequencies, sources, receivers.

This module builds the *inputs* of the Helmholtz problem and nothing else: it
holds none of the method's arithmetic (no operator, no solver, no network), so
the CPU oracle and the GPU library can both be fed from it.

The paper's media (SEG/EAGE salt, Marmousi; Sec. 5.2 and 5.5) are 2:1 grids with
a slow top, layered sediments, faults and a fast body.  Those models are not
available here; the generators below reproduce their *structure* (layers, a
Gaussian-random-field texture, a dipping fault, a fast elliptic inclusion) on
seeded synthetic grids.  Units: km and km/s, so kappa2 = 1/c**2 in s^2/km^2 and
omega in rad/s.

Conventions shared by every consumer:
  * arrays are row-major [nz][nx], x (columns) fastest, row 0 is the surface;
  * gamma is the dimensionless attenuation fraction of eq. (3.1), used as
    H = -Lap - omega^2 kappa2 (1 - i gamma);
  * a point source is the grid delta e_s / (hx*hz) (Sec. 3.1, "discretization of
    a delta function").
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

H_DEFAULT = 0.0125      # km (12.5 m)
C_MIN, C_MAX = 1.5, 4.5  # km/s
ABL_WIDTH = 16
GAMMA_MAX = 0.5


def rng_for(config: int, item: int = 0) -> np.random.Generator:
    """Seed scheme 1000*config + item."""
    return np.random.default_rng(1000 * config + item)


# ----------------------------------------------------------------------------
# random fields and media
# ----------------------------------------------------------------------------
def grf(nz: int, nx: int, rng: np.random.Generator, corr_len: float = 20.0) -> np.ndarray:
    """Gaussian random field: white N(0,1) filtered in Fourier space so that its
    covariance is Gaussian with correlation length `corr_len` cells, then
    normalised to zero mean and unit standard deviation."""
    w = rng.standard_normal((nz, nx))
    kz = np.fft.fftfreq(nz) * 2.0 * np.pi
    kx = np.fft.fftfreq(nx) * 2.0 * np.pi
    k2 = kz[:, None] ** 2 + kx[None, :] ** 2
    # covariance exp(-r^2 / (2 l^2)) has spectral density ~ exp(-l^2 k^2 / 2);
    # the amplitude filter is its square root
    f = np.exp(-(corr_len ** 2) * k2 / 4.0)
    g = np.real(np.fft.ifft2(np.fft.fft2(w) * f))
    g -= g.mean()
    s = g.std()
    return g / s if s > 0 else g


def velocity_grf(nz: int, nx: int, rng: np.random.Generator) -> np.ndarray:
    """Smooth GRF velocity rescaled exactly onto [1.5, 4.5] km/s."""
    g = grf(nz, nx, rng)
    span = g.max() - g.min()
    if span <= 1e-12 * max(1.0, abs(g).max()):   # grid far smaller than the correlation length
        return np.full((nz, nx), 0.5 * (C_MIN + C_MAX))
    return C_MIN + (C_MAX - C_MIN) * (g - g.min()) / span


def _layer_params(rng: np.random.Generator, nlayers: int = 8):
    """Relative interface depths in [16/256, 240/256) and sorted velocities."""
    depths = np.sort(rng.uniform(16.0 / 256.0, 240.0 / 256.0, size=nlayers - 1))
    vels = np.sort(rng.uniform(C_MIN, C_MAX, size=nlayers))
    return depths, vels


def _layered_from_params(nz: int, nx: int, depths: np.ndarray, vels: np.ndarray,
                         depth_field: np.ndarray | None = None) -> np.ndarray:
    zrel = (np.arange(nz)[:, None] + 0.5) / nz * np.ones((1, nx))
    if depth_field is not None:
        zrel = depth_field
    idx = np.searchsorted(depths, zrel, side="right")
    return vels[idx]


def velocity_layered(nz: int, nx: int, rng: np.random.Generator, sigma: float = 0.1,
                     nlayers: int = 8) -> np.ndarray:
    """8 random flat layers, velocity increasing with depth, times (1 + sigma*GRF),
    clipped to [1.5, 4.5] km/s."""
    depths, vels = _layer_params(rng, nlayers)
    c = _layered_from_params(nz, nx, depths, vels)
    c = c * (1.0 + sigma * grf(nz, nx, rng))
    return np.clip(c, C_MIN, C_MAX)


@dataclass
class FaultedModel:
    """One physical model (layers + dipping fault + fast elliptic inclusion),
    sampled on any grid by `sample(nz, nx)` (relative coordinates in [0,1))."""
    depths: np.ndarray
    vels: np.ndarray
    fault_x0: float
    fault_angle: float
    throw: float
    ell_cx: float
    ell_cz: float
    ell_ax: float
    ell_az: float
    c_incl: float = 4.5

    def sample(self, nz: int, nx: int) -> np.ndarray:
        z = (np.arange(nz)[:, None] + 0.5) / nz * np.ones((1, nx))
        x = (np.arange(nx)[None, :] + 0.5) / nx * np.ones((nz, 1))
        # fault plane x = x0 + z / tan(angle) (relative units, aspect 2:1)
        xf = self.fault_x0 + z * 0.5 / math.tan(self.fault_angle)
        hanging = x > xf
        zeff = np.where(hanging, z - self.throw * z, z)
        c = _layered_from_params(nz, nx, self.depths, self.vels, depth_field=zeff)
        inside = ((x - self.ell_cx) / self.ell_ax) ** 2 + ((z - self.ell_cz) / self.ell_az) ** 2 <= 1.0
        c = np.where(inside, self.c_incl, c)
        return c


def faulted_model(rng: np.random.Generator) -> FaultedModel:
    depths, vels = _layer_params(rng)
    angle = math.radians(rng.uniform(20.0, 70.0))
    throw = rng.uniform(0.05, 0.15)
    x0 = rng.uniform(0.25, 0.55)
    ax = rng.uniform(0.10, 0.20)
    az = rng.uniform(0.05, 0.12)
    cz = rng.uniform(1.0 / 3.0 + az, 1.0 - az - 16.0 / 256.0)
    cx = rng.uniform(0.2 + ax, 0.8 - ax)
    return FaultedModel(depths, vels, x0, angle, throw, cx, cz, ax, az)


def velocity_linear(nz: int, nx: int, rng: np.random.Generator) -> np.ndarray:
    """Random linear slowness-squared model (the pre-training media of Sec. 4.1):
    velocities for the top and the bottom row drawn at random within the
    physical range (top 1.5-2.5 km/s, bottom up to 4.5 km/s, faster than the
    top), and m = 1/c^2 in uniform steps between the two rows' values;
    returned as the velocity 1/sqrt(m)."""
    top = rng.uniform(1.5, 2.5)
    bot = rng.uniform(max(top, 2.5), 4.5)
    z = np.arange(nz)[:, None] / max(nz - 1, 1)
    m = 1.0 / top ** 2 + (1.0 / bot ** 2 - 1.0 / top ** 2) * z
    return np.repeat(1.0 / np.sqrt(m), nx, axis=1)


def kappa2_from_velocity(c: np.ndarray) -> np.ndarray:
    """Squared slowness m = 1/c^2 (eq. 3.1)."""
    return 1.0 / (c.astype(np.float64) ** 2)


# ----------------------------------------------------------------------------
# absorbing layer, frequency, sources, receivers
# ----------------------------------------------------------------------------
def abl_gamma(nz: int, nx: int, width: int = ABL_WIDTH, gmax: float = GAMMA_MAX,
              sides: str = "lrb") -> np.ndarray:
    """Attenuation fraction gamma(x): 0 in the interior, rising quadratically to
    `gmax` at the outer node of a `width`-cell layer on the listed sides
    ('l','r','b','t'); the top is reflecting by default (sea surface)."""
    i = np.arange(nz)[:, None] * np.ones((1, nx))
    k = np.arange(nx)[None, :] * np.ones((nz, 1))
    d = np.zeros((nz, nx))
    if "l" in sides:
        d = np.maximum(d, width - k)
    if "r" in sides:
        d = np.maximum(d, width - (nx - 1 - k))
    if "b" in sides:
        d = np.maximum(d, width - (nz - 1 - i))
    if "t" in sides:
        d = np.maximum(d, width - i)
    d = np.clip(d, 0, width)
    return gmax * (d / width) ** 2


def omega_for_ppw(c_min: float, ppw: float, h: float = H_DEFAULT) -> float:
    """Angular frequency with `ppw` grid points per minimum wavelength:
    lambda_min = c_min / f = ppw * h."""
    return 2.0 * math.pi * c_min / (ppw * h)


def surface_positions(nx: int, count: int, width: int = ABL_WIDTH) -> np.ndarray:
    """`count` columns evenly spaced over the non-ABL columns [width, nx-width)."""
    span = nx - 2 * width
    return np.array([width + int(round((s + 0.5) * span / count)) for s in range(count)], dtype=np.int64)


def rademacher(nsrc: int, p: int, rng: np.random.Generator) -> np.ndarray:
    """nsrc x p matrix of independent +-1 entries (the simultaneous-source
    encoding draws), float32."""
    return np.where(rng.random((nsrc, p)) < 0.5, -1.0, 1.0).astype(np.float32)


def point_sources(nz: int, nx: int, cols: np.ndarray, row: int = 4, h: float = H_DEFAULT,
                  hz: float | None = None) -> np.ndarray:
    """Grid deltas e_s/(hx*hz) at (row, col) for each col; complex64 [ns][nz][nx]."""
    hz = h if hz is None else hz
    g = np.zeros((len(cols), nz, nx), dtype=np.complex64)
    for s, c in enumerate(cols):
        g[s, row, c] = 1.0 / (h * hz)
    return g


def random_complex(shape, rng: np.random.Generator, dtype=np.complex128) -> np.ndarray:
    """Complex normal CN(0,1): real and imaginary parts i.i.d. N(0, 1/2)."""
    s = math.sqrt(0.5)
    return (rng.standard_normal(shape) * s + 1j * rng.standard_normal(shape) * s).astype(dtype)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
@dataclass
class Medium:
    kappa2: np.ndarray          # float64 [nz][nx]
    gamma: np.ndarray           # float64 [nz][nx]
    omega: float
    h: float = H_DEFAULT
    c_min: float = C_MIN
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        return self.kappa2.shape


def medium_from_velocity(c: np.ndarray, ppw: float = 10.0, h: float = H_DEFAULT,
                         gamma: np.ndarray | None = None, c_min: float | None = None) -> Medium:
    nz, nx = c.shape
    cm = float(c.min()) if c_min is None else c_min
    g = abl_gamma(nz, nx) if gamma is None else gamma
    return Medium(kappa2_from_velocity(c), g, omega_for_ppw(cm, ppw, h), h, cm)


def config1_medium() -> tuple[Medium, np.ndarray]:
    """128x128 GRF medium, one source at (row 4, col 64)."""
    c = velocity_grf(128, 128, rng_for(1, 1))
    med = medium_from_velocity(c)
    src = point_sources(128, 128, np.array([64]), h=med.h)
    return med, src


def config2_medium(nsrc: int = 32, n: int = 256) -> tuple[Medium, np.ndarray]:
    """256x256 layered medium + GRF texture, 32 surface sources."""
    c = velocity_layered(n, n, rng_for(2, 1))
    med = medium_from_velocity(c)
    src = point_sources(n, n, surface_positions(n, nsrc), h=med.h)
    return med, src


def config3_media(nsrc: int = 64, ppws=(5.0, 8.0, 12.0)):
    """One faulted physical model sampled on 256x512, 384x768, 512x1024 grids;
    per grid 3 frequencies at 5/8/12 points per wavelength of that grid."""
    model = faulted_model(rng_for(3, 1))
    out = []
    for nz, nx in ((256, 512), (384, 768), (512, 1024)):
        c = model.sample(nz, nx)
        h = H_DEFAULT * 512.0 / nx     # same physical extent on every grid
        for ppw in ppws:
            med = medium_from_velocity(c, ppw=ppw, h=h)
            src = point_sources(nz, nx, surface_positions(nx, nsrc), h=h)
            out.append((med, src))
    return out


def config4_medium(n: int = 256) -> Medium:
    """Config-2 model perturbed by a 5% GRF update."""
    c = velocity_layered(n, n, rng_for(2, 1))
    c = np.clip(c * (1.0 + 0.05 * grf(n, n, rng_for(4, 1))), C_MIN, C_MAX)
    # keep the frequency of the unperturbed model (same acquisition)
    c0 = velocity_layered(n, n, rng_for(2, 1))
    return medium_from_velocity(c, c_min=float(c0.min()))


FWI_FREQ_RATIOS = (2.6, 2.9, 3.2, 3.5)   # low band of Sec. 5.2, highest scaled to 10 ppw


def config5_media(n: int = 512, nsrc: int = 128, nrec: int = 128):
    """Initial and true media for the FWI gradient, 4 frequencies, sources and
    receivers on row 4 over the non-ABL columns."""
    c0 = velocity_layered(n, n, rng_for(5, 1))
    ct = np.clip(c0 * (1.0 + 0.05 * grf(n, n, rng_for(5, 2))), C_MIN, C_MAX)
    cmin = float(c0.min())
    top = omega_for_ppw(cmin, 10.0)
    omegas = [top * f / FWI_FREQ_RATIOS[-1] for f in FWI_FREQ_RATIOS]
    gamma = abl_gamma(n, n)
    src_cols = surface_positions(n, nsrc)
    rec_cols = surface_positions(n, nrec)
    return dict(kappa2_init=kappa2_from_velocity(c0), kappa2_true=kappa2_from_velocity(ct),
                gamma=gamma, omegas=omegas, h=H_DEFAULT, src_idx=4 * n + src_cols,
                rec_idx=4 * n + rec_cols)
