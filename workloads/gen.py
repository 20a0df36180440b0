"""Seeded draws of synthetic LSST-like galaxy populations.

The paper's dataset (Section 2: 320k GalSim stamps) is not available, so every
input is synthetic.  Five workloads are defined, each by its sizes and the
distributions it draws from:

  tiny      16 galaxies, 32x32 stamps, PSF FWHM 0.7", SNR 15-100, 1 chain,
            10 leapfrog steps, fixed step 0.005, 100 burn-in + 500 draws,
            41x41 shear grid on [-0.25, 0.25]^2
  uniform   10,000 galaxies, 53x53 stamps, PSF FWHM 0.7", SNR 15-100, 4 chains,
            20 leapfrog steps, 300 dual-averaging warmup + 1,000 draws
  uneven    100,000 galaxies, stamp side from {25, 41, 53, 73, 101} chosen
            by a flux-containment rule, PSF FWHM ~ U(0.6", 0.9"), SNR 10-200
  diff      10,000 galaxies x 1,000 interim samples for the shear-level
            sampler over (g1, g2, mu_ln_s, sigma_ln_s, sigma_e)
  serving   Poisson arrivals at 2,000/s, sizes {25,41,53,73,101} with
            weights 0.3/0.3/0.2/0.15/0.05, 300 effective samples each

Common population (all workloads): ln hlr ~ N(ln 0.6", 0.3); intrinsic
(e1, e2) ~ N(0, 0.2^2) per component, rejection-truncated to |e| < 0.7;
centroid offsets dx, dy ~ U(-0.5, 0.5) px; ln F ~ N(mu, sd) with its 2.5 %
and 97.5 % points at the fluxes giving the SNR range for the median galaxy
(hlr 0.6", FWHM 0.7", 0.2"/px), using SNR = ||m||_2 / sigma (Section 2
footnote); pixel noise N(0, 1); applied shear g = (0.02, 0).  The caller
applies the shear to the intrinsic ellipticities with its own implementation
of the shear response.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SIZE_CLASSES = (25, 41, 53, 73, 101)
PIXEL_SCALE = 0.2

# ||m||_2 of a unit-flux exponential, hlr 0.6", Gaussian PSF FWHM 0.7",
# 0.2"/px, centred on a 53x53 stamp.  Written by tests/golden/make_golden.py
# (oracle renderer); tests/test_workloads.py checks it against the oracle.
UNIT_FLUX_NORM_MEDIAN = 0.09093264107520191

# Radius enclosing 99.5 % of an exponential profile's flux, in scale radii
# (root of (1 + x) exp(-x) = 0.005); used only to choose stamp sizes.
def _r995() -> float:
    x = 7.0
    for _ in range(60):
        x -= ((1.0 + x) * math.exp(-x) - 0.005) / (-x * math.exp(-x))
    return x


R995_OVER_R0 = _r995()
HLR_OVER_R0 = 1.6783469900166608   # exponential half-light radius in scale radii


def data_seed(k: int) -> int:
    return 220480 + k


def chain_seed(k: int) -> int:
    return 221480 + k


@dataclass
class Workload:
    name: str
    index: int
    n_gal: int
    n_pix: int | None            # None: per-galaxy sizes from the size rule
    psf_fwhm: float | tuple      # scalar or (lo, hi) uniform range
    snr: tuple
    chains: int
    leapfrog: int
    warmup: int
    samples: int
    step_size: float = 0.01
    adapt: bool = True
    g_true: tuple = (0.02, 0.0)
    sigma: float = 1.0
    extra: dict = field(default_factory=dict)


CONFIGS = {
    "tiny": Workload("tiny", 0, 16, 32, 0.7, (15.0, 100.0), 1, 10, 100, 500, step_size=0.005,
                     adapt=False, extra=dict(grid_lo=-0.25, grid_hi=0.25, grid_n=41)),
    "uniform": Workload("uniform", 1, 10_000, 53, 0.7, (15.0, 100.0), 4, 20, 300, 1000),
    "uneven": Workload("uneven", 2, 100_000, None, (0.6, 0.9), (10.0, 200.0), 4, 20, 300, 1000),
    "diff": Workload("diff", 3, 10_000, 53, 0.7, (15.0, 100.0), 4, 20, 300, 1000,
                     extra=dict(K=1000, shear_warmup=500, shear_samples=3000, shear_leapfrog=10,
                                fd_sets=256, fd_step=1e-4)),
    "serving": Workload("serving", 4, 1_000_000, None, (0.6, 0.9), (10.0, 200.0), 1, 20, 300, 0,
                        extra=dict(rate=2000.0, size_weights=(0.3, 0.3, 0.2, 0.15, 0.05),
                                   target_ess=300.0)),
}


@dataclass
class Truth:
    """True intrinsic properties; ellipticities are pre-shear."""
    flux: np.ndarray
    hlr: np.ndarray         # arcsec
    e1: np.ndarray
    e2: np.ndarray
    dx: np.ndarray          # pixels from the stamp centre
    dy: np.ndarray
    psf_fwhm: np.ndarray    # arcsec
    n_pix: np.ndarray       # stamp side per galaxy
    sigma: np.ndarray
    g: tuple

    def __len__(self):
        return self.flux.shape[0]


def flux_lognormal(snr_lo, snr_hi, sigma=1.0):
    """(mu, sd) of ln F with the SNR range at its 2.5 % / 97.5 % points."""
    f_lo = snr_lo * sigma / UNIT_FLUX_NORM_MEDIAN
    f_hi = snr_hi * sigma / UNIT_FLUX_NORM_MEDIAN
    mu = 0.5 * (math.log(f_lo) + math.log(f_hi))
    sd = (math.log(f_hi) - math.log(f_lo)) / (2.0 * 1.959963984540054)
    return mu, sd


def stamp_size_rule(hlr, e, psf_fwhm, sizes=SIZE_CLASSES, pixel_scale=PIXEL_SCALE):
    """Smallest side from ``sizes`` whose half-width covers the 99.5 % flux
    radius of the major axis (stretched by sqrt((1+|e|)/(1-|e|))), added in
    quadrature to three PSF sigmas."""
    r0 = np.asarray(hlr) / pixel_scale / HLR_OVER_R0
    stretch = np.sqrt((1.0 + np.abs(e)) / (1.0 - np.abs(e)))
    sp = np.asarray(psf_fwhm) / pixel_scale / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    R = np.sqrt((R995_OVER_R0 * r0 * stretch) ** 2 + (3.0 * sp) ** 2)
    out = np.full(np.shape(R), sizes[-1], dtype=np.int32)
    for s in sorted(sizes, reverse=True):
        out[2.0 * R <= s] = s
    return out


def _truncated_ellipticity(rng, n, sd=0.2, e_max=0.7):
    e1 = np.empty(n)
    e2 = np.empty(n)
    filled = 0
    while filled < n:
        m = 2 * (n - filled) + 16
        a = rng.normal(0.0, sd, m)
        b = rng.normal(0.0, sd, m)
        ok = a * a + b * b < e_max * e_max
        a, b = a[ok], b[ok]
        take = min(n - filled, a.shape[0])
        e1[filled:filled + take] = a[:take]
        e2[filled:filled + take] = b[:take]
        filled += take
    return e1, e2


def draw_truth(cfg: Workload, n_gal: int | None = None, seed: int | None = None,
               size_override=None) -> Truth:
    n = cfg.n_gal if n_gal is None else n_gal
    rng = np.random.default_rng(data_seed(cfg.index) if seed is None else seed)
    hlr = np.exp(rng.normal(math.log(0.6), 0.3, n))
    e1, e2 = _truncated_ellipticity(rng, n)
    dx = rng.uniform(-0.5, 0.5, n)
    dy = rng.uniform(-0.5, 0.5, n)
    mu, sd = flux_lognormal(*cfg.snr, sigma=cfg.sigma)
    flux = np.exp(rng.normal(mu, sd, n))
    if isinstance(cfg.psf_fwhm, tuple):
        psf = rng.uniform(cfg.psf_fwhm[0], cfg.psf_fwhm[1], n)
    else:
        psf = np.full(n, float(cfg.psf_fwhm))
    if size_override is not None:
        npix = np.asarray(size_override, dtype=np.int32)
    elif cfg.n_pix is not None:
        npix = np.full(n, cfg.n_pix, dtype=np.int32)
    elif "size_weights" in cfg.extra:
        npix = rng.choice(np.array(SIZE_CLASSES, dtype=np.int32), size=n,
                          p=np.array(cfg.extra["size_weights"]))
    else:
        npix = stamp_size_rule(hlr, np.hypot(e1, e2), psf)
    return Truth(flux=flux, hlr=hlr, e1=e1, e2=e2, dx=dx, dy=dy, psf_fwhm=psf, n_pix=npix,
                 sigma=np.full(n, cfg.sigma), g=cfg.g_true)


def draw_noise(truth: Truth, seed: int, dtype=np.float32):
    """Packed noise for all stamps (row-major [y][x], galaxies back to back)."""
    rng = np.random.default_rng(seed)
    sizes = truth.n_pix.astype(np.int64) ** 2
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    total = int(sizes.sum())
    noise = rng.standard_normal(total, dtype=np.float64) * np.repeat(truth.sigma, sizes)
    return noise.astype(dtype), off


def draw_interim_samples(n_gal: int, K: int, seed: int, g=(0.02, 0.0), noise_e=0.05, noise_ln_s=0.05):
    """Stand-in interim samples for the shear phase: per galaxy an intrinsic
    ellipticity of the population (truncated Gaussian), sheared by g with the
    reduced-shear map, and a lognormal size; its K samples scatter around them
    (e' kept inside |e'| < 0.95).  Returns float32 (e1', e2', log10 s), each
    [n_gal, K]."""
    rng = np.random.default_rng(seed)
    e1, e2 = _truncated_ellipticity(rng, n_gal)
    e = e1 + 1j * e2
    gg = complex(*g)
    ep = (e + gg) / (1.0 + np.conj(gg) * e)
    ln_s = rng.normal(np.log(0.6), 0.3, n_gal)
    smp = ep[:, None] + rng.normal(0, noise_e, (n_gal, K)) + 1j * rng.normal(0, noise_e, (n_gal, K))
    r = np.abs(smp)
    smp = np.where(r < 0.95, smp, smp * 0.9 / np.maximum(r, 1e-12))
    l10s = (ln_s[:, None] + rng.normal(0, noise_ln_s, (n_gal, K))) / np.log(10.0)
    return [a.astype(np.float32) for a in (smp.real, smp.imag, l10s)]


def draw_requests(n_req: int, rate: float, seed: int):
    """Poisson arrival times (seconds) of n_req requests."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n_req))


def bootstrap_indices(n_boot: int, n_gal: int, seed: int):
    """Galaxy indices of n_boot bootstrap resamples, each n_gal draws with
    replacement: int64 [n_boot, n_gal]."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, n_gal, (n_boot, n_gal))


def bootstrap_counts(n_boot: int, n_gal: int, seed: int):
    """Times each galaxy is drawn in each resample of bootstrap_indices:
    int32 [n_boot, n_gal]."""
    idx = bootstrap_indices(n_boot, n_gal, seed)
    out = np.zeros((n_boot, n_gal), np.int32)
    for b in range(n_boot):
        out[b] = np.bincount(idx[b], minlength=n_gal)
    return out


def noise_kernel_ps(rng, N):
    """DFT-mode noise powers |DFT kappa|^2 (FFT order) of a random positive 3 x 3
    correlation kernel kappa wrapped on the N grid (centre 1, the others in
    [0, 0.1], normalised to unit pixel variance); and kappa itself."""
    kap = np.zeros((N, N))
    w = rng.uniform(0.0, 0.1, (3, 3))
    w[1, 1] = 1.0
    for a in range(3):
        for b in range(3):
            kap[(a - 1) % N, (b - 1) % N] = w[a, b]
    kap /= math.sqrt(np.sum(kap * kap))
    return np.abs(np.fft.fft2(kap)) ** 2, kap


def correlated_noise(rng, kap, sigma, n=None):
    """sigma times the circular convolution of white noise with kappa: one
    N x N field, or n of them ([n, N, N])."""
    N = kap.shape[0]
    shape = (N, N) if n is None else (n, N, N)
    wn = rng.standard_normal(shape)
    return sigma * np.real(np.fft.ifft2(np.fft.fft2(wn) * np.fft.fft2(kap)))
