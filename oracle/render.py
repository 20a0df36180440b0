"""Oracle stamp renderer, pixel likelihood and gradient (float64, dense).

Test infrastructure only (see ``oracle/__init__``).

Model (Section 2 and Section 3.2 of the paper): an exponential (Sersic n=1)
galaxy with flux ``F`` and half-light radius ``s`` (arcsec), sheared by the
area-preserving ellipticity ``(e1, e2)`` in the reduced-shear convention of
eq. ellip-phi-transform, offset by ``(dx, dy)`` pixels from the stamp centre,
convolved with a Gaussian PSF of given FWHM and integrated over square
pixels.  The paper renders with JAX-GalSim and does not describe the drawing
method; the definition used here is the truncated Fourier series on the
stamp's own frequency grid:

    m[j, i] = N^-2 sum_{u,v} w_u w_v T(u, v) exp(i (k_u x_i + k_v y_j))

with k_u = 2 pi u / N, pixel centres x_i = i - (N-1)/2, y_j = j - (N-1)/2,
u, v over -floor(N/2) .. floor(N/2) and weights w = 1, except w = 1/2 at
u = +-N/2 when N is even (the symmetric treatment of the Nyquist
frequency, which makes m exactly real).  The spectrum is

    T = F * G(q) * exp(-sigma_psf^2 |k|^2 / 2) * sinc(u/N) sinc(v/N)
          * exp(-i (k_x dx + k_y dy))
    q = [(1+E) |k|^2 + 2 e1 (k_x^2 - k_y^2) + 4 e2 k_x k_y] / (1 - E),
    E = e1^2 + e2^2,

G(q) = (1 + r0^2 q)^(-3/2) for the exponential profile (its 2-D Fourier
transform) and G(q) = exp(-sigma_g^2 q / 2) for the Gaussian test profile.

Appendix B of the paper also fits Spergel profiles of fixed index nu (the
model-bias study).  A Spergel profile (Spergel 2010) has the surface
brightness I(r) = F / (2 pi r0^2) (r/r0)^nu K_nu(r/r0) / (2^nu Gamma(nu + 1))
(K_nu the modified Bessel function of the second kind) and the unit-flux
Fourier transform (1 + k^2 r0^2)^(-(1 + nu)), so G(q) = (1 + r0^2 q)^(-(1+nu));
nu = 1/2 is the exponential profile.  Its half-light radius is eta_nu r0,
eta_nu the root of x^(nu+1) K_(nu+1)(x) = 2^(nu-1) Gamma(nu + 1) (the
enclosed flux 1 - x^(nu+1) K_(nu+1)(x) / (2^nu Gamma(nu + 1)) equal to 1/2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

# Half-light radius of exp(-r/r0) in units of r0: the root of
# (1 + eta) exp(-eta) = 1/2 (enclosed-flux fraction of an exponential disk).
def exponential_hlr_factor() -> float:
    eta = 1.7
    for _ in range(60):
        f = (1.0 + eta) * np.exp(-eta) - 0.5
        df = -eta * np.exp(-eta)
        eta -= f / df
    return float(eta)


ETA_EXP = exponential_hlr_factor()
FWHM_TO_SIGMA = 1.0 / (2.0 * np.sqrt(2.0 * np.log(2.0)))
HLR_TO_SIGMA_GAUSS = 1.0 / np.sqrt(2.0 * np.log(2.0))

PROFILE_EXP = 0
PROFILE_GAUSS = 1
PROFILE_SPERGEL = 2


def spergel_hlr_factor(nu: float) -> float:
    """eta_nu = half-light radius / r0 of the Spergel profile of index nu:
    the root of x^(nu+1) K_(nu+1)(x) = 2^(nu-1) Gamma(nu+1), by bisection."""
    from scipy.special import gamma, kv
    target = 2.0 ** (nu - 1.0) * gamma(nu + 1.0)
    f = lambda x: x ** (nu + 1.0) * kv(nu + 1.0, x) - target     # decreasing in x
    lo, hi = 1e-8, 1.0
    while f(hi) > 0.0:
        hi *= 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


class Spergel:
    """Spergel profile of fixed index nu (pass as ``profile``)."""

    def __init__(self, nu: float):
        self.nu = float(nu)
        self.eta = spergel_hlr_factor(self.nu)


def _kind(profile) -> int:
    return PROFILE_SPERGEL if isinstance(profile, Spergel) else int(profile)


def freq_points(N: int):
    """Integer frequencies u and their weights w_u for an N-pixel axis."""
    h = N // 2
    u = np.arange(-h, h + 1)   # N points for odd N, N + 1 for even N
    w = np.ones(u.shape, dtype=np.float64)
    if N % 2 == 0:
        w[0] = 0.5
        w[-1] = 0.5
    return u.astype(np.float64), w


def pixel_centres(N: int) -> np.ndarray:
    return np.arange(N, dtype=np.float64) - (N - 1) / 2.0


def scales(s_arcsec, psf_fwhm_arcsec, pixel_scale, profile=PROFILE_EXP):
    """Profile scale (pixels) and PSF sigma (pixels)."""
    s_pix = np.asarray(s_arcsec, dtype=np.float64) / pixel_scale
    kind = _kind(profile)
    if kind == PROFILE_SPERGEL:
        r = s_pix / profile.eta        # Spergel scale radius r0
    elif kind == PROFILE_EXP:
        r = s_pix / ETA_EXP            # exponential scale radius r0
    else:
        r = s_pix * HLR_TO_SIGMA_GAUSS  # Gaussian sigma
    sig_psf = np.asarray(psf_fwhm_arcsec, dtype=np.float64) * FWHM_TO_SIGMA / pixel_scale
    return r, sig_psf


def _grid(N):
    u, w = freq_points(N)
    k = 2.0 * np.pi * u / N
    KX = k[None, :]      # columns: x frequency
    KY = k[:, None]      # rows: y frequency
    WW = w[:, None] * w[None, :]
    SINC = np.sinc(u / N)[:, None] * np.sinc(u / N)[None, :]
    return u, k, KX, KY, WW, SINC


def quad_form(KX, KY, e1, e2):
    E = e1 * e1 + e2 * e2
    K = KX * KX + KY * KY
    D = KX * KX - KY * KY
    P = KX * KY
    return ((1.0 + E) * K + 2.0 * e1 * D + 4.0 * e2 * P) / (1.0 - E)


def spectrum(params, N, pixel_scale, psf_fwhm, profile=PROFILE_EXP, derivs=False):
    """T(u, v) for one galaxy on the (n_u x n_u) frequency-point grid.

    params = (F, s_arcsec, e1, e2, dx_px, dy_px).  Rows index v (y), columns u (x).
    If derivs, also return dT/dparams as a (6, n_u, n_u) complex array.
    """
    F, s, e1, e2, dx, dy = [float(v) for v in params]
    _, _, KX, KY, _, SINC = _grid(N)
    r, sp = scales(s, psf_fwhm, pixel_scale, profile)
    E = e1 * e1 + e2 * e2
    q = quad_form(KX, KY, e1, e2)
    kind = _kind(profile)
    if kind == PROFILE_SPERGEL:
        a = 1.0 + r * r * q
        G = a ** -(1.0 + profile.nu)
    elif kind == PROFILE_EXP:
        a = 1.0 + r * r * q
        G = a ** -1.5
    else:
        G = np.exp(-0.5 * r * r * q)
    psf = np.exp(-0.5 * sp * sp * (KX * KX + KY * KY))
    phase = np.exp(-1j * (KX * dx + KY * dy))
    T = F * G * psf * SINC * phase
    if not derivs:
        return T
    K = KX * KX + KY * KY
    D = KX * KX - KY * KY
    P = KX * KY
    dq_de1 = (2.0 * e1 * K + 2.0 * D + 2.0 * e1 * q) / (1.0 - E)
    dq_de2 = (2.0 * e2 * K + 4.0 * P + 2.0 * e2 * q) / (1.0 - E)
    if kind == PROFILE_SPERGEL:
        dlnG_dq = -(1.0 + profile.nu) * r * r / a
        dlnG_ds = -2.0 * (1.0 + profile.nu) * r * r * q / (s * a)
    elif kind == PROFILE_EXP:
        dlnG_dq = -1.5 * r * r / a
        dlnG_ds = -3.0 * r * r * q / (s * a)
    else:
        dlnG_dq = -0.5 * r * r * np.ones_like(q)
        dlnG_ds = -r * r * q / s
    dT = np.empty((6,) + T.shape, dtype=np.complex128)
    dT[0] = T / F
    dT[1] = dlnG_ds * T
    dT[2] = dlnG_dq * dq_de1 * T
    dT[3] = dlnG_dq * dq_de2 * T
    dT[4] = -1j * KX * T
    dT[5] = -1j * KY * T
    return T, dT


def synthesis_matrix(N):
    """W[i, u] = w_u exp(i k_u x_i): maps frequency points to pixel centres."""
    u, w = freq_points(N)
    k = 2.0 * np.pi * u / N
    x = pixel_centres(N)
    return w[None, :] * np.exp(1j * x[:, None] * k[None, :])


def synthesize(T, N):
    """Pixel image N^-2 Re(W_y T W_x^T) of a spectrum on the frequency-point grid."""
    W = synthesis_matrix(N)
    return np.real(W @ T @ W.T) / (N * N)


def render_one(params, N, pixel_scale, psf_fwhm, profile=PROFILE_EXP):
    return synthesize(spectrum(params, N, pixel_scale, psf_fwhm, profile), N)


def render(params, N, pixel_scale, psf_fwhm, profile=PROFILE_EXP):
    """Stamps for a batch: params (G, 6), psf_fwhm scalar or (G,). Returns (G, N, N)."""
    params = np.atleast_2d(np.asarray(params, dtype=np.float64))
    psf = np.broadcast_to(np.asarray(psf_fwhm, dtype=np.float64), (params.shape[0],))
    return np.stack([render_one(p, N, pixel_scale, f, profile) for p, f in zip(params, psf)])


def render_bruteforce(params, N, pixel_scale, psf_fwhm, profile=PROFILE_EXP):
    """O(N^4) double sum of the Fourier series, pixel by pixel (small N only)."""
    T = spectrum(params, N, pixel_scale, psf_fwhm, profile)
    u, w = freq_points(N)
    k = 2.0 * np.pi * u / N
    x = pixel_centres(N)
    m = np.zeros((N, N))
    for j in range(N):
        for i in range(N):
            acc = 0.0 + 0.0j
            for iv in range(len(u)):
                for iu in range(len(u)):
                    acc += w[iv] * w[iu] * T[iv, iu] * np.exp(1j * (k[iu] * x[i] + k[iv] * x[j]))
            m[j, i] = acc.real / (N * N)
    return m


def loglik(data, params, N, pixel_scale, psf_fwhm, sigma, profile=PROFILE_EXP):
    """eq. likelihood-pixels with b = sigma^2 and the constant C = 0."""
    m = render_one(params, N, pixel_scale, psf_fwhm, profile)
    r = np.asarray(data, dtype=np.float64) - m
    return -0.5 * float(np.sum(r * r)) / (sigma * sigma)


def loglik_grad(data, params, N, pixel_scale, psf_fwhm, sigma, profile=PROFILE_EXP):
    """log L and d log L / d(F, s, e1, e2, dx, dy) by forward mode.

    Each stamp derivative dm/dp is synthesized from dT/dp, then
    d log L/dp = sigma^-2 sum_pixels (d - m) dm/dp.
    """
    T, dT = spectrum(params, N, pixel_scale, psf_fwhm, profile, derivs=True)
    m = synthesize(T, N)
    r = np.asarray(data, dtype=np.float64) - m
    ll = -0.5 * float(np.sum(r * r)) / (sigma * sigma)
    g = np.array([np.sum(r * synthesize(dT[j], N)) for j in range(6)]) / (sigma * sigma)
    return ll, g


def loglik_grad_batch(data, params, N, pixel_scale, psf_fwhm, sigma, profile=PROFILE_EXP):
    G = params.shape[0]
    psf = np.broadcast_to(np.asarray(psf_fwhm, dtype=np.float64), (G,))
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (G,))
    ll = np.empty(G)
    gr = np.empty((G, 6))
    for n in range(G):
        ll[n], gr[n] = loglik_grad(data[n], params[n], N, pixel_scale, psf[n], sig[n], profile)
    return ll, gr


# ---- Appendix C: correlated noise and several exposures ----------------------
#
# Stationary noise on the stamp (periodic, as the stamp's own DFT grid assumes)
# has a circulant covariance Sigma[x, x'] = sigma^2 c(x - x' mod N); its
# eigenvalues are sigma^2 lambda_k with lambda_k = sum_x c(x) exp(-i k.x), the
# noise power of DFT mode k.  ``noise_ps`` holds lambda on the N x N DFT grid
# in FFT order (row v, column u, indices 0..N-1, numpy.fft layout); all ones
# is white noise.  The likelihood of eq. covar-pixel-likelihood is evaluated
# here by forming Sigma explicitly and solving with it.

def covariance_matrix(noise_ps, sigma):
    """Sigma (N^2 x N^2, pixels row-major) of stationary noise with the DFT-mode
    powers noise_ps (N x N, FFT order) times sigma^2."""
    ps = np.asarray(noise_ps, dtype=np.float64)
    N = ps.shape[0]
    c = np.real(np.fft.ifft2(ps))                     # c(dy, dx), lags mod N
    iy, ix = np.divmod(np.arange(N * N), N)
    dy = (iy[:, None] - iy[None, :]) % N
    dx = (ix[:, None] - ix[None, :]) % N
    return sigma * sigma * c[dy, dx]


_COV_FACTORS: dict = {}


def _cov_factor(noise_ps, sigma):
    """Cholesky factor of covariance_matrix(noise_ps, sigma) (symmetric
    positive definite), kept for the last few (noise_ps, sigma) pairs so that
    a chain's evaluations factor each exposure's N^2 x N^2 matrix once."""
    ps = np.ascontiguousarray(noise_ps, dtype=np.float64)
    key = (ps.shape, ps.tobytes(), float(sigma))
    f = _COV_FACTORS.get(key)
    if f is None:
        if len(_COV_FACTORS) >= 4:
            _COV_FACTORS.pop(next(iter(_COV_FACTORS)))
        f = scipy.linalg.cho_factor(covariance_matrix(ps, sigma), lower=True)
        _COV_FACTORS[key] = f
    return f


def cov_solve(noise_ps, sigma, r):
    """Sigma^-1 r with the explicit covariance (a Cholesky solve)."""
    return scipy.linalg.cho_solve(_cov_factor(noise_ps, sigma), r)


def loglik_grad_cov(data, params, N, pixel_scale, psf_fwhm, sigma, noise_ps, profile=PROFILE_EXP):
    """eq. covar-pixel-likelihood (C = 0) and its gradient by forward mode:
    d log L / dp = (dm/dp)^T Sigma^-1 (d - m)."""
    T, dT = spectrum(params, N, pixel_scale, psf_fwhm, profile, derivs=True)
    r = (np.asarray(data, dtype=np.float64) - synthesize(T, N)).ravel()
    y = cov_solve(noise_ps, sigma, r)
    ll = -0.5 * float(r @ y)
    g = np.array([synthesize(dT[j], N).ravel() @ y for j in range(6)])
    return ll, g


def loglik_grad_exposures(datas, params, N, pixel_scale, psfs, sigmas, noise_pss=None,
                          profile=PROFILE_EXP):
    """Several independent exposures of one galaxy (Appendix C): the same
    parameters, each exposure its own PSF, noise level and noise power; log L
    and its gradient are sums over the exposures."""
    ll, g = 0.0, np.zeros(6)
    for j in range(len(datas)):
        ps = np.ones((N, N)) if noise_pss is None else noise_pss[j]
        lj, gj = loglik_grad_cov(datas[j], params, N, pixel_scale, psfs[j], sigmas[j], ps, profile)
        ll += lj
        g += gj
    return ll, g


def fisher_diag_exposures(params, N, pixel_scale, psfs, sigmas, noise_pss=None, profile=PROFILE_EXP):
    """Diagonal of sum_j (dm_j/dp)^T Sigma_j^-1 (dm_j/dp) (physical parameters)."""
    f = np.zeros(6)
    for j in range(len(psfs)):
        ps = np.ones((N, N)) if noise_pss is None else noise_pss[j]
        _, dT = spectrum(params, N, pixel_scale, psfs[j], profile, derivs=True)
        for i in range(6):
            dm = synthesize(dT[i], N).ravel()
            f[i] += dm @ cov_solve(ps, sigmas[j], dm)
    return f
