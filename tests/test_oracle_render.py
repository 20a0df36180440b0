"""Pins of the oracle renderer and pixel likelihood against closed forms,
quadrature, brute force and exact invariants (no GPU)."""
import math

import numpy as np
import pytest
from scipy import integrate, special

from oracle import render

PS = 0.2


def test_hlr_factor_by_quadrature():
    # enclosed fraction of exp(-r) within r = eta, by radial quadrature
    eta = render.ETA_EXP
    inner, _ = integrate.quad(lambda r: r * math.exp(-r), 0.0, eta)
    total, _ = integrate.quad(lambda r: r * math.exp(-r), 0.0, np.inf)
    assert abs(inner / total - 0.5) < 1e-13
    assert abs(eta - 1.6783469900166608) < 1e-14


@pytest.mark.parametrize("k", [0.0, 0.3, 1.1, 2.5])
def test_exponential_ft_against_hankel_quadrature(k):
    # 2-D FT of exp(-r/r0)/(2 pi r0^2) is the Hankel transform 2 pi int r J0(kr) I(r) dr
    r0 = 2.3
    f = lambda r: r * special.j0(k * r) * math.exp(-r / r0) / r0**2
    hank, _ = integrate.quad(f, 0.0, 80 * r0, limit=800, epsabs=1e-15, epsrel=1e-13)
    # oracle spectrum at e=0, dx=dy=0, tiny PSF, with the pixel sinc divided out
    N = 64
    s = r0 * render.ETA_EXP * PS
    T = render.spectrum([1.0, s, 0, 0, 0, 0], N, PS, 1e-9)
    u, _ = render.freq_points(N)
    kk = 2 * np.pi * u / N
    # pick the grid point with ky = 0 closest to k; compare at that exact k
    iu = int(np.argmin(np.abs(kk - k)))
    kx = kk[iu]
    hank, _ = integrate.quad(lambda r: r * special.j0(kx * r) * math.exp(-r / r0) / r0**2,
                             0.0, 80 * r0, limit=800, epsabs=1e-15, epsrel=1e-13)
    iv = int(np.argmin(np.abs(kk)))
    val = T[iv, iu].real / (np.sinc(u[iu] / N) * np.sinc(0.0))
    assert abs(val - hank) < 1e-11
    assert abs(val - (1 + (kx * r0) ** 2) ** -1.5) < 1e-14


def _pixel_gauss_1d(x, c, sig, N, images=3):
    out = np.zeros_like(x)
    for m in range(-images, images + 1):
        a = (x + 0.5 - c + m * N) / (sig * math.sqrt(2))
        b = (x - 0.5 - c + m * N) / (sig * math.sqrt(2))
        out += 0.5 * (special.erf(a) - special.erf(b))
    return out


@pytest.mark.parametrize("N,e1,dx,dy", [(53, 0.3, 0.2, -0.4), (53, -0.5, -1.3, 0.7),
                                        (41, 0.0, 0.0, 0.0), (32, 0.25, 0.5, -0.25)])
def test_gaussian_profile_equals_erf_product(N, e1, dx, dy):
    # Gaussian galaxy (e2 = 0) x Gaussian PSF, pixel-integrated: separable erf product
    F, s, fw = 7.0, 0.5, 0.8
    m = render.render_one([F, s, e1, 0.0, dx, dy], N, PS, fw, render.PROFILE_GAUSS)
    sg = s / PS * render.HLR_TO_SIGMA_GAUSS
    sp = fw / PS * render.FWHM_TO_SIGMA
    sx = math.sqrt(sg * sg * (1 + e1) / (1 - e1) + sp * sp)
    sy = math.sqrt(sg * sg * (1 - e1) / (1 + e1) + sp * sp)
    x = render.pixel_centres(N)
    ref = F * np.outer(_pixel_gauss_1d(x, dy, sy, N), _pixel_gauss_1d(x, dx, sx, N))
    assert np.max(np.abs(m - ref)) < 1e-10 * np.max(ref)


@pytest.mark.parametrize("N", [25, 32, 41, 53])
def test_flux_conservation(N):
    rng = np.random.default_rng(N)
    for _ in range(3):
        p = [rng.uniform(10, 1000), rng.uniform(0.2, 1.2), rng.uniform(-0.5, 0.5),
             rng.uniform(-0.5, 0.5), rng.uniform(-2, 2), rng.uniform(-2, 2)]
        m = render.render_one(p, N, PS, 0.7)
        assert abs(m.sum() - p[0]) < 1e-12 * p[0]


def test_flux_in_stamp_tends_to_one_on_large_stamps():
    # periodic wrap-around shrinks as the stamp grows: flux inside a fixed window
    p = [1.0, 0.6, 0.2, -0.1, 0.0, 0.0]
    inside = []
    for N in (33, 65, 129):
        m = render.render_one(p, N, PS, 0.7)
        c = N // 2
        inside.append(m[c - 12:c + 13, c - 12:c + 13].sum())
    assert abs(inside[2] - inside[1]) < abs(inside[1] - inside[0])
    assert 0.9 < inside[2] < 1.0


@pytest.mark.parametrize("N", [8, 9])
def test_separable_equals_bruteforce(N):
    p = [3.0, 0.4, 0.35, -0.2, 0.3, -0.45]
    a = render.render_one(p, N, PS, 0.7)
    b = render.render_bruteforce(p, N, PS, 0.7)
    assert np.max(np.abs(a - b)) < 1e-14 * max(1.0, np.max(np.abs(a))) * 50


@pytest.mark.parametrize("N", [25, 32])
def test_transpose_and_rotation_symmetries(N):
    F, s, e1, e2, dx, dy = 50.0, 0.5, 0.3, -0.2, 0.4, -0.7
    m = render.render_one([F, s, e1, e2, dx, dy], N, PS, 0.7)
    mt = render.render_one([F, s, -e1, e2, dy, dx], N, PS, 0.7)
    assert np.max(np.abs(m.T - mt)) < 1e-12 * np.max(m)
    mr = render.render_one([F, s, e1, e2, -dx, -dy], N, PS, 0.7)
    assert np.max(np.abs(m[::-1, ::-1] - mr)) < 1e-12 * np.max(m)


def test_ellipticity_axes_by_second_moments():
    N = 65
    x = render.pixel_centres(N)
    X, Y = np.meshgrid(x, x)

    def moments(e1, e2):
        m = render.render_one([1.0, 0.6, e1, e2, 0, 0], N, PS, 0.7)
        return (m * X * X).sum(), (m * Y * Y).sum(), (m * X * Y).sum()

    ixx, iyy, ixy = moments(0.3, 0.0)
    assert ixx > 1.5 * iyy and abs(ixy) < 1e-10
    ixx, iyy, ixy = moments(0.0, 0.3)
    assert ixy > 0.2 * ixx and abs(ixx - iyy) < 1e-10


def test_gaussian_second_moments_closed_form():
    # pixel-integrated Gaussian moments: sigma^2 matrix + PSF + pixel box (1/12)
    N, s, fw, e1, e2 = 81, 0.6, 0.7, 0.2, 0.25
    m = render.render_one([1.0, s, e1, e2, 0, 0], N, PS, fw, render.PROFILE_GAUSS)
    x = render.pixel_centres(N)
    X, Y = np.meshgrid(x, x)
    sg = s / PS * render.HLR_TO_SIGMA_GAUSS
    sp = fw / PS * render.FWHM_TO_SIGMA
    E = e1 * e1 + e2 * e2
    # covariance of the sheared Gaussian: sg^2 * S^2 with S the shear matrix
    S2 = np.array([[1 + E + 2 * e1, 2 * e2], [2 * e2, 1 + E - 2 * e1]]) / (1 - E)
    C = sg * sg * S2 + (sp * sp + 1.0 / 12.0) * np.eye(2)
    got = np.array([[(m * X * X).sum(), (m * X * Y).sum()], [(m * X * Y).sum(), (m * Y * Y).sum()]])
    assert np.max(np.abs(got - C)) < 1e-8 * np.max(C)


@pytest.mark.parametrize("profile", [render.PROFILE_EXP, render.PROFILE_GAUSS])
@pytest.mark.parametrize("N", [25, 32])
def test_gradient_against_central_differences(profile, N):
    rng = np.random.default_rng(7 + N + profile)
    p = np.array([200.0, 0.55, 0.25, -0.3, 0.35, -0.2])
    d = render.render_one(p * [1.1, 0.95, 1, 1, 1, 1] + [0, 0, 0.05, 0.02, 0.1, -0.1],
                          N, PS, 0.7, profile) + rng.normal(0, 1, (N, N))
    ll, g = render.loglik_grad(d, p, N, PS, 0.7, 1.0, profile)
    assert abs(ll - render.loglik(d, p, N, PS, 0.7, 1.0, profile)) < 1e-12 * abs(ll)
    # gradient scale: sqrt of the Fisher information sigma^-2 sum (dm/dp)^2
    _, dT = render.spectrum(p, N, PS, 0.7, profile, derivs=True)
    scale = [math.sqrt(np.sum(render.synthesize(dT[j], N) ** 2)) for j in range(6)]
    f = lambda q: render.loglik(d, q, N, PS, 0.7, 1.0, profile)
    for j in range(6):
        h = 1e-4 * max(1.0, abs(p[j]))
        e = np.zeros(6)
        e[j] = h
        # fourth-order central difference
        fd = (8 * (f(p + e) - f(p - e)) - (f(p + 2 * e) - f(p - 2 * e))) / (12 * h)
        assert abs(fd - g[j]) <= 1e-6 * (abs(g[j]) + scale[j]), (j, fd, g[j], scale[j])


def test_loglik_perfect_model_is_zero():
    p = [100.0, 0.5, 0.1, 0.2, 0.1, 0.1]
    m = render.render_one(p, 25, PS, 0.7)
    assert render.loglik(m, p, 25, PS, 0.7, 1.0) == 0.0
    ll, g = render.loglik_grad(m, p, 25, PS, 0.7, 1.0)
    assert np.all(np.abs(g) < 1e-9)


def test_gradient_central_differences_on_256_parameter_sets():
    """The analytic gradient against plain central differences (relative step
    1e-4) on 256 parameter sets drawn like the 32 x 32 plain-method workload,
    each evaluated on its own noisy stamp at a perturbed position."""
    from workloads import gen
    cfg = gen.CONFIGS["tiny"]
    tr = gen.draw_truth(cfg, n_gal=256, seed=4242)
    rng = np.random.default_rng(4243)
    N = 32
    worst = 0.0
    for i in range(256):
        t = np.array([tr.flux[i], tr.hlr[i], tr.e1[i], tr.e2[i], tr.dx[i], tr.dy[i]])
        d = render.render_one(t, N, PS, tr.psf_fwhm[i]) + rng.normal(0, 1, (N, N))
        p = t * [rng.uniform(0.9, 1.1), rng.uniform(0.9, 1.1), 1, 1, 1, 1] + \
            np.r_[0, 0, rng.uniform(-0.05, 0.05, 2), rng.uniform(-0.2, 0.2, 2)]
        _, g = render.loglik_grad(d, p, N, PS, tr.psf_fwhm[i], 1.0)
        _, dT = render.spectrum(p, N, PS, tr.psf_fwhm[i], derivs=True)
        scale = [math.sqrt(np.sum(render.synthesize(dT[j], N) ** 2)) for j in range(6)]
        f = lambda q: render.loglik(d, q, N, PS, tr.psf_fwhm[i], 1.0)
        for j in range(6):
            h = 1e-4 * max(1.0, abs(p[j]))
            e = np.zeros(6)
            e[j] = h
            fd = (f(p + e) - f(p - e)) / (2 * h)
            err = abs(fd - g[j]) / (abs(g[j]) + scale[j])
            worst = max(worst, err)
            assert err <= 1e-5, (i, j, fd, g[j], scale[j])
    assert worst > 0.0


# ---- Spergel profiles (the paper's Appendix B model-bias fits) -------------

def _spergel_intensity(r, nu, r0=1.0):
    """Unit-flux Spergel surface brightness (Spergel 2010), written out."""
    x = r / r0
    return x ** nu * special.kv(nu, x) / (2 ** nu * special.gamma(nu + 1) * 2 * math.pi * r0 * r0)


@pytest.mark.parametrize("nu", [-0.6, 0.0, 0.5, 1.5, 3.0])
def test_spergel_hlr_factor_by_quadrature(nu):
    # the enclosed flux at eta_nu r0, integrated from the intensity itself, is 1/2
    eta = render.spergel_hlr_factor(nu)
    f = lambda r: 2 * math.pi * r * _spergel_intensity(r, nu)
    inner, _ = integrate.quad(f, 0.0, eta, limit=400, epsabs=1e-14, epsrel=1e-12)
    total, _ = integrate.quad(f, 0.0, np.inf, limit=400, epsabs=1e-14, epsrel=1e-12)
    assert abs(total - 1.0) < 1e-9
    assert abs(inner - 0.5) < 1e-9, (nu, inner)


@pytest.mark.parametrize("nu", [-0.6, 0.0, 1.5, 3.0])
def test_spergel_ft_against_hankel_quadrature(nu):
    # the oracle's G at e = 0 (pixel sinc divided out) against the Hankel
    # transform 2 pi int r J0(k r) I(r) dr of the intensity
    r0 = 1.9
    prof = render.Spergel(nu)
    N = 64
    s = r0 * prof.eta * PS
    T = render.spectrum([1.0, s, 0, 0, 0, 0], N, PS, 1e-9, prof)
    u, _ = render.freq_points(N)
    kk = 2 * np.pi * u / N
    iv = int(np.argmin(np.abs(kk)))
    for kt in (0.0, 0.4, 1.2):
        iu = int(np.argmin(np.abs(kk - kt)))
        kx = kk[iu]
        f = lambda r: 2 * math.pi * r * special.j0(kx * r) * _spergel_intensity(r, nu, r0)
        hank, _ = integrate.quad(f, 0.0, 120 * r0, limit=2000, epsabs=1e-13, epsrel=1e-11)
        val = T[iv, iu].real / np.sinc(u[iu] / N)
        assert abs(val - hank) < 2e-9, (nu, kx, val, hank)


def test_spergel_half_is_the_exponential():
    p = [150.0, 0.45, 0.3, -0.2, 0.4, -0.7]
    for N in (25, 32):
        a = render.render_one(p, N, PS, 0.7)
        b = render.render_one(p, N, PS, 0.7, render.Spergel(0.5))
        assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))
        _, da = render.spectrum(p, N, PS, 0.7, derivs=True)
        _, db = render.spectrum(p, N, PS, 0.7, render.Spergel(0.5), derivs=True)
        assert np.max(np.abs(da - db)) < 1e-11 * np.max(np.abs(da))


@pytest.mark.parametrize("nu", [-0.6, 1.5])
def test_spergel_flux_and_gradient(nu):
    prof = render.Spergel(nu)
    N = 32
    p = np.array([180.0, 0.5, 0.2, -0.25, 0.3, -0.2])
    m = render.render_one(p, N, PS, 0.7, prof)
    assert abs(m.sum() - p[0]) < 1e-11 * p[0]
    rng = np.random.default_rng(31)
    d = render.render_one(p * [1.1, 0.95, 1, 1, 1, 1] + [0, 0, 0.05, 0.02, 0.1, -0.1],
                          N, PS, 0.7, prof) + rng.normal(0, 1, (N, N))
    ll, g = render.loglik_grad(d, p, N, PS, 0.7, 1.0, prof)
    _, dT = render.spectrum(p, N, PS, 0.7, prof, derivs=True)
    scale = [math.sqrt(np.sum(render.synthesize(dT[j], N) ** 2)) for j in range(6)]
    f = lambda q: render.loglik(d, q, N, PS, 0.7, 1.0, prof)
    for j in range(6):
        h = 1e-4 * max(1.0, abs(p[j]))
        e = np.zeros(6)
        e[j] = h
        fd = (8 * (f(p + e) - f(p - e)) - (f(p + 2 * e) - f(p - 2 * e))) / (12 * h)
        assert abs(fd - g[j]) <= 1e-6 * (abs(g[j]) + scale[j]), (nu, j, fd, g[j])
