"""Pins of the Appendix C likelihood extensions in the oracle (stationary
correlated noise, several exposures) against closed forms and limits."""
import math

import numpy as np

from oracle import hmc, render

PS = 0.2


def _kernel_noise_ps(N, rng):
    """A small positive convolution kernel kappa (wrapped on the N grid) and the
    DFT-mode powers |DFT kappa|^2 of the noise it correlates."""
    kap = np.zeros((N, N))
    w = rng.uniform(0.2, 1.0, (3, 3))
    for a in range(3):
        for b in range(3):
            kap[(a - 1) % N, (b - 1) % N] = w[a, b]
    kap[0, 0] += 2.0                      # well conditioned
    return kap, np.abs(np.fft.fft2(kap)) ** 2


def test_white_noise_power_is_the_pixel_likelihood():
    rng = np.random.default_rng(1)
    N = 16
    p = np.array([300.0, 0.5, 0.2, -0.1, 0.3, -0.4])
    d = render.render_one(p * [1.05, 0.9, 1, 1, 1, 1], N, PS, 0.7) + rng.normal(0, 1.3, (N, N))
    a = render.loglik_grad(d, p, N, PS, 0.7, 1.3)
    b = render.loglik_grad_cov(d, p, N, PS, 0.7, 1.3, np.ones((N, N)))
    assert abs(a[0] - b[0]) < 1e-10 * abs(a[0])
    assert np.max(np.abs(a[1] - b[1])) < 1e-9 * np.max(np.abs(a[1]))


def test_covariance_of_convolved_white_noise():
    # noise n = K w (K the circular convolution by kappa, w white): Sigma = sigma^2 K K^T
    # and r^T Sigma^-1 r = |K^-1 r|^2 / sigma^2
    rng = np.random.default_rng(2)
    N, sig = 12, 0.8
    kap, ps = _kernel_noise_ps(N, rng)
    K = np.zeros((N * N, N * N))
    for y in range(N):
        for x in range(N):
            for yy in range(N):
                for xx in range(N):
                    K[y * N + x, yy * N + xx] = kap[(y - yy) % N, (x - xx) % N]
    S = render.covariance_matrix(ps, sig)
    assert np.max(np.abs(S - sig * sig * K @ K.T)) < 1e-10 * np.max(np.abs(S))
    p = np.array([200.0, 0.4, -0.2, 0.15, -0.3, 0.2])
    d = render.render_one(p, N, PS, 0.7) + sig * (K @ rng.normal(0, 1, N * N)).reshape(N, N)
    q = p * [0.95, 1.1, 1, 1, 1, 1] + [0, 0, 0.03, -0.02, 0.1, 0.05]
    r = (d - render.render_one(q, N, PS, 0.7)).ravel()
    want = -0.5 * float(np.sum(np.linalg.solve(K, r) ** 2)) / (sig * sig)
    ll, _ = render.loglik_grad_cov(d, q, N, PS, 0.7, sig, ps)
    assert abs(ll - want) < 1e-9 * abs(want)


def test_identical_exposures_add():
    rng = np.random.default_rng(3)
    N = 14
    p = np.array([250.0, 0.45, 0.1, 0.25, -0.2, 0.1])
    _, ps = _kernel_noise_ps(N, rng)
    d = render.render_one(p, N, PS, 0.8) + rng.normal(0, 1, (N, N))
    q = p * [1.1, 0.9, 1, 1, 1, 1]
    one = render.loglik_grad_cov(d, q, N, PS, 0.8, 0.9, ps)
    three = render.loglik_grad_exposures([d, d, d], q, N, PS, [0.8] * 3, [0.9] * 3, [ps] * 3)
    assert abs(three[0] - 3 * one[0]) < 1e-10 * abs(three[0])
    assert np.max(np.abs(three[1] - 3 * one[1])) < 1e-9 * np.max(np.abs(three[1]))


def test_exposures_gradient_against_central_differences():
    rng = np.random.default_rng(4)
    N = 16
    p = np.array([280.0, 0.5, 0.2, -0.15, 0.25, -0.3])
    psfs, sigs = [0.65, 0.85], [1.0, 1.4]
    pss = [_kernel_noise_ps(N, rng)[1], np.ones((N, N))]
    datas = [render.render_one(p * [1.1, 0.95, 1, 1, 1, 1], N, PS, f) + rng.normal(0, s, (N, N))
             for f, s in zip(psfs, sigs)]
    ll, g = render.loglik_grad_exposures(datas, p, N, PS, psfs, sigs, pss)
    f = lambda q: render.loglik_grad_exposures(datas, q, N, PS, psfs, sigs, pss)[0]
    for j in range(6):
        h = 1e-4 * max(1.0, abs(p[j]))
        e = np.zeros(6)
        e[j] = h
        fd = (8 * (f(p + e) - f(p - e)) - (f(p + 2 * e) - f(p - 2 * e))) / (12 * h)
        assert abs(fd - g[j]) <= 1e-6 * (abs(g[j]) + 1.0), (j, fd, g[j])


def test_exposure_fisher_is_curvature_at_the_model():
    # with data equal to the model, -d2 log L / dp_j^2 = (dm/dp_j)^T Sigma^-1 dm/dp_j
    rng = np.random.default_rng(5)
    N = 14
    p = np.array([260.0, 0.5, 0.15, 0.1, 0.2, -0.1])
    psfs, sigs = [0.7, 0.9], [1.0, 0.7]
    pss = [_kernel_noise_ps(N, rng)[1], _kernel_noise_ps(N, rng)[1]]
    datas = [render.render_one(p, N, PS, f) for f in psfs]
    fi = render.fisher_diag_exposures(p, N, PS, psfs, sigs, pss)
    for j in range(6):
        h = 1e-4 * max(1.0, abs(p[j]))
        e = np.zeros(6)
        e[j] = h
        gp = render.loglik_grad_exposures(datas, p + e, N, PS, psfs, sigs, pss)[1][j]
        gm = render.loglik_grad_exposures(datas, p - e, N, PS, psfs, sigs, pss)[1][j]
        assert abs(-(gp - gm) / (2 * h) - fi[j]) < 1e-5 * fi[j], (j, -(gp - gm) / (2 * h), fi[j])


def test_exposures_potential_matches_single_stamp_form():
    # one white-noise exposure: the Exposures potential is the single-stamp one
    rng = np.random.default_rng(6)
    N = 16
    p = np.array([300.0, 0.5, 0.2, -0.1, 0.3, -0.4])
    d = render.render_one(p, N, PS, 0.7) + rng.normal(0, 1, (N, N))
    g1 = hmc.Galaxy(data=d, N=N, pixel_scale=PS, psf_fwhm=0.7, sigma=1.0, ref_xy=(0.2, -0.3))
    g2 = hmc.Exposures(datas=[d], N=N, pixel_scale=PS, psf_fwhm=[0.7], sigma=[1.0], ref_xy=(0.2, -0.3))
    th = np.array([math.log10(290.0), math.log10(0.52), 0.18, -0.08, 0.1, -0.1])
    U1, gU1 = hmc.potential(g1, th)
    U2, gU2 = hmc.potential(g2, th)
    assert abs(U1 - U2) < 1e-10 * abs(U1) and np.max(np.abs(gU1 - gU2)) < 1e-9 * np.max(np.abs(gU1))
    m1, m2 = hmc.fisher_inv_mass(g1, th), hmc.fisher_inv_mass(g2, th)
    assert np.max(np.abs(m1 - m2) / m1) < 1e-9
