"""Pins of the oracle shear posterior: the shear map and its Jacobian, prior
normalisers against quadrature, the interim = true special case, mirror
symmetry, the change-of-variables density of lensed ellipticities, the
closed-form gradient against differences, and end-to-end shear recovery from
exact ellipticities (no GPU)."""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import shear

G = complex(0.03, -0.02)


def test_shear_map_roundtrip():
    rng = np.random.default_rng(0)
    e = rng.uniform(-0.6, 0.6, 200) + 1j * rng.uniform(-0.6, 0.6, 200)
    e = e[np.abs(e) < 0.95]
    assert np.max(np.abs(shear.shear_inverse(shear.shear_forward(e, G), G) - e)) < 1e-14
    assert np.max(np.abs(shear.shear_forward(e, 0.0) - e)) == 0.0


def test_jacobian_closed_form_against_differences():
    rng = np.random.default_rng(1)
    for _ in range(20):
        ep = complex(*rng.uniform(-0.6, 0.6, 2))
        h = 1e-6
        f = lambda z: shear.shear_inverse(z, G)
        d1 = (f(ep + h) - f(ep - h)) / (2 * h)            # d eps / d e1'
        d2 = (f(ep + 1j * h) - f(ep - 1j * h)) / (2 * h)  # d eps / d e2'
        det = d1.real * d2.imag - d1.imag * d2.real
        assert abs(math.log(abs(det)) - shear.log_jacobian(ep, G)) < 1e-9


@pytest.mark.parametrize("sig", [0.05, 0.2, 0.3, 0.7])
def test_ellipticity_normalisers_by_quadrature(sig):
    ba, _ = integrate.quad(lambda r: 2 * math.pi * r * (1 - r * r) ** 2 *
                           math.exp(-r * r / (2 * sig * sig)), 0.0, 1.0, epsabs=1e-14, epsrel=1e-13)
    assert abs(ba / shear.z_ba14(sig) - 1) < 1e-10
    tg, _ = integrate.quad(lambda r: 2 * math.pi * r * math.exp(-r * r / (2 * sig * sig)),
                           0.0, 0.7, epsabs=1e-14, epsrel=1e-13)
    assert abs(tg / shear.z_trunc_gauss(sig, 0.7) - 1) < 1e-10
    for kind in (shear.E_KIND_BA14, shear.E_KIND_TRUNC_GAUSS):
        h = 1e-6
        zf = shear.z_ba14 if kind == 0 else (lambda s: shear.z_trunc_gauss(s, 0.7))
        fd = (math.log(zf(sig + h)) - math.log(zf(sig - h))) / (2 * h)
        assert abs(fd - shear.dlogZ_dsig(sig, kind, 0.7)) < 1e-6 * max(1, abs(fd))


def _samples(n_gal, K, seed):
    rng = np.random.default_rng(seed)
    e1 = rng.normal(0, 0.25, (n_gal, K))
    e2 = rng.normal(0, 0.25, (n_gal, K))
    r = np.hypot(e1, e2)
    e1 = np.where(r < 0.9, e1, e1 * 0.5)
    e2 = np.where(r < 0.9, e2, e2 * 0.5)
    ls = rng.normal(math.log10(0.6), 0.13, (n_gal, K))
    lf = rng.normal(3.0, 0.2, (n_gal, K))
    return e1, e2, ls, lf


def test_interim_equals_true_gives_unit_weights():
    e1, e2, ls, lf = _samples(5, 50, 2)
    tp = shear.TruePrior(e_kind=shear.E_KIND_BA14, size_term=False)
    ip = shear.Interim()
    for n in range(5):
        lw = shear.log_weights(e1[n], e2[n], ls[n], lf[n], 0j, (0.0, 0.3, 0.3), tp, ip)
        assert np.max(np.abs(lw)) < 1e-13
        assert abs(shear.galaxy_loglike(e1[n], e2[n], ls[n], lf[n], 0j, (0.0, 0.3, 0.3), tp, ip)) < 1e-13


def test_mirror_symmetry():
    e1, e2, ls, lf = _samples(3, 40, 3)
    tp, ip = shear.TruePrior(), shear.Interim()
    a = shear.log_posterior((e1, e2, ls, lf), G, (-0.5, 0.3, 0.2), tp, ip)
    b = shear.log_posterior((-e1, -e2, ls, lf), -G, (-0.5, 0.3, 0.2), tp, ip)
    assert abs(a - b) < 1e-10 * abs(a)


def test_lensed_density_is_change_of_variables():
    # draw intrinsic ellipticities from the truncated Gaussian, lens them, and
    # compare the histogram of e' with p_e(h_g^-1(e')) |d eps/d eps'|
    rng = np.random.default_rng(4)
    g = complex(0.2, 0.1)          # large shear so the test has power
    sig, emax = 0.25, 0.7
    n = 4_000_000
    e = rng.normal(0, sig, n) + 1j * rng.normal(0, sig, n)
    e = e[np.abs(e) < emax]
    ep = shear.shear_forward(e, g)
    H, xe, ye = np.histogram2d(ep.real, ep.imag, bins=30, range=[[-0.6, 0.6], [-0.6, 0.6]])
    xc, yc = 0.5 * (xe[1:] + xe[:-1]), 0.5 * (ye[1:] + ye[:-1])
    X, Y = np.meshgrid(xc, yc, indexing="ij")
    Z = X + 1j * Y
    dens = np.exp(shear.log_pe(np.abs(shear.shear_inverse(Z, g)) ** 2, sig, 1, emax)
                  + shear.log_jacobian(Z, g))
    expect = dens * e.shape[0] * (xe[1] - xe[0]) * (ye[1] - ye[0])
    m = expect > 400
    chi = (H[m] - expect[m]) / np.sqrt(expect[m])
    assert np.mean(chi ** 2) < 1.6
    assert abs(np.mean(chi)) < 0.2


@pytest.mark.parametrize("kind", [shear.E_KIND_BA14, shear.E_KIND_TRUNC_GAUSS])
def test_gradient_against_differences(kind):
    e1, e2, ls, lf = _samples(4, 60, 5)
    tp = shear.TruePrior(e_kind=kind, e_max=0.95, mu_lnf=math.log(1000.0), sig_lnf=0.5)
    ip = shear.Interim()
    S = (e1, e2, ls, lf)
    x0 = np.array([G.real, G.imag, math.log(0.6), 0.3, 0.22])

    def f(x):
        return shear.log_posterior(S, complex(x[0], x[1]), tuple(x[2:]), tp, ip)

    lp, gr = shear.log_posterior_grad(S, complex(x0[0], x0[1]), tuple(x0[2:]), tp, ip)
    assert abs(lp - f(x0)) < 1e-12 * abs(lp)
    for j in range(5):
        h = 1e-4 * max(1.0, abs(x0[j]))
        e = np.zeros(5)
        e[j] = h
        fd = (8 * (f(x0 + e) - f(x0 - e)) - (f(x0 + 2 * e) - f(x0 - 2 * e))) / (12 * h)
        assert abs(fd - gr[j]) < 1e-6 * max(1.0, abs(gr[j])), (j, fd, gr[j])


def test_exact_ellipticities_recover_shear_on_grid():
    # K = 1 exact lensed ellipticities of 4000 galaxies: posterior must contain g
    rng = np.random.default_rng(6)
    n, sig, emax = 4000, 0.2, 0.7
    e = rng.normal(0, sig, 3 * n) + 1j * rng.normal(0, sig, 3 * n)
    e = e[np.abs(e) < emax][:n]
    g = complex(0.02, 0.0)
    ep = shear.shear_forward(e, g)
    ls = np.full((n, 1), math.log10(0.6))
    S = (ep.real[:, None], ep.imag[:, None], ls, ls)
    tp = shear.TruePrior(e_kind=1, e_max=emax)
    ip = shear.Interim()
    g1s = np.linspace(-0.02, 0.06, 33)
    g2s = np.linspace(-0.04, 0.04, 33)
    lp, m1, m2 = shear.grid_posterior(S, g1s, g2s, (math.log(0.6), 0.3, sig), tp, ip)
    w = np.exp(lp - lp.max())
    G1, G2 = np.meshgrid(g1s, g2s)
    s1 = math.sqrt(np.sum(w * (G1 - m1) ** 2) / np.sum(w))
    # exact intrinsic shapes: the posterior centre is g plus the shape-noise mean
    assert abs(m1 - 0.02) < 4 * s1 and abs(m2) < 4 * s1
    assert 0.001 < s1 < 0.01


def test_shear_level_hmc_against_importance_sampling():
    """Shear-level HMC (the per-galaxy sampler on the five population
    parameters) against an estimate built without it: self-normalised
    importance sampling of the posterior from a widened Gaussian around the
    mode (quasi-Newton optimum, finite-difference Hessian).  Chain means and
    standard deviations agree within their Monte-Carlo errors."""
    from scipy.optimize import minimize
    from oracle import diagnostics, hmc
    from tests import synth
    S = [a.astype(np.float64) for a in synth.interim_population(40, 64, 11)]
    tp = shear.TruePrior(e_kind=shear.E_KIND_TRUNC_GAUSS, e_max=0.95)
    ip = shear.Interim()
    pot = shear.hyper_potential(S, tp, ip)
    x0 = np.array([0.0, 0.0, math.log(0.6), 0.3, 0.25])
    res = minimize(lambda x: pot(x)[0], x0, jac=lambda x: pot(x)[1], method="L-BFGS-B",
                   bounds=[(-0.5, 0.5), (-0.5, 0.5), (-2.0, 1.0), (0.05, 1.0), (0.05, 0.9)],
                   options=dict(gtol=1e-9, ftol=1e-14))
    xm = res.x
    H = np.zeros((5, 5))
    for j in range(5):
        e = np.zeros(5)
        e[j] = 1e-5
        H[j] = (pot(xm + e)[1] - pot(xm - e)[1]) / 2e-5
    cov = np.linalg.inv(0.5 * (H + H.T))
    sd = np.sqrt(np.diag(cov))
    # importance sampling from N(xm, 1.5^2 cov)
    rng = np.random.default_rng(12)
    n_is = 3000
    Lc = np.linalg.cholesky(2.25 * cov)
    z = rng.normal(size=(n_is, 5))
    xs = xm + z @ Lc.T
    lq = -0.5 * np.sum(z * z, axis=1)
    lp = np.array([shear.log_posterior(S, complex(x[0], x[1]), tuple(x[2:]), tp, ip) for x in xs])
    lw = lp - lq
    w = np.exp(lw - lw.max())
    w /= w.sum()
    n_is_eff = 1.0 / np.sum(w * w)
    assert n_is_eff > 500
    m_is = w @ xs
    s_is = np.sqrt(w @ (xs - m_is) ** 2)
    out = hmc.run_chain(pot, xm, seed=99, uid=3, L=6, n_warmup=80, n_samples=240,
                        eps0=0.5, adapt=True, inv_mass=sd ** 2, jitter=0.1)
    x = out["samples"]
    assert out["accept_rate"] > 0.5
    for j in range(5):
        n_eff = max(diagnostics.ess(x[None, :, j]), 20.0)
        se = math.sqrt(s_is[j] ** 2 / n_eff + s_is[j] ** 2 / n_is_eff)
        assert abs(x[:, j].mean() - m_is[j]) < 4 * se, (j, x[:, j].mean(), m_is[j], se)
        assert 0.7 < x[:, j].std() / s_is[j] < 1.4, (j, x[:, j].std(), s_is[j])


# The hyper-priors of Section 3.4 as the paper prints them, in log10 units of
# size (its Section 2 population is lognormal in log10 s): mu_s ~ U(-2, 2),
# sigma_s ~ U(0, 0.5); sigma_e ~ U(1e-4, 1); g uniform on the unit disk.  The
# oracle takes alpha in natural-log units (reading R14), so its boxes are
# these times ln 10.  Each edge is probed just inside (finite) and just outside
# (-inf); the log10-unit points inside the paper's boxes but outside the
# unconverted ones catch a box left in log10 units.
PAPER_MU10 = (-2.0, 2.0)
PAPER_SIG10 = (0.0, 0.5)
PAPER_SIGE = (1e-4, 1.0)


def _edge_points(rel=1e-9):
    """(g, alpha, inside?) around every edge of the paper's boxes."""
    base_g, base = complex(0.01, -0.02), (math.log(0.6), 0.3, 0.25)
    out = []
    for mu10 in PAPER_MU10:
        for s, ins in ((-1.0, True), (1.0, False)):
            mu = mu10 * (1.0 + s * rel) * shear.LN10
            out.append((base_g, (mu, base[1], base[2]), ins))
    hi = PAPER_SIG10[1]
    out += [(base_g, (base[0], hi * (1.0 - rel) * shear.LN10, base[2]), True),
            (base_g, (base[0], hi * (1.0 + rel) * shear.LN10, base[2]), False),
            (base_g, (base[0], 0.0, base[2]), False),
            (base_g, (base[0], -1e-3, base[2]), False)]
    lo, hi = PAPER_SIGE
    out += [(base_g, (base[0], base[1], lo * (1.0 + 1e3 * rel)), True),
            (base_g, (base[0], base[1], lo), False),
            (base_g, (base[0], base[1], lo * (1.0 - 1e3 * rel)), False),
            (base_g, (base[0], base[1], hi * (1.0 - rel)), True),
            (base_g, (base[0], base[1], hi), False)]
    for phi in (0.0, 1.0, 2.5):
        u = complex(math.cos(phi), math.sin(phi))
        out += [((1.0 - 1e3 * rel) * u, base, True), (u, base, False), ((1.0 + rel) * u, base, False)]
    # inside the paper's log10 boxes, outside the same numbers read as ln-unit boxes
    out += [(base_g, (1.3 * shear.LN10, base[1], base[2]), True),
            (base_g, (-1.3 * shear.LN10, base[1], base[2]), True),
            (base_g, (base[0], 0.4 * shear.LN10, base[2]), True)]
    return out


@pytest.mark.parametrize("kind", [shear.E_KIND_BA14, shear.E_KIND_TRUNC_GAUSS])
def test_hyper_prior_box_edges(kind):
    e1, e2, ls, lf = _samples(3, 40, 13)
    # near |g| = 1 the inverse shear maps every sample close to the unit circle,
    # so the truncated Gaussian is taken with e_max = 1 (support the unit disk)
    tp = shear.TruePrior(e_kind=kind, e_max=1.0)
    ip = shear.Interim()
    n_checked = 0
    for g, alpha, inside in _edge_points():
        assert shear.in_hyper_support(g, alpha) == inside, (g, alpha)
        lp = shear.log_posterior((e1, e2, ls, lf), g, alpha, tp, ip)
        if inside:
            assert np.isfinite(lp), (g, alpha, lp)
        else:
            assert lp == -math.inf, (g, alpha, lp)
        n_checked += 1
    assert n_checked == 25
